"""Independent brute-force constructions used to pin the oracle.

Nothing here calls the oracle: dense matrices are assembled element by element
with explicit loops, occupations use scipy's logistic and root finder.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq
from scipy.special import expit


def dense_hamiltonian(V: np.ndarray, n, L) -> np.ndarray:
    """Dense M x M matrix of -1/2 Lap_h + diag(V) on a periodic grid, assembled point
    by point (x fastest); every n_d >= 3 so that the two neighbours differ."""
    nx, ny, nz = n
    hx, hy, hz = (L[0] / nx, L[1] / ny, L[2] / nz)
    M = nx * ny * nz
    H = np.zeros((M, M))

    def idx(x, y, z):
        return (z % nz) * ny * nx + (y % ny) * nx + (x % nx)

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                p = idx(x, y, z)
                H[p, p] += 1.0 / hx ** 2 + 1.0 / hy ** 2 + 1.0 / hz ** 2 + V[z, y, x]
                for q, hd in ((idx(x + 1, y, z), hx), (idx(x - 1, y, z), hx),
                              (idx(x, y + 1, z), hy), (idx(x, y - 1, z), hy),
                              (idx(x, y, z + 1), hz), (idx(x, y, z - 1), hz)):
                    H[p, q] += -0.5 / hd ** 2
    return H


def occupations(eps, mu, kT):
    return expit(-(np.asarray(eps) - mu) / kT)


def fermi_level(eps, n_electrons, kT, s):
    eps = np.asarray(eps).ravel()
    g = lambda mu: s * np.sum(occupations(eps, mu, kT)) - n_electrons  # noqa: E731
    lo = eps.min() - 60 * kT
    hi = eps.max() + 60 * kT
    return brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)


def projected(Psi2d: np.ndarray, dV: np.ndarray) -> np.ndarray:
    """H'_ij = sum_p Psi_ip dV_p Psi_jp written as an explicit index contraction."""
    return np.einsum("ip,p,jp->ij", Psi2d, dV.ravel(), Psi2d, optimize=False)


def subspace_density(Psi2d, D, Hp, lam, n_electrons, kT, s, dv):
    """(s/dv) diag(Psi f(D + lam H', mu(lam)) Psi^T) by diagonalising D + lam H' and
    re-solving the electron count: no divided differences anywhere."""
    w, W = np.linalg.eigh(np.diag(D) + lam * Hp)
    mu = fermi_level(w, n_electrons, kT, s)
    f = occupations(w, mu, kT)
    B = Psi2d.T @ W                                  # M x N
    return (s / dv) * np.sum(B * B * f[None, :], axis=1)


def richardson_derivative(fun, h):
    """Central difference with one Richardson step: (4 D(h/2) - D(h)) / 3."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


def full_space_density(V, n, L, n_electrons, kT, s):
    """rho(V) = (s/dv) sum_i f_i |q_i|^2 from a dense diagonalisation of all M states."""
    H = dense_hamiltonian(V, n, L)
    w, Q = np.linalg.eigh(H)
    mu = fermi_level(w, n_electrons, kT, s)
    f = occupations(w, mu, kT)
    dv = (L[0] / n[0]) * (L[1] / n[1]) * (L[2] / n[2])
    return (s / dv) * np.sum(Q * Q * f[None, :], axis=1)


def fd_scalar(e1, e2, mu, kT):
    """Divided difference of the Fermi function from its definition: the plain
    quotient when the energies differ by more than 1e-6, else the derivative at the
    midpoint (error O(d^2 / kT^3), below 1e-12 here)."""
    if abs(e1 - e2) > 1e-6:
        return (occupations(e1, mu, kT) - occupations(e2, mu, kT)) / (e1 - e2)
    m = 0.5 * (e1 + e2)
    f = occupations(m, mu, kT)
    return -f * (1 - f) / kT


def dense_bloch_hamiltonian(V: np.ndarray, n, L, kvec) -> np.ndarray:
    """Dense complex M x M matrix of the Bloch Hamiltonian for the cell-periodic
    part, assembled point by point: the hop from point p to its neighbour at +h_d
    carries exp(i k_d h_d), the hop to -h_d exp(-i k_d h_d)."""
    nx, ny, nz = n
    h = (L[0] / nx, L[1] / ny, L[2] / nz)
    M = nx * ny * nz
    H = np.zeros((M, M), dtype=np.complex128)

    def idx(x, y, z):
        return (z % nz) * ny * nx + (y % ny) * nx + (x % nx)

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                p = idx(x, y, z)
                H[p, p] += sum(1.0 / hd ** 2 for hd in h) + V[z, y, x]
                for d, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    ph = np.exp(1j * kvec[d] * h[d])
                    H[p, idx(x + dx, y + dy, z + dz)] += -0.5 * ph / h[d] ** 2
                    H[p, idx(x - dx, y - dy, z - dz)] += -0.5 * np.conj(ph) / h[d] ** 2
    return H
