"""Pins of the oracle: each function returns an error measure that is small for a
correct oracle.  ``test_oracle_*.py`` asserts they are small; the mutation tests
plant mistakes in the oracle and assert that at least one pin notices.

Each pin compares the oracle with something other than itself: a closed form,
a dense diagonalisation, a finite difference, 50-digit decimal arithmetic or an
invariant of the mathematics.
"""
from __future__ import annotations

import decimal

import numpy as np
from numpy.polynomial import chebyshev as npcheb

import oracle as O
from tests import bruteforce as bf


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def small_wells(n, L, seed, nwells=3, depth=(1.0, 2.0)):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (nwells, 3)) * np.asarray(L)
    d = rng.uniform(*depth, nwells)
    w = rng.uniform(0.6, 1.0, nwells)
    from inputs import gaussian_wells
    return gaussian_wells(n, L, d, w, pos)


# ------------------------------------------------------------------ stencil
def pin_plane_wave():
    """cos(k.x) is an eigenvector of -1/2 Lap_h + V0 with eigenvalue
    sum_d (1 - cos(2 pi k_d / n_d)) / h_d^2 + V0."""
    n, L = (6, 5, 7), (3.0, 2.5, 3.3)
    g = O.Grid(n, L)
    V0 = 0.37
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    err = 0.0
    for k in [(1, 0, 0), (2, 1, 3), (0, 2, 1), (3, 2, 0)]:
        th = [2 * np.pi * k[d] / n[d] for d in range(3)]
        Y = np.cos(th[0] * x + th[1] * y + th[2] * z)[None]
        lam = sum((1 - np.cos(th[d])) / g.h[d] ** 2 for d in range(3)) + V0
        HY = O.hamiltonian_apply(Y, np.full(g.shape, V0), g)
        err = max(err, _rel(HY, lam * Y))
    return err


def pin_dense_stencil():
    n, L = (4, 3, 5), (2.0, 1.7, 2.6)
    g = O.Grid(n, L)
    rng = np.random.default_rng(1)
    V = rng.standard_normal(g.shape)
    Y = rng.standard_normal((3,) + g.shape)
    H = bf.dense_hamiltonian(V, n, L)
    ref = (H @ Y.reshape(3, -1).T).T.reshape(Y.shape)
    return _rel(O.hamiltonian_apply(Y, V, g), ref)


# ------------------------------------------------------------------ filter
def pin_filter_polynomial(degree=9):
    """T_c(Hbar) X / T_c(ybar0) from the dense eigendecomposition, with T_c evaluated
    by numpy's Chebyshev series routine."""
    n, L = (4, 4, 4), (3.0, 3.0, 3.0)
    g = O.Grid(n, L)
    V = small_wells(n, L, 2)
    H = bf.dense_hamiltonian(V, n, L)
    lam, Q = np.linalg.eigh(H)
    a0, a, b = lam[0] - 0.05, lam[10], lam[-1] + 0.02
    e, c0 = (b - a) / 2, (b + a) / 2
    coef = np.zeros(degree + 1)
    coef[-1] = 1.0
    scale = npcheb.chebval((lam - c0) / e, coef) / npcheb.chebval((a0 - c0) / e, coef)
    X = np.random.default_rng(3).standard_normal((5,) + g.shape)
    Xc = X.reshape(5, -1).T
    ref = (Q @ (scale[:, None] * (Q.T @ Xc))).T.reshape(X.shape)
    return _rel(O.chebyshev_filter(X, V, g, degree, a, b, a0), ref)


def pin_filter_scalar_identity(degree=7):
    """On a plane wave with eigenvalue lam inside [a, b], the filter multiplies by
    cos(c arccos(lbar)) / ((-1)^c cosh(c arccosh(-ybar0))), closed form."""
    n, L = (5, 6, 4), (2.0, 2.4, 1.6)
    g = O.Grid(n, L)
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    k = (2, 1, 1)
    th = [2 * np.pi * k[d] / n[d] for d in range(3)]
    Y = np.cos(th[0] * x + th[1] * y + th[2] * z)[None]
    lam = sum((1 - np.cos(th[d])) / g.h[d] ** 2 for d in range(3))
    b = sum(2.0 / hd ** 2 for hd in g.h)            # top of the spectrum of -1/2 Lap_h
    a, a0 = lam - 0.7, -0.4
    e, c0 = (b - a) / 2, (b + a) / 2
    lbar, ybar0 = (lam - c0) / e, (a0 - c0) / e
    factor = np.cos(degree * np.arccos(lbar)) / ((-1) ** degree * np.cosh(degree * np.arccosh(-ybar0)))
    out = O.chebyshev_filter(Y, np.zeros(g.shape), g, degree, a, b, a0)
    return _rel(out, factor * Y)


def chfsi_passes(V, g, N, passes, degree, seed=4):
    X = np.random.default_rng(seed).standard_normal((N,) + g.shape)
    b = sum(2.0 / hd ** 2 for hd in g.h) + float(V.max())
    a0 = float(V.min())
    a = a0 + 0.3 * (b - a0)
    eps = None
    for _ in range(passes):
        Y = O.chebyshev_filter(X, V, g, degree, a, b, a0)
        eps, X = O.rayleigh_ritz(Y, V, g)
        a = float(eps[-1])
        a0 = float(eps[0]) - 0.5
    return eps, X


def pin_chfsi_exact_subspace():
    """Repeated filter + Rayleigh-Ritz converges to the exact lowest eigenpairs
    (dense diagonalisation): returns (max Ritz error, sin of the largest principal
    angle) over the lowest N - 4 states."""
    n, L = (6, 6, 6), (4.0, 4.0, 4.0)
    g = O.Grid(n, L)
    V = small_wells(n, L, 5, nwells=4)
    lam, Q = np.linalg.eigh(bf.dense_hamiltonian(V, n, L))
    N, keep = 14, 10
    eps, Psi = chfsi_passes(V, g, N, passes=12, degree=12)
    ritz_err = float(np.max(np.abs(eps[:keep] - lam[:keep])))
    P = Psi[:keep].reshape(keep, -1).T
    s = np.linalg.svd(Q[:, :keep].T @ P, compute_uv=False)
    sin_max = float(np.sqrt(max(0.0, 1 - s.min() ** 2)))
    return ritz_err, sin_max


# ------------------------------------------------------------------ Rayleigh-Ritz
def pin_rr_exact_eigenvectors():
    n, L = (4, 4, 3), (3.0, 3.0, 2.4)
    g = O.Grid(n, L)
    V = small_wells(n, L, 6)
    lam, Q = np.linalg.eigh(bf.dense_hamiltonian(V, n, L))
    idx = [0, 1, 2, 5, 7, 11]
    rng = np.random.default_rng(7)
    mix = np.linalg.qr(rng.standard_normal((len(idx), len(idx))))[0]
    Y = (Q[:, idx] @ mix * rng.uniform(0.5, 3, len(idx))[None, :]).T.reshape((len(idx),) + g.shape)
    eps, _ = O.rayleigh_ritz(Y, V, g)
    return float(np.max(np.abs(eps - lam[idx])))


def pin_rr_generalized():
    """Ritz values of span(Y) equal the generalized eigenvalues of (Y^T H Y, Y^T Y)
    (scipy), the Ritz vectors are orthonormal and diagonalise H."""
    from scipy.linalg import eigh as geigh
    n, L = (5, 4, 4), (3.0, 2.4, 2.4)
    g = O.Grid(n, L)
    V = small_wells(n, L, 8)
    H = bf.dense_hamiltonian(V, n, L)
    Y = np.random.default_rng(9).standard_normal((9,) + g.shape)
    Yc = Y.reshape(9, -1).T
    ref = geigh(Yc.T @ H @ Yc, Yc.T @ Yc, eigvals_only=True)
    eps, Psi = O.rayleigh_ritz(Y, V, g)
    P = Psi.reshape(9, -1).T
    e1 = float(np.max(np.abs(eps - ref)))
    e2 = float(np.max(np.abs(P.T @ P - np.eye(9))))
    e3 = float(np.max(np.abs(P.T @ H @ P - np.diag(eps))))
    return max(e1, e2, e3)


# ------------------------------------------------------------------ occupations
def pin_fermi_level():
    rng = np.random.default_rng(10)
    errs = []
    for nspin, kT in ((1, 0.01), (2, 0.005), (1, 0.1)):
        eps = np.sort(rng.uniform(-2, 1, (nspin, 40)), axis=1)
        s = O.spin_factor(nspin)
        ne = 0.39 * s * 40 * nspin
        mu, conv = O.fermi_level(eps, ne, kT, nspin)
        count = s * np.sum(bf.occupations(eps, mu, kT))
        errs.append(abs(count - ne) / ne)
        errs.append(abs(mu - bf.fermi_level(eps, ne, kT, s)))
        if not conv:
            errs.append(1.0)
    return max(errs)


def pin_fermi_gap():
    """With a gap of 1 Ha between the 4th and 5th levels, 8 electrons and a small kT,
    mu sits inside the gap."""
    eps = np.array([-3.0, -2.5, -2.2, -2.0, -1.0, -0.7, -0.2, 0.3])
    mu, _ = O.fermi_level(eps, 8.0, 0.005, 1)
    return 0.0 if (-2.0 < mu < -1.0) else 1.0


def _dec_fermi(e, mu, kT):
    return decimal.Decimal(1) / (decimal.Decimal(1) + ((decimal.Decimal(e) - decimal.Decimal(mu)) / decimal.Decimal(kT)).exp())


def pin_divided_differences_decimal():
    """F against 50-digit decimal arithmetic of (f_i - f_j)/(e_i - e_j) and of
    -f(1-f)/kT on the diagonal, including near-degenerate pairs."""
    decimal.getcontext().prec = 50
    rng = np.random.default_rng(11)
    mu, kT = 0.13, 0.01
    base = rng.uniform(-0.1, 0.35, 12)
    eps = np.concatenate([base, base[:4] + np.array([1e-11, 3e-9, 2e-7, 5e-5]), [mu, mu + 1e-12]])
    F = O.divided_differences(eps, mu, kT)
    err = 0.0
    for i in range(len(eps)):
        for j in range(len(eps)):
            if eps[i] == eps[j]:
                fi = _dec_fermi(eps[i], mu, kT)
                ref = -fi * (1 - fi) / decimal.Decimal(kT)
            else:
                ref = (_dec_fermi(eps[i], mu, kT) - _dec_fermi(eps[j], mu, kT)) / \
                      (decimal.Decimal(eps[i]) - decimal.Decimal(eps[j]))
            ref = float(ref)
            scale = max(abs(ref), 1e-300)
            if abs(ref) > 1e-250:
                err = max(err, abs(F[i, j] - ref) / scale)
    return err


def pin_divided_differences_naive():
    rng = np.random.default_rng(12)
    eps = np.sort(rng.uniform(-1, 1, 30))
    mu, kT = 0.05, 0.02
    F = O.divided_differences(eps, mu, kT)
    scale = float(np.abs(F).max())
    err = 0.0
    for i in range(30):
        for j in range(30):
            # the plain quotient cancels when both occupations are near 1, so the
            # comparison is in units of the largest entry
            ref = bf.fd_scalar(eps[i], eps[j], mu, kT)
            err = max(err, abs(F[i, j] - ref) / scale)
    sym = float(np.max(np.abs(F - F.T)))
    nonpos = float(max(F.max(), 0.0))
    return max(err, sym, nonpos)


# ------------------------------------------------------------------ response
def _rr_system(n, L, N, seed, passes=4, degree=10):
    g = O.Grid(n, L)
    V = small_wells(n, L, seed, nwells=4)
    eps, Psi = chfsi_passes(V, g, N, passes=passes, degree=degree, seed=seed)
    return g, V, eps, Psi


def pin_response_subspace_fd(nspin=1):
    """delta rho from the oracle against a Richardson central difference in lam of the
    subspace density (s/dv) diag(Psi f(eigh(D + lam H'), mu(lam)) Psi^T)."""
    n, L = (5, 5, 4), (3.2, 3.2, 2.6)
    N = 16
    g, V, eps, Psi = _rr_system(n, L, N, seed=13)
    rng = np.random.default_rng(14)
    kT = 0.03
    s = O.spin_factor(nspin)
    ne = 0.7 * N * (2.0 if nspin == 1 else 2.0)
    if nspin == 2:
        eps2 = np.stack([eps, eps + rng.uniform(-0.02, 0.02, N)])
        Psi2 = np.stack([Psi, Psi])
    else:
        eps2, Psi2 = eps[None], Psi[None]
    dV = rng.standard_normal((1, nspin) + g.shape)
    drho, mu, dmu = O.density_response(Psi2, eps2, g, ne, kT, dV, nspin)

    P = [Psi2[c].reshape(N, -1) for c in range(nspin)]
    Hp = [bf.projected(P[c], dV[0, c]) for c in range(nspin)]

    def rho_all(lam):
        # common mu(lam) across channels: diagonalise each channel, solve one count
        ws, Ws = [], []
        for c in range(nspin):
            w, W = np.linalg.eigh(np.diag(eps2[c]) + lam * Hp[c])
            ws.append(w)
            Ws.append(W)
        mu_l = bf.fermi_level(np.concatenate(ws), ne, kT, s)
        out = []
        for c in range(nspin):
            f = bf.occupations(ws[c], mu_l, kT)
            B = P[c].T @ Ws[c]
            out.append((s / g.dv) * np.sum(B * B * f[None, :], axis=1))
        return np.concatenate(out)

    ref = bf.richardson_derivative(rho_all, 2e-4)
    return _rel(drho[0].reshape(-1), ref)


def pin_response_full_space():
    """With N = M (all states) the subspace response is the exact full response:
    Richardson central difference of the dense-diagonalisation density rho(V + lam dV)."""
    n, L = (4, 4, 3), (3.0, 3.0, 2.2)
    g = O.Grid(n, L)
    V = small_wells(n, L, 15)
    kT, ne, s = 0.05, 10.0, 2.0
    lam_all, Q = np.linalg.eigh(bf.dense_hamiltonian(V, n, L))
    Psi = Q.T.reshape((g.M,) + g.shape)
    dV = np.random.default_rng(16).standard_normal(g.shape)
    drho, _, _ = O.density_response(Psi[None], lam_all[None], g, ne, kT, dV[None, None], 1)
    ref = bf.richardson_derivative(lambda t: bf.full_space_density(V + t * dV, n, L, ne, kT, s), 1e-3)
    return _rel(drho.reshape(-1), ref)


def invariants():
    """Returns a dict of invariant violations: integral of delta rho, symmetry and
    sign of chi0, constant perturbation, linearity, degenerate-rotation invariance."""
    n, L = (5, 4, 4), (3.2, 2.6, 2.6)
    N = 14
    g, V, eps, Psi = _rr_system(n, L, N, seed=17)
    kT, ne = 0.02, 14.0
    rng = np.random.default_rng(18)
    dV = rng.standard_normal((3, 1) + g.shape)
    drho, mu, dmu = O.density_response(Psi[None], eps[None], g, ne, kT, dV, 1)
    out = {}
    norm = np.abs(drho).max()
    out["integral"] = float(np.max(np.abs(g.dv * drho.reshape(3, -1).sum(axis=1)))) / (g.dv * norm * g.M)
    ip = lambda a, b: g.dv * float(np.sum(a * b))  # noqa: E731
    c01, c10 = ip(dV[0], drho[1]), ip(dV[1], drho[0])
    out["symmetry"] = abs(c01 - c10) / max(abs(c01), 1e-300)
    quad = [ip(dV[k], drho[k]) for k in range(3)]
    out["nsd"] = max(0.0, max(quad))
    const = np.full((1, 1) + g.shape, 0.7)
    dc, _, _ = O.density_response(Psi[None], eps[None], g, ne, kT, const, 1)
    out["constant"] = float(np.abs(dc).max()) / norm
    comb = (2.0 * dV[0] - 0.5 * dV[2])[None]
    dl, _, _ = O.density_response(Psi[None], eps[None], g, ne, kT, comb, 1)
    out["linearity"] = _rel(dl[0], 2.0 * drho[0] - 0.5 * drho[2])
    # rotation inside an exactly degenerate pair leaves delta rho unchanged
    eps_d = eps.copy()
    eps_d[6] = eps_d[5]
    d1, _, _ = O.density_response(Psi[None], eps_d[None], g, ne, kT, dV[:1], 1)
    Pr = Psi.copy()
    c, s_ = np.cos(0.7), np.sin(0.7)
    Pr[5], Pr[6] = c * Psi[5] + s_ * Psi[6], -s_ * Psi[5] + c * Psi[6]
    d2, _, _ = O.density_response(Pr[None], eps_d[None], g, ne, kT, dV[:1], 1)
    out["degenerate_rotation"] = _rel(d2, d1)
    return out


def pin_lindhard():
    """V = 0 with all M states: dV = cos(q.x) gives delta rho = chi0(q) cos(q.x) with the
    discrete Lindhard sum chi0(q) = (s/Omega) sum_k F(e_k, e_{k+q}) over grid
    wavevectors, e_k = sum_d (1 - cos(2 pi k_d/n_d))/h_d^2 in closed form."""
    n, L = (4, 4, 4), (2.8, 2.8, 2.8)
    g = O.Grid(n, L)
    kT, ne, s = 0.15, 12.0, 2.0
    lam, Q = np.linalg.eigh(bf.dense_hamiltonian(np.zeros(g.shape), n, L))
    Psi = Q.T.reshape((g.M,) + g.shape)
    ks = [(kx, ky, kz) for kz in range(n[2]) for ky in range(n[1]) for kx in range(n[0])]
    ek = {k: sum((1 - np.cos(2 * np.pi * k[d] / n[d])) / g.h[d] ** 2 for d in range(3)) for k in ks}
    mu = bf.fermi_level(np.array(list(ek.values())), ne, kT, s)
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    err = 0.0
    for q in [(1, 0, 0), (1, 1, 0), (2, 1, 3), (2, 2, 2)]:
        dV = np.cos(2 * np.pi * (q[0] * x / n[0] + q[1] * y / n[1] + q[2] * z / n[2]))
        drho, mu_o, _ = O.density_response(Psi[None], lam[None], g, ne, kT, dV[None, None], 1)
        chi = 0.0
        for k in ks:
            kq = tuple((k[d] + q[d]) % n[d] for d in range(3))
            chi += bf.fd_scalar(ek[k], ek[kq], mu, kT)
        chi *= s / (g.M * g.dv)
        err = max(err, _rel(drho[0, 0], chi * dV), abs(mu_o - mu))
    return err


# ------------------------------------------------------------------ Hartree kernel
def pin_hartree_plane_wave():
    n, L = (6, 5, 8), (3.0, 2.5, 4.1)
    g = O.Grid(n, L)
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    err = 0.0
    for q in [(1, 0, 0), (1, 2, 3), (3, 1, 4), (0, 0, 1)]:
        th = [2 * np.pi * q[d] / n[d] for d in range(3)]
        u = np.cos(th[0] * x + th[1] * y + th[2] * z + 0.3)
        lam = sum((2 - 2 * np.cos(th[d])) / g.h[d] ** 2 for d in range(3))
        err = max(err, _rel(O.hartree_kernel(u, g), (4 * np.pi / lam) * u))
    return err


def pin_hartree_poisson():
    """-Lap_h (K u) = 4 pi (u - mean u), with the Laplacian taken from the stencil
    (H with V = 0 is -1/2 Lap_h) rather than the Fourier symbol."""
    n, L = (6, 7, 5), (3.0, 3.5, 2.5)
    g = O.Grid(n, L)
    u = np.random.default_rng(19).standard_normal(g.shape)
    vh = O.hartree_kernel(u, g)
    lap = -2.0 * O.hamiltonian_apply(vh[None], np.zeros(g.shape), g)[0]
    return _rel(-lap, 4 * np.pi * (u - u.mean()))


def pin_residual_derivative_spin():
    """Spin pairs: every channel sees the Hartree potential of u_up + u_down, and
    t = delta rho - u."""
    n, L = (4, 4, 4), (3.0, 3.0, 3.0)
    N = 10
    g, V, eps, Psi = _rr_system(n, L, N, seed=20, passes=3, degree=8)
    rng = np.random.default_rng(21)
    u = rng.standard_normal((2, 2) + g.shape)
    eps2 = np.stack([eps, eps + 0.01])
    Psi2 = np.stack([Psi, Psi])
    t, mu, dmu = O.residual_derivative(Psi2, eps2, g, 9.0, 0.02, u, 2)
    dV = np.empty_like(u)
    for k in range(2):
        vh = O.hartree_kernel(u[k, 0] + u[k, 1], g)
        dV[k, 0] = vh
        dV[k, 1] = vh
    drho, _, _ = O.density_response(Psi2, eps2, g, 9.0, 0.02, dV, 2)
    return _rel(t, drho - u)


# ------------------------------------------------------------------ recursion (Eqs. (23)-(24))
def recursion_errors(depths=(4, 6, 8, 10, 12)):
    """Error of the recursive Fermi-operator response against the exact divided
    differences, for growing recursion depth T (fixed mu)."""
    rng = np.random.default_rng(22)
    N = 24
    eps = np.sort(rng.uniform(-0.3, 0.3, N))
    A = rng.standard_normal((N, N))
    Hp = 0.5 * (A + A.T)
    mu, kT = 0.01, 0.02
    exact = O.divided_differences(eps, mu, kT) * Hp
    errs = []
    for T in depths:
        _, xp = O.recursive_fermi_response(eps, mu, kT, Hp, T)
        errs.append(_rel(xp, exact))
    return errs


# ------------------------------------------------------------------ adjoint of the response
def _dec_fermi_derivs(e, mu, kT):
    """f, f' and f'' of the Fermi function in 50-digit decimal."""
    f = _dec_fermi(e, mu, kT)
    a = f * (1 - f)
    k = decimal.Decimal(kT)
    return f, -a / k, a * (1 - 2 * f) / (k * k)


def pin_second_divided_differences_decimal():
    """D_ij = f[e_i, e_i, e_j] against 50-digit decimal (f[e_i,e_j] - f'(e_i))/(e_j - e_i)
    and f''(e_i)/2 at coincidence, for separations from 0 to 5 kT on both sides of
    the Taylor threshold; error in units of f(1-f)/kT^2 at e_i."""
    decimal.getcontext().prec = 50
    mu, kT = 0.13, 0.01
    rng = np.random.default_rng(21)
    base = rng.uniform(mu - 0.06, mu + 0.06, 6)
    offs = np.array([0.0, 1e-9, 1e-6, 1e-4, 9.9e-4, 1.01e-3, 1e-2, 0.1, 1.0, 5.0]) * kT
    eps = np.concatenate([base, base[0] + offs[1:], base[3] - offs[1:]])
    D = O.second_divided_differences(eps, mu, kT)
    err = 0.0
    for i in range(len(eps)):
        fi, f1i, f2i = _dec_fermi_derivs(eps[i], mu, kT)
        scale = float(fi * (1 - fi)) / kT ** 2
        for j in range(len(eps)):
            if eps[i] == eps[j]:
                ref = f2i / 2
            else:
                fj = _dec_fermi(eps[j], mu, kT)
                dij = (fi - fj) / (decimal.Decimal(eps[i]) - decimal.Decimal(eps[j]))
                ref = (dij - f1i) / (decimal.Decimal(eps[j]) - decimal.Decimal(eps[i]))
            err = max(err, abs(D[i, j] - float(ref)) / scale)
    return err


def _vjp_case(nspin, seed=0):
    rng = np.random.default_rng(seed)
    g = O.Grid((5, 4, 3), (2.5, 2.0, 1.5))
    N = 9
    Psi = np.stack([np.linalg.qr(rng.standard_normal((g.M, N)))[0].T.reshape((N,) + g.shape)
                    for _ in range(nspin)])
    eps = np.sort(rng.uniform(-1.0, 0.5, (nspin, N)), axis=1)
    eps[0, 3] = eps[0, 2] + 1e-6           # a near-degenerate pair
    ne = 0.6 * N
    kT = 0.05
    dV = rng.standard_normal((2, nspin) + g.shape)
    G = rng.standard_normal((2, nspin) + g.shape)
    return rng, g, Psi, eps, ne, kT, dV, G


def pin_vjp_fd():
    """<dL/dx, u> against Richardson-extrapolated central differences of
    L = <G, delta rho> along random u, for x = dV, Psi, eps and both spin cases
    (uses only the forward oracle).  Returns the largest relative error."""
    worst = 0.0
    for nspin in (1, 2):
        rng, g, Psi, eps, ne, kT, dV, G = _vjp_case(nspin)
        gdV, gP, ge = O.density_response_vjp(Psi, eps, g, ne, kT, dV, G, nspin)
        base = {"dV": dV, "Psi": Psi, "eps": eps}
        for name, gx in (("dV", gdV), ("Psi", gP), ("eps", ge)):
            u = rng.standard_normal(base[name].shape)

            def L(t):
                a = dict(base)
                a[name] = base[name] + t * u
                d = O.density_response(a["Psi"], a["eps"], g, ne, kT, a["dV"], nspin)[0]
                return float(np.sum(G * d))
            h = 2e-4
            c1 = (L(h) - L(-h)) / (2 * h)
            c2 = (L(h / 2) - L(-h / 2)) / h
            fd = (4 * c2 - c1) / 3
            an = float(np.sum(gx * u))
            worst = max(worst, abs(fd - an) / max(abs(an), 1e-300))
    return worst


def pin_vjp_self_adjoint():
    """The response is a symmetric linear map of dV, so dL/ddV for L = <G, delta rho>
    is the response to G itself."""
    worst = 0.0
    for nspin in (1, 2):
        _, g, Psi, eps, ne, kT, dV, G = _vjp_case(nspin, seed=3)
        gdV, _, _ = O.density_response_vjp(Psi, eps, g, ne, kT, dV, G, nspin)
        ref = O.density_response(Psi, eps, g, ne, kT, G, nspin)[0]
        worst = max(worst, float(np.linalg.norm(gdV - ref) / np.linalg.norm(ref)))
    return worst


# ------------------------------------------------------------------ low-rank step
def _linear_residual(n=(5, 4, 2), L=(2.5, 2.0, 1.0), seed=11, strength=0.6):
    """A linear residual map t = J u with J = -(I + strength A), A a seeded
    nonsymmetric Gaussian matrix scaled by 1/sqrt(M)."""
    g = O.Grid(n, L)
    rng = np.random.default_rng(seed)
    M = g.M
    J = -(np.eye(M) + strength * rng.standard_normal((M, M)) / np.sqrt(M))
    R = rng.standard_normal(g.shape)

    def apply_t(u):
        return (J @ u.ravel()).reshape(u.shape)
    return g, J, R, apply_t


def pin_lowrank_krylov_lstsq(ranks=(1, 2, 3, 4, 5)):
    """For a linear residual map, P^lr_r R is the minimiser of ||J x - R|| over the
    Krylov space span{R, J R, ..., J^{r-1} R} (the GMRES iterate from zero):
    here found by numpy's least squares on the monomial Krylov basis, with no
    Gram-Schmidt and no S.  s_rel is that minimum over ||R||."""
    g, J, R, apply_t = _linear_residual()
    b = R.ravel()
    err = 0.0
    for r in ranks:
        drho, _, _, hist = O.lowrank_preconditioner(R, apply_t, g, 0.0, r)
        K = np.stack([np.linalg.matrix_power(J, k) @ b for k in range(r)], axis=1)
        y = np.linalg.lstsq(J @ K, b, rcond=None)[0]
        x = K @ y
        err = max(err, _rel(drho.ravel(), x),
                  abs(hist[-1] - np.linalg.norm(J @ x - b) / np.linalg.norm(b)))
    return err


def pin_lowrank_full_rank_newton():
    """At full rank (r = M) the low-rank step is the Newton step J^{-1} R and
    s_rel vanishes."""
    g, J, R, apply_t = _linear_residual(n=(3, 2, 2), L=(1.5, 1.0, 1.0), seed=5, strength=0.4)
    drho, _, _, hist = O.lowrank_preconditioner(R, apply_t, g, 0.0, g.M)
    return max(_rel(drho.ravel(), np.linalg.solve(J, R.ravel())), hist[-1])


def pin_lowrank_directions():
    """The directions are orthonormal in the cell integral (Eq. (7)), t_i = J u_i,
    s_rel does not grow with the rank, and the adaptive rank is the first rank
    whose s_rel is below the tolerance (Eq. (10))."""
    g, J, R, apply_t = _linear_residual()
    _, U, T, hist = O.lowrank_preconditioner(R, apply_t, g, 0.0, 8)
    Um = U.reshape(len(U), -1)
    err = np.abs(g.dv * Um @ Um.T - np.eye(len(U))).max()
    err = max(err, max(_rel(T[i].ravel(), J @ Um[i]) for i in range(len(U))))
    err = max(err, float(np.max(np.diff(hist), initial=0.0)) if len(hist) > 1 else 0.0)
    k = 3
    tol = 0.5 * (hist[k - 1] + hist[k])       # between the s_rel of ranks k and k + 1
    _, U2, _, _ = O.lowrank_preconditioner(R, apply_t, g, tol, 8)
    return max(err, 0.0 if len(U2) == k + 1 else 1.0)


def _scf_case(nspin=1, n=(4, 4, 4), L=(4.0, 4.0, 4.0), N=None, ne=8.0, kT=0.1, seed=2):
    g = O.Grid(n, L)
    V = small_wells(n, L, seed, nwells=2, depth=(1.0, 1.5))
    N = g.M if N is None else N
    eps0, Psi0 = O.lowest_states(V, g, N)
    rho, _ = O.density(np.stack([Psi0] * nspin), np.stack([eps0] * nspin), g, ne, kT, nspin)
    return g, V, N, ne, kT, rho


def pin_scf_derivative_fd(nspin=1):
    """In the full space (N = M), t = chi0 K_c u - u (Eq. (7)) equals the
    derivative of the SCF residual R[rho] = F[V_eff[rho]] - rho along u, taken
    by Richardson-extrapolated central differences of the dense-diagonalisation
    residual (no divided-difference code on that side)."""
    g, V, N, ne, kT, rho = _scf_case(nspin)
    rng = np.random.default_rng(7 + nspin)
    u = rng.standard_normal((nspin,) + g.shape)
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u /= np.sqrt(O.inner(u, u, g))
    _, Psi, eps = O.scf_residual(rho, V, g, N, ne, kT, nspin)
    t = O.residual_derivative(Psi, eps, g, ne, kT, u[None], nspin)[0][0]

    def central(lam):
        Rp = O.scf_residual(rho + lam * u, V, g, N, ne, kT, nspin)[0]
        Rm = O.scf_residual(rho - lam * u, V, g, N, ne, kT, nspin)[0]
        return (Rp - Rm) / (2 * lam)
    lam = 2e-3
    fd = (4 * central(lam / 2) - central(lam)) / 3
    return _rel(t, fd)


def scf_fixed_points(n=(6, 6, 6), L=(6.0, 6.0, 6.0), N=40, ne=12.0, kT=0.05, seed=3):
    """The LRDM SCF (Eq. (4) with P^lr_r, Sec. II B) against plain damped mixing
    rho <- rho + 0.1 R, both from a uniform density.  Returns (max difference of
    the two fixed points, LRDM steps, mixing steps, largest |integral of rho -
    N_e| over the LRDM iterates, final ||R|| of each)."""
    g = O.Grid(n, L)
    V = small_wells(n, L, seed, nwells=3, depth=(1.0, 2.0))
    rho0 = np.full((1,) + g.shape, ne / (g.M * g.dv))
    rho_l, log = O.lrdm_scf(rho0, V, g, N, ne, kT, 1, s_tol=0.3, r_max=20, tol=1e-10,
                            max_iter=60)
    rho_m = rho0.copy()
    steps = 0
    for steps in range(1, 400):
        R = O.scf_residual(rho_m, V, g, N, ne, kT)[0]
        nR = np.sqrt(O.inner(R, R, g))
        if nR < 1e-10:
            break
        rho_m = rho_m + 0.1 * R
    count = abs(g.dv * rho_l.sum() - ne)
    return (float(np.abs(rho_l - rho_m).max()), len(log), steps, count, log[-1][0], nR)


# ------------------------------------------------------------------ recursive Fermi expansion
def _matrix_recursion(A, mu, kT, depth):
    """P_T(...P_0(A - mu I)) for a full symmetric matrix A, with explicit matrix
    products and inverses (Eqs. (23)-(24) as written, no diagonal shortcut)."""
    N = A.shape[0]
    X = 0.5 * np.eye(N) - (2.0 ** (-(depth + 2))) * (A - mu * np.eye(N)) / kT
    for _ in range(depth):
        X2 = X @ X
        IX = np.eye(N) - X
        X = X2 @ np.linalg.inv(X2 + IX @ IX)
    return X


def pin_recursive_response_fd(depth=8):
    """The oracle's first-order perturbation of the recursion at diagonal D equals
    the Richardson central difference in lam of the full-matrix recursion applied
    to D + lam H' (fixed mu)."""
    rng = np.random.default_rng(31)
    N = 12
    eps = np.sort(rng.uniform(-0.2, 0.2, N))
    eps[5] = eps[4]                                  # a degenerate pair
    A = rng.standard_normal((N, N))
    Hp = 0.5 * (A + A.T)
    mu, kT = 0.01, 0.03
    _, xp = O.recursive_fermi_response(eps, mu, kT, Hp, depth)
    D = np.diag(eps)

    def central(lam):
        return (_matrix_recursion(D + lam * Hp, mu, kT, depth)
                - _matrix_recursion(D - lam * Hp, mu, kT, depth)) / (2 * lam)
    lam = 1e-4
    fd = (4 * central(lam / 2) - central(lam)) / 3
    return _rel(xp, fd)


def pin_recursive_density_response(depths=(6, 10, 16, 24)):
    """delta rho with the recursive expansion: its integral vanishes (the
    traceless condition conserves the electron count) and it converges to the
    exact divided-difference response as T grows.  Returns (largest |integral|,
    relative errors vs the exact response per depth)."""
    g, N, ne, kT = O.Grid((5, 4, 4), (2.5, 2.0, 2.0)), 12, 8.0, 0.05
    rng = np.random.default_rng(41)
    Q, _ = np.linalg.qr(rng.standard_normal((g.M, N)))
    Psi = Q.T.reshape((N,) + g.shape)
    eps = np.sort(rng.uniform(-0.6, 0.4, N))
    dV = rng.standard_normal((2, 1) + g.shape)
    exact, _, _ = O.density_response(Psi, eps, g, ne, kT, dV, 1)
    errs = []
    integral = 0.0
    for T in depths:
        d, _, _ = O.density_response_recursive(Psi, eps, g, ne, kT, dV, T, 1)
        integral = max(integral, float(np.abs(g.dv * d.sum(axis=(1, 2, 3, 4))).max()))
        errs.append(_rel(d, exact))
    return integral, errs


# ------------------------------------------------------------------ accumulated low-rank step
def pin_accumulate_union_lstsq():
    """For a linear residual map, the accumulated step over kept directions (from
    an earlier residual) plus new ones equals the least-squares minimiser of
    ||J x - R|| over the span of all of them: U lstsq(J U, R), with J U formed
    from the matrix (no S, no Gram-Schmidt).  Also checks the kept directions
    enter unchanged and the new ones are orthonormal to them."""
    g, J, R0, apply_t = _linear_residual(seed=13)
    _, U0, T0, _ = O.lowrank_preconditioner(R0, apply_t, g, 0.0, 3)
    R1 = np.random.default_rng(14).standard_normal(R0.shape)
    drho, U, T, s_rel, added, fit = O.lowrank_accumulate(R1, apply_t, g, 0.0, list(U0), list(T0), 4)
    Um = U.reshape(len(U), -1).T
    JU = J @ Um
    y = np.linalg.lstsq(JU, R1.ravel(), rcond=None)[0]
    err = _rel(drho.ravel(), Um @ y)
    err = max(err, abs(s_rel - np.linalg.norm(JU @ y - R1.ravel()) / np.linalg.norm(R1.ravel())))
    err = max(err, _rel(fit.ravel(), JU @ y), float(added != 4))
    err = max(err, _rel(U[:3], U0), np.abs(g.dv * Um.T @ Um - np.eye(len(U))).max())
    return err


def pin_accumulate_empty_history():
    """With no history the accumulated step is the LRDM step of Eqs. (8)-(10)."""
    g, J, R, apply_t = _linear_residual()
    d1, U1, _, h1 = O.lowrank_preconditioner(R, apply_t, g, 0.3, 10)
    d2, U2, _, s2, added, _ = O.lowrank_accumulate(R, apply_t, g, 0.3, [], [], 10)
    return max(_rel(d2, d1), abs(s2 - h1[-1]), float(added != len(U1)))


def pin_linear_prediction():
    """Eq. (12): for a linear residual map with exact directional derivatives the
    predicted residual R - alpha I_r^t R equals the residual after the step
    rho - alpha drho_bar, so beta of Eq. (13) vanishes."""
    g, J, R0, apply_t = _linear_residual(seed=17)
    alpha = 0.5
    drho, _, _, _, _, fit = O.lowrank_accumulate(R0, apply_t, g, 0.3, [], [], 5)
    R_lin = O.predicted_residual(R0, fit, alpha)
    R1 = R0 + apply_t(-alpha * drho)                 # R[rho - alpha drho] of the linear map
    beta = O.linearity_indicator(np.sqrt(O.inner(R_lin, R_lin, g)), np.sqrt(O.inner(R1, R1, g)))
    return max(_rel(R_lin, R1), beta)


def lrdma_vs_lrdm(n=(8, 8, 8), L=(9.0, 9.0, 9.0), N=60, ne=16.0, kT=0.02, seed=5):
    """LRDMA and LRDM SCF from a uniform density: (max density difference of their
    fixed points, LRDMA directions, LRDM directions, LRDMA events, final ||R||)."""
    g = O.Grid(n, L)
    V = small_wells(n, L, seed, nwells=4, depth=(1.0, 2.0))
    rho0 = np.full((1,) + g.shape, ne / (g.M * g.dv))
    rho_a, log_a = O.lrdma_scf(rho0, V, g, N, ne, kT, 1, tol=1e-9, max_iter=80)
    rho_l, log_l = O.lrdm_scf(rho0, V, g, N, ne, kT, 1, tol=1e-9, max_iter=80)
    return (float(np.abs(rho_a - rho_l).max()), sum(x[2] for x in log_a),
            sum(x[1] for x in log_l), [x[3] for x in log_a], log_a[-1][0])


# ------------------------------------------------------------------ LDA exchange-correlation
def pin_pz81_continuity():
    """The Perdew-Zunger fit joins its two branches at rs = 1 with a continuous
    value and slope (that is how its constants were chosen), for the
    unpolarised and the polarised gas: returns the largest relative jump."""
    err = 0.0
    for kind in ("U", "P"):
        lo = O.pz81_eps_c(np.array([1.0 + 1e-9]), kind)[0]
        hi = O.pz81_eps_c(np.array([1.0 - 1e-9]), kind)[0]
        d_lo = (O.pz81_eps_c(np.array([1.0 + 1e-5]), kind)[0] - lo) / (1e-5 - 1e-9)
        d_hi = (hi - O.pz81_eps_c(np.array([1.0 - 1e-5]), kind)[0]) / (1e-5 - 1e-9)
        err = max(err, abs(lo - hi) / abs(lo), abs(d_lo - d_hi) / abs(d_lo))
    return err


def pin_lda_exchange_uniform_gas():
    """The exchange part of the LDA energy per electron is the uniform-gas value
    -(3/4)(9/(4 pi^2))^{1/3} / rs = -0.458165... / rs (one channel), and the
    spin-scaled form gives the same at zero polarisation and 2^{1/3} times it
    when fully polarised."""
    rs = np.array([0.5, 1.0, 2.0, 5.0])
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    ex_ref = -0.75 * (9.0 / (4.0 * np.pi ** 2)) ** (1.0 / 3.0) / rs
    ex1 = O.lda_energy_density(n[None]) / n - O.pz81_eps_c(rs, "U")
    ex2 = O.lda_energy_density(np.stack([n / 2, n / 2])) / n - O.pz81_eps_c(rs, "U")
    # fully polarised: exchange of the channel density at twice the unpolarised value
    eps_full = O.lda_energy_density(np.stack([n, np.zeros_like(n)])) / n - O.pz81_eps_c(rs, "P")
    return max(_rel(ex1, ex_ref), _rel(ex2, ex_ref), _rel(eps_full, 2 ** (1 / 3) * ex_ref))


def pin_lda_derivatives_fd():
    """V and f of lda_xc against central differences of the energy density and
    of V, one and two channels; and the spin identities at zero polarisation:
    V_up = V of the total density, f_up,up + f_up,down = 2 f of the total."""
    rng = np.random.default_rng(8)
    rho1 = rng.uniform(1e-3, 0.5, (1, 7))
    rho2 = rng.uniform(1e-3, 0.3, (2, 7))
    err = 0.0
    for rho in (rho1, rho2):
        V, f = O.lda_xc(rho)
        ns = rho.shape[0]
        for a in range(ns):
            h = 1e-6 * rho[a]
            up, dn = rho.copy(), rho.copy()
            up[a] += h
            dn[a] -= h
            dE = (O.lda_energy_density(up) - O.lda_energy_density(dn)) / (2 * h)
            err = max(err, _rel(V[a], dE))
            Vu, _ = O.lda_xc(up)
            Vd, _ = O.lda_xc(dn)
            for b in range(ns):
                err = max(err, _rel(f[b][a], (Vu[b] - Vd[b]) / (2 * h)))
    n = rho1[0]
    V1, f1 = O.lda_xc(rho1)
    V2, f2 = O.lda_xc(np.stack([n / 2, n / 2]))
    err = max(err, _rel(V2[0], V1[0]), _rel(f2[0][0] + f2[0][1], 2 * f1[0][0]))
    return err


def pin_scf_derivative_fd_xc(nspin=1):
    """With the LDA term, t = chi0 (K_c + K_xc) u - u equals the Richardson central
    difference of the dense-diagonalisation SCF residual with V_eff = V_ext + V_H
    + V_xc (full space, N = M); for two channels at an unequal spin split."""
    g, V, N, ne, kT, rho = _scf_case(nspin)
    if nspin == 2:
        rho = np.stack([1.3 * rho[0], 0.7 * rho[1]])
    rng = np.random.default_rng(27 + nspin)
    u = rng.standard_normal((nspin,) + g.shape)
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u /= np.sqrt(O.inner(u, u, g))
    _, Psi, eps = O.scf_residual(rho, V, g, N, ne, kT, nspin, xc=True)
    fxc = O.lda_xc(rho)[1]
    t = O.residual_derivative(Psi, eps, g, ne, kT, u[None], nspin, fxc)[0][0]

    def central(lam):
        Rp = O.scf_residual(rho + lam * u, V, g, N, ne, kT, nspin, xc=True)[0]
        Rm = O.scf_residual(rho - lam * u, V, g, N, ne, kT, nspin, xc=True)[0]
        return (Rp - Rm) / (2 * lam)
    lam = 2e-3
    fd = (4 * central(lam / 2) - central(lam)) / 3
    return _rel(t, fd)


# ------------------------------------------------------------------ parameters printed in Sec. III A
def sec3a_parameters():
    """The preconditioner parameters Sec. III A prints (tests/golden fixture)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "sec3a_parameters.json")) as f:
        return json.load(f)


def pin_damping_schedule():
    """alpha = 0.1 until ||R|| goes below 2.0, then 0.5 from that step on."""
    p = sec3a_parameters()
    far, near, sw = p["alpha_far"], p["alpha_near"], p["alpha_switch_below_norm_R"]
    return (O.damping(5.0) == far and O.damping(sw) == far and O.damping(1.5) == near
            and O.damping(0.5) == near and O.damping(np.nextafter(sw, 0.0)) == near
            and O.damping(3.0, switched=True) == near)


def pin_lrdma_gates():
    """Accumulation only while ||R|| < 1.0 (CR at 1.5, where alpha is already
    0.5); CL once beta exceeds 0.1; reuse when the kept fit meets s_tol."""
    p = sec3a_parameters()
    gate, btol = p["lrdma_accumulate_only_below_norm_R"], p["lrdma_beta_tol"]
    s_tol = p["s_tol_range"][1]

    def ev(**kw):
        args = dict(has_history=True, clear_pending=False, beta=0.0, kept_s_rel=0.9,
                    norm_R=0.5, s_tol=s_tol)
        args.update(kw)
        return O.lrdma_event(**args)
    return (ev(norm_R=1.5) == "CR" and O.damping(1.5) == p["alpha_near"]
            and ev(norm_R=gate) == "CR" and ev(norm_R=np.nextafter(gate, 0.0)) == "accumulate"
            and ev(beta=btol * 1.01) == "CL" and ev(beta=btol) == "accumulate"
            and ev(kept_s_rel=0.5 * s_tol, norm_R=1.5) == "reuse"
            and ev(clear_pending=True) == "CT" and ev(has_history=False) == "fresh")


# ------------------------------------------------------------------ Brillouin-zone sampling
def pin_bloch_plane_wave():
    """exp(i q.x) is an eigenvector of H_k for a constant potential V0, with
    eigenvalue sum_d (1 - cos((q_d + k_d) h_d)) / h_d^2 + V0 (q on the grid)."""
    g = O.Grid((6, 5, 4), (3.0, 2.6, 2.2))
    V0, k = 0.37, (0.41, -0.77, 1.3)
    z, y, x = np.meshgrid(*(np.arange(m) * hd for m, hd in zip(g.shape, g.h[::-1])),
                          indexing="ij")
    err = 0.0
    for m in ((1, 2, 3), (0, 0, 0), (5, 4, 1)):
        q = [2 * np.pi * m[d] / g.L[d] for d in range(3)]
        u = np.exp(1j * (q[0] * x + q[1] * y + q[2] * z))
        lam = sum((1 - np.cos((q[d] + k[d]) * g.h[d])) / g.h[d] ** 2 for d in range(3)) + V0
        err = max(err, _rel(O.bloch_hamiltonian_apply(u, V0 * np.ones(g.shape), g, k), lam * u))
    return err


def pin_bloch_dense():
    """H_k applied to the identity against the Bloch matrix assembled hop by hop."""
    n, L = (4, 3, 3), (2.4, 2.0, 2.1)
    g = O.Grid(n, L)
    V = np.random.default_rng(31).uniform(-1, 0, g.shape)
    k = (0.9, -0.4, 0.3)
    Hd = O.bloch_hamiltonian_apply(np.eye(g.M).reshape((g.M,) + g.shape), V, g, k)
    return _rel(Hd.reshape(g.M, g.M).T, bf.dense_bloch_hamiltonian(V, n, L, k))


def _supercell(seed=33):
    """A primitive cell and its double along x; k = 0 and pi/Lx sample the
    double's zone-folded spectrum (Bloch's theorem)."""
    n, L = (4, 3, 3), (2.4, 2.0, 2.1)
    g = O.Grid(n, L)
    V = small_wells(n, L, seed, nwells=2)
    n2, L2 = (8, 3, 3), (4.8, 2.0, 2.1)
    g2 = O.Grid(n2, L2)
    V2 = np.concatenate([V, V], axis=2)
    ks = [(0.0, 0.0, 0.0), (np.pi / L[0], 0.0, 0.0)]
    return g, V, g2, V2, ks


def pin_bloch_supercell_spectrum():
    """The eigenvalues of H_k at k = 0 and pi/Lx on the primitive cell, together,
    are those of H on the cell doubled along x."""
    g, V, g2, V2, ks = _supercell()
    lam_k = np.sort(np.concatenate([O.lowest_bloch_states(V, g, k, g.M)[0] for k in ks]))
    lam_2 = np.linalg.eigvalsh(bf.dense_hamiltonian(V2, g2.n, g2.L))
    return float(np.max(np.abs(lam_k - lam_2)) / np.max(np.abs(lam_2)))


def pin_bz_supercell_response():
    """Full space (every state of every k): the zone-sampled response at k = 0
    and pi/Lx (weights 1/2) equals the response of the doubled cell at one point,
    which is the dense-diagonalisation derivative of its density, for a
    perturbation with the primitive period."""
    g, V, g2, V2, ks = _supercell()
    ne, kT = 9.0, 0.05
    states = [O.lowest_bloch_states(V, g, k, g.M) for k in ks]
    eps = np.stack([e for e, _ in states])[None]
    Psi = np.stack([p for _, p in states])[None]
    dV = np.random.default_rng(34).standard_normal(g.shape)
    drho, _, _ = O.density_response_bz(Psi, eps, [0.5, 0.5], g, ne, kT, dV[None, None], 1)
    dV2 = np.concatenate([dV, dV], axis=2)
    ref = bf.richardson_derivative(
        lambda t: bf.full_space_density(V2 + t * dV2, g2.n, g2.L, 2 * ne, kT, 2.0), 1e-3)
    ref = ref.reshape(g2.shape)
    return max(_rel(drho[0, 0], ref[:, :, :4]), _rel(drho[0, 0], ref[:, :, 4:]))


def _bz_subspace_case(nspin=1, seed=35):
    n, L = (5, 4, 4), (3.0, 2.5, 2.5)
    g = O.Grid(n, L)
    V = small_wells(n, L, seed)
    ks = [(0.3, -0.5, 0.2), (-0.8, 0.1, 0.6)]
    w = [0.3, 0.7]
    N = 14
    rng = np.random.default_rng(seed + 1)
    Psi, eps = [], []
    for c in range(nspin):
        Vc = V + (0.05 * c) * rng.standard_normal(g.shape)
        st = [O.lowest_bloch_states(Vc, g, k, N) for k in ks]
        eps.append(np.stack([e for e, _ in st]))
        Psi.append(np.stack([p for _, p in st]))
    ne = 0.6 * N * (2.0 if nspin == 1 else 2.0)
    return g, np.stack(Psi), np.stack(eps), w, ne, 0.04


def pin_bz_subspace_fd(nspin=1):
    """The zone-sampled subspace response against a Richardson central difference
    in lam of (s/dv) sum_k w_k diag(Psi_k f(eigh(D_k + lam H'_k), mu(lam)) Psi_k^H),
    with mu(lam) re-solved from the zone-averaged count (no divided differences)."""
    g, Psi, eps, w, ne, kT = _bz_subspace_case(nspin)
    nk, N = len(w), eps.shape[-1]
    s = O.spin_factor(nspin)
    dV = np.random.default_rng(37).standard_normal((1, nspin) + g.shape)
    drho, _, _ = O.density_response_bz(Psi, eps, w, g, ne, kT, dV, nspin)
    P = [[Psi[c, k].reshape(N, -1) for k in range(nk)] for c in range(nspin)]
    Hp = [[np.einsum("ip,p,jp->ij", P[c][k].conj(), dV[0, c].ravel(), P[c][k], optimize=False)
           for k in range(nk)] for c in range(nspin)]

    def rho_all(lam):
        ws, Ws = {}, {}
        for c in range(nspin):
            for k in range(nk):
                ws[c, k], Ws[c, k] = np.linalg.eigh(np.diag(eps[c, k]) + lam * Hp[c][k])

        def count(mu):
            return s * sum(w[k] * np.sum(bf.occupations(ws[c, k], mu, kT))
                           for c in range(nspin) for k in range(nk)) - ne
        allw = np.concatenate(list(ws.values()))
        from scipy.optimize import brentq
        mu_l = brentq(count, allw.min() - 60 * kT, allw.max() + 60 * kT, xtol=1e-15, rtol=1e-15)
        out = []
        for c in range(nspin):
            rho = 0.0
            for k in range(nk):
                f = bf.occupations(ws[c, k], mu_l, kT)
                B = P[c][k].T @ Ws[c, k]
                rho = rho + w[k] * (s / g.dv) * np.sum(np.abs(B) ** 2 * f[None, :], axis=1)
            out.append(rho)
        return np.concatenate(out)

    ref = bf.richardson_derivative(rho_all, 2e-4)
    return _rel(drho[0].reshape(-1), ref)


def pin_bz_gamma_is_the_real_path():
    """One k-point at k = 0 with real states: the zone-sampled response is the
    real one."""
    n, L = (5, 5, 4), (3.2, 3.2, 2.6)
    g, V, eps, Psi = _rr_system(n, L, 16, seed=13)
    dV = np.random.default_rng(38).standard_normal((2, 1) + g.shape)
    a, mu_a, dmu_a = O.density_response(Psi[None], eps[None], g, 12.0, 0.03, dV, 1)
    b, mu_b, dmu_b = O.density_response_bz(Psi[None, None].astype(np.complex128),
                                           eps[None, None], [1.0], g, 12.0, 0.03, dV, 1)
    return max(_rel(b, a), abs(mu_a - mu_b), _rel(dmu_b, dmu_a))


def bz_invariants(nspin=1):
    """Zone-sampled response: the integral of delta rho vanishes (zone traceless
    condition), <dV_a, chi dV_b> is symmetric and <dV, chi dV> <= 0."""
    g, Psi, eps, w, ne, kT = _bz_subspace_case(nspin)
    dV = np.random.default_rng(39).standard_normal((3, nspin) + g.shape)
    drho, _, _ = O.density_response_bz(Psi, eps, w, g, ne, kT, dV, nspin)
    integral = max(abs(g.dv * drho[q].sum()) / (g.dv * np.abs(drho[q]).sum()) for q in range(3))
    X = np.array([[g.dv * np.sum(dV[a] * drho[b]) for b in range(3)] for a in range(3)])
    sym = float(np.max(np.abs(X - X.T)) / np.max(np.abs(X)))
    return dict(integral=integral, symmetry=sym, nsd=float(np.max(np.linalg.eigvalsh(0.5 * (X + X.T)))))


def pin_bz_time_reversal():
    """For a real potential u_{-k} = conj(u_k): sampling {k, -k} with weights 1/2
    gives the response of {k} alone."""
    g, Psi, eps, w, ne, kT = _bz_subspace_case(1)
    dV = np.random.default_rng(40).standard_normal((1, 1) + g.shape)
    one, _, _ = O.density_response_bz(Psi[:, :1], eps[:, :1], [1.0], g, ne, kT, dV, 1)
    Psi2 = np.concatenate([Psi[:, :1], Psi[:, :1].conj()], axis=1)
    eps2 = np.concatenate([eps[:, :1], eps[:, :1]], axis=1)
    two, _, _ = O.density_response_bz(Psi2, eps2, [0.5, 0.5], g, ne, kT, dV, 1)
    return _rel(two, one)
