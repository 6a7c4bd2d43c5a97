"""FP64 oracle of the LRDM hot path (test infrastructure only; see package doc).

Notation follows the paper, carried to a periodic finite-difference grid (the
paper states the method carries over to finite differences, end of Sec. II D):

* grid of n = (nx, ny, nz) points, spacings h_d = L_d / n_d, cell volume
  element dv = hx*hy*hz, arrays laid out [..., nz, ny, nx];
* a block of N vectors is stored state-major, Psi[i] is state i;
* vectors are l2-orthonormal (sum_p Psi_ip Psi_jp = delta_ij), so real-space
  orbitals are Psi / sqrt(dv) and the FE overlap matrix of Eq. (16) becomes
  dv * I, with n^e(x) the point value;
* s = 2 (spin restricted, Eq. (1)) or s = 1 per channel (spin polarised,
  Sec. II D, which drops the factor 2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    n: tuple      # (nx, ny, nz)
    L: tuple      # (Lx, Ly, Lz)

    @property
    def M(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def h(self):
        return tuple(self.L[d] / self.n[d] for d in range(3))

    @property
    def dv(self):
        hx, hy, hz = self.h
        return hx * hy * hz

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])


def spin_factor(nspin: int) -> float:
    """Occupation per spatial state: 2 for spin-restricted (Eq. (1)), 1 per channel
    when spin polarised (Sec. II D, response per channel without the factor 2)."""
    return 2.0 if nspin == 1 else 1.0


# ---------------------------------------------------------------------------
# Hamiltonian and Chebyshev-filtered subspace iteration (Sec. II C)
# ---------------------------------------------------------------------------
def hamiltonian_apply(Y: np.ndarray, V: np.ndarray, grid: Grid) -> np.ndarray:
    """H Y with H = -1/2 Laplacian + V (Eq. (1)); the Laplacian is the 7-point
    periodic second difference.  Y: [..., nz, ny, nx]."""
    hx, hy, hz = grid.h
    lap = np.zeros_like(Y)
    for axis, hd in ((-1, hx), (-2, hy), (-3, hz)):
        lap += (np.roll(Y, 1, axis=axis) + np.roll(Y, -1, axis=axis) - 2.0 * Y) / (hd * hd)
    return -0.5 * lap + V * Y


def chebyshev_filter(X: np.ndarray, V: np.ndarray, grid: Grid, degree: int,
                     a: float, b: float, a0: float) -> np.ndarray:
    """Scaled Chebyshev filter T_c(Hbar) X / T_c(ybar0) of degree c (Sec. II C).

    Hbar = (H - c0)/e maps the unwanted interval [a, b] to [-1, 1] and the wanted
    spectrum below a to (-inf, -1); e = (b - a)/2, c0 = (b + a)/2, and a0 (a lower
    bound of the spectrum) fixes the scaling ybar0 = (a0 - c0)/e.  This is the
    three-term recurrence of Zhou, Saad, Tiago and Chelikowsky (J. Comput. Phys.
    219, 2006), written out below:
        sigma_1 = e / (a0 - c0),   Y_1 = (sigma_1 / e)(H - c0) X,
        sigma_k = 1 / (2/sigma_1 - sigma_{k-1}),
        Y_k = (2 sigma_k / e)(H - c0) Y_{k-1} - sigma_{k-1} sigma_k Y_{k-2},   Y_0 = X.
    """
    return _chebyshev(X.astype(np.float64, copy=True), lambda Y: hamiltonian_apply(Y, V, grid),
                      degree, a, b, a0)


def _chebyshev(X: np.ndarray, apply_H, degree: int, a: float, b: float, a0: float):
    """The scaled three-term recurrence of chebyshev_filter for any H (apply_H)."""
    e = (b - a) / 2.0
    c0 = (b + a) / 2.0
    sigma1 = e / (a0 - c0)
    y_prev = X
    y = (sigma1 / e) * (apply_H(y_prev) - c0 * y_prev)
    sigma = sigma1
    for _ in range(2, degree + 1):
        sigma_new = 1.0 / (2.0 / sigma1 - sigma)
        y_new = (2.0 * sigma_new / e) * (apply_H(y) - c0 * y) - (sigma * sigma_new) * y_prev
        y_prev, y = y, y_new
        sigma = sigma_new
    return y


def rayleigh_ritz(Y: np.ndarray, V: np.ndarray, grid: Grid):
    """Orthonormalise the filtered block and solve the projected problem (Sec. II C,
    Eq. (15)): Psi_o = orth(Y), Hhat = Psi_o^T H Psi_o, Hhat Q = Q D,
    Psi_R = Psi_o Q.  Returns (eps ascending [N], Psi_R [N][nz][ny][nx])."""
    N = Y.shape[0]
    Ycols = Y.reshape(N, -1).T                       # M x N, the paper's orientation
    Psi_o, _ = np.linalg.qr(Ycols)                   # Householder QR
    HPsi = hamiltonian_apply(Psi_o.T.reshape(Y.shape), V, grid).reshape(N, -1).T
    Hhat = Psi_o.T @ HPsi
    Hhat = 0.5 * (Hhat + Hhat.T)
    eps, Q = np.linalg.eigh(Hhat)
    Psi_R = Psi_o @ Q
    return eps, Psi_R.T.reshape(Y.shape).copy()


# ---------------------------------------------------------------------------
# Occupations and Fermi level (Eq. (1))
# ---------------------------------------------------------------------------
def _logistic(y: np.ndarray) -> np.ndarray:
    """1 / (1 + exp(y)) without overflow."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    pos = y >= 0
    ey = np.exp(-y[pos])
    out[pos] = ey / (1.0 + ey)
    out[~pos] = 1.0 / (1.0 + np.exp(y[~pos]))
    return out


def fermi_dirac(eps: np.ndarray, mu: float, kT: float):
    """f = 1/(1 + exp((eps - mu)/kT)) (Eq. (1)), 1 - f computed as f of the
    negated argument (no subtraction), and f' = df/deps = -f (1 - f) / kT."""
    y = (np.asarray(eps, dtype=np.float64) - mu) / kT
    f = _logistic(y)
    omf = _logistic(-y)
    fp = -f * omf / kT
    return f, omf, fp


def fermi_level(eps: np.ndarray, n_electrons: float, kT: float, nspin: int = 1,
                max_iter: int = 200):
    """mu solving s * sum_{sigma,i} f(eps_sigma,i, mu) = N_e (Eq. (1)) by bisection on
    [min eps - 50 kT, max eps + 50 kT]; stops when the bracket is within 2 ulp of
    its midpoint or after max_iter halvings.  Returns (mu, converged)."""
    eps = np.asarray(eps, dtype=np.float64).reshape(nspin, -1)
    s = spin_factor(nspin)
    lo = float(eps.min()) - 50.0 * kT
    hi = float(eps.max()) + 50.0 * kT
    converged = False
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if hi - lo <= 2.0 * np.spacing(abs(mid)):
            converged = True
            break
        count = s * float(np.sum(fermi_dirac(eps, mid, kT)[0]))
        if count > n_electrons:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi), converged


def divided_differences(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """F_ij = (f_i - f_j)/(eps_i - eps_j), F_ii = f'_i: the Hadamard multiplier that
    gives the derivative of f(D + lam H', mu) at lam = 0 for diagonal D (Eqs. (21)-(22);
    Daleckii-Krein).  For eps_lo <= eps_hi and z = (eps_lo - eps_hi)/kT <= 0 the exact
    identity f_lo - f_hi = -f_lo (1 - f_hi) expm1(z) gives
        F = -(1/kT) f_lo (1 - f_hi) expm1(z)/z,
    which neither overflows nor cancels near degeneracy (expm1(z)/z -> 1)."""
    eps = np.asarray(eps, dtype=np.float64)
    e_lo = np.minimum(eps[:, None], eps[None, :])
    e_hi = np.maximum(eps[:, None], eps[None, :])
    f_lo, _, _ = fermi_dirac(e_lo, mu, kT)
    _, omf_hi, _ = fermi_dirac(e_hi, mu, kT)
    z = (e_lo - e_hi) / kT
    phi = np.ones_like(z)
    nz = z != 0.0
    phi[nz] = np.expm1(z[nz]) / z[nz]
    return -(f_lo * omf_hi * phi) / kT


# ---------------------------------------------------------------------------
# Subspace density response (Sec. II C, Eqs. (19)-(22) and the traceless condition)
# ---------------------------------------------------------------------------
def projected_perturbation(Psi: np.ndarray, dV: np.ndarray) -> np.ndarray:
    """Hbreve' = Psi_R^T H' Psi_R with H' = diag(dV) (Eq. (21)); Psi: [N][...]."""
    N = Psi.shape[0]
    P = Psi.reshape(N, -1).T                         # M x N
    return P.T @ (dV.reshape(-1)[:, None] * P)


def fermi_shift(Hp: list, fprime: list) -> float:
    """mu' from Tr Gamma^(1) = 0 summed over channels (text after Eq. (24)):
    mu' = sum f'_i H'_ii / sum f'_i; zero when sum f' underflows (mu in a gap)."""
    num = 0.0
    den = 0.0
    for H, fp in zip(Hp, fprime):
        num += float(np.sum(fp * np.diag(H)))
        den += float(np.sum(fp))
    if abs(den) < 1e-300:
        return 0.0
    return num / den


def response_density_matrix(F: np.ndarray, Hp: np.ndarray, dmu: float,
                            fprime: np.ndarray) -> np.ndarray:
    """Gammabreve^(1) = d/dlam f(D + lam H', mu + lam mu') = F o H' - mu' diag(f')
    (Eq. (22) with the exact Fermi-Dirac divided differences)."""
    return F * Hp - dmu * np.diag(fprime)


def density_from_matrix(Psi: np.ndarray, Gamma: np.ndarray, dv: float, s: float) -> np.ndarray:
    """(s/dv) diag(Psi_R Gamma Psi_R^T) at every grid point (Eqs. (16), (20) with
    M = dv I and point-value n^e)."""
    N = Psi.shape[0]
    P = Psi.reshape(N, -1).T                         # M x N
    Z = P @ Gamma
    return ((s / dv) * np.sum(P * Z, axis=1)).reshape(Psi.shape[1:])


def density(Psi: np.ndarray, eps: np.ndarray, grid: Grid, n_electrons: float, kT: float,
            nspin: int = 1):
    """Output density rho = (s/dv) sum_i f_i |Psi_i|^2 per channel (Eq. (16))."""
    Psi = Psi.reshape((nspin,) + Psi.shape[-4:])
    eps = np.asarray(eps).reshape(nspin, -1)
    mu, _ = fermi_level(eps, n_electrons, kT, nspin)
    s = spin_factor(nspin)
    rho = np.empty((nspin,) + grid.shape)
    for c in range(nspin):
        f, _, _ = fermi_dirac(eps[c], mu, kT)
        rho[c] = density_from_matrix(Psi[c], np.diag(f), grid.dv, s)
    return rho, mu


def density_response(Psi: np.ndarray, eps: np.ndarray, grid: Grid, n_electrons: float,
                     kT: float, dV: np.ndarray, nspin: int = 1):
    """delta rho_k for each perturbation dV_k in the Ritz subspace (Eqs. (20)-(22),
    Sec. II D for two channels with a common mu and mu').

    Psi [nspin][N][nz][ny][nx], eps [nspin][N], dV [r][nspin][nz][ny][nx].
    Returns (drho [r][nspin][nz][ny][nx], mu, dmu [r])."""
    Psi = Psi.reshape((nspin,) + Psi.shape[-4:])
    eps = np.asarray(eps, dtype=np.float64).reshape(nspin, -1)
    dV = dV.reshape((-1, nspin) + grid.shape)
    r = dV.shape[0]
    s = spin_factor(nspin)
    mu, _ = fermi_level(eps, n_electrons, kT, nspin)
    occ = [fermi_dirac(eps[c], mu, kT) for c in range(nspin)]
    Fm = [divided_differences(eps[c], mu, kT) for c in range(nspin)]
    drho = np.empty_like(dV)
    dmu = np.empty(r)
    for k in range(r):
        Hp = [projected_perturbation(Psi[c], dV[k, c]) for c in range(nspin)]
        dmu[k] = fermi_shift(Hp, [occ[c][2] for c in range(nspin)])
        for c in range(nspin):
            G = response_density_matrix(Fm[c], Hp[c], dmu[k], occ[c][2])
            drho[k, c] = density_from_matrix(Psi[c], G, grid.dv, s)
    return drho, mu, dmu


# ---------------------------------------------------------------------------
# Residual derivative t = chi0 K u - u (Eqs. (3), (7))
# ---------------------------------------------------------------------------
def hartree_kernel(u: np.ndarray, grid: Grid) -> np.ndarray:
    """K_c u: the Hartree potential of density u, -Lap_h dV = 4 pi u (Eq. (3)),
    with the same 7-point Laplacian as H; the q = 0 component is set to zero."""
    nx, ny, nz = grid.n
    hx, hy, hz = grid.h
    kx = 2 * np.pi * np.arange(nx) / nx
    ky = 2 * np.pi * np.arange(ny) / ny
    kz = 2 * np.pi * np.arange(nz) / nz
    lam = ((2 - 2 * np.cos(kz))[:, None, None] / hz ** 2
           + (2 - 2 * np.cos(ky))[None, :, None] / hy ** 2
           + (2 - 2 * np.cos(kx))[None, None, :] / hx ** 2)
    mult = np.zeros_like(lam)
    mult[lam > 0] = 4 * np.pi / lam[lam > 0]
    mult[0, 0, 0] = 0.0
    uh = np.fft.fftn(u, axes=(-3, -2, -1))
    return np.real(np.fft.ifftn(uh * mult, axes=(-3, -2, -1)))


def residual_derivative(Psi: np.ndarray, eps: np.ndarray, grid: Grid, n_electrons: float,
                        kT: float, u: np.ndarray, nspin: int = 1, fxc=None):
    """t_k = d/dlam R[rho + lam u_k] = chi0 K u_k - u_k (Eqs. (3), (7)).  K = K_c by
    default: the Hartree potential couples to the total density, so every channel
    sees dV = K_c (sum_sigma u_sigma).  With fxc [nspin][nspin][nz][ny][nx] (the
    LDA kernel, lda_xc) K = K_c + K_xc, and channel c also sees the local term
    sum_c' fxc[c][c'] u_c'.  u, t: [r][nspin][nz][ny][nx]."""
    u = u.reshape((-1, nspin) + grid.shape)
    dV = np.empty_like(u)
    for k in range(u.shape[0]):
        vh = hartree_kernel(u[k].sum(axis=0), grid)
        for c in range(nspin):
            dV[k, c] = vh
            if fxc is not None:
                dV[k, c] = dV[k, c] + sum(fxc[c][d] * u[k, d] for d in range(nspin))
    drho, mu, dmu = density_response(Psi, eps, grid, n_electrons, kT, dV, nspin)
    return drho - u, mu, dmu


# ---------------------------------------------------------------------------
# LDA exchange-correlation (the K_xc part of K in Eq. (3), Sec. II D for spin)
# ---------------------------------------------------------------------------
# Perdew-Zunger (1981) fit of the Ceperley-Alder correlation energy per electron,
# eps_c(rs) = gamma / (1 + beta1 sqrt(rs) + beta2 rs) for rs >= 1 and
# A ln rs + B + C rs ln rs + D rs for rs < 1, unpolarised (U) and fully
# polarised (P) gas, interpolated in the spin polarisation zeta with the
# von Barth-Hedin function f(zeta).
PZ81 = {
    "U": dict(gamma=-0.1423, beta1=1.0529, beta2=0.3334, A=0.0311, B=-0.048, C=0.0020, D=-0.0116),
    "P": dict(gamma=-0.0843, beta1=1.3981, beta2=0.2611, A=0.01555, B=-0.0269, C=0.0007,
              D=-0.0048),
}
XC_RHO_MIN = 1e-12      # points where a channel density is below this carry no xc term


def pz81_eps_c(rs, kind):
    """eps_c(rs) of the Perdew-Zunger fit for the unpolarised ("U") or fully
    polarised ("P") gas; works on numpy arrays and torch tensors."""
    c = PZ81[kind]
    lib = torch_or_numpy(rs)
    low = c["gamma"] / (1.0 + c["beta1"] * lib.sqrt(rs) + c["beta2"] * rs)
    lnrs = lib.log(rs)
    high = c["A"] * lnrs + c["B"] + c["C"] * rs * lnrs + c["D"] * rs
    return lib.where(rs >= 1.0, low, high)


def torch_or_numpy(x):
    import torch
    return torch if isinstance(x, torch.Tensor) else np


def lda_energy_density(rho):
    """LDA exchange-correlation energy per volume e_xc at each point.
    rho: [nspin][...] with nspin = 1 (total density) or 2 (spin densities).
    Exchange: Slater, -(3/4)(3/pi)^{1/3} rho^{4/3} for the total density, or the
    spin-scaled sum -(3/4)(6/pi)^{1/3} sum_sigma rho_sigma^{4/3}.
    Correlation: rho eps_c(rs, zeta) with rs = (3/(4 pi rho))^{1/3},
    eps_c = eps_c^U + f(zeta)(eps_c^P - eps_c^U),
    f(zeta) = ((1+zeta)^{4/3} + (1-zeta)^{4/3} - 2) / (2^{4/3} - 2).
    Works on numpy arrays and torch tensors (for the derivatives)."""
    lib = torch_or_numpy(rho)
    nspin = rho.shape[0]
    n = rho.sum(axis=0) if lib is np else rho.sum(dim=0)
    rs = (3.0 / (4.0 * np.pi * n)) ** (1.0 / 3.0)
    if nspin == 1:
        ex = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (4.0 / 3.0)
        ec = n * pz81_eps_c(rs, "U")
    else:
        ex = -0.75 * (6.0 / np.pi) ** (1.0 / 3.0) * (rho[0] ** (4.0 / 3.0) + rho[1] ** (4.0 / 3.0))
        zeta = (rho[0] - rho[1]) / n
        fz = ((1 + zeta) ** (4.0 / 3.0) + (1 - zeta) ** (4.0 / 3.0) - 2.0) / (2 ** (4.0 / 3.0) - 2.0)
        eu, ep = pz81_eps_c(rs, "U"), pz81_eps_c(rs, "P")
        ec = n * (eu + fz * (ep - eu))
    return ex + ec


def lda_xc(rho: np.ndarray):
    """Potential and kernel of the LDA: V_sigma = d e_xc / d rho_sigma and
    f_{sigma sigma'} = d^2 e_xc / d rho_sigma d rho_sigma' at every point, by
    double-precision automatic differentiation (torch, CPU) of
    lda_energy_density.  Points where any channel density is below XC_RHO_MIN
    get zero.  rho: [nspin][...].  Returns (V [nspin][...],
    f [nspin][nspin][...])."""
    import torch
    r = torch.tensor(np.asarray(rho, dtype=np.float64), requires_grad=True)
    nspin = r.shape[0]
    live = torch.all(r.detach() >= XC_RHO_MIN, dim=0)
    safe = torch.where(live, r, torch.ones_like(r))          # keeps the derivatives finite
    e = lda_energy_density(safe)
    (V,) = torch.autograd.grad(e.sum(), r, create_graph=True)
    f = torch.empty((nspin,) + tuple(r.shape), dtype=torch.float64)
    for a in range(nspin):
        (row,) = torch.autograd.grad(V[a].sum(), r, retain_graph=True)
        f[a] = row
    zero = torch.zeros((), dtype=torch.float64)
    V = torch.where(live, V, zero)
    f = torch.where(live, f, zero)
    return V.detach().numpy(), f.detach().numpy()


# ---------------------------------------------------------------------------
# Low-rank approximation of J and the damped quasi-Newton step (Sec. II B,
# Eqs. (4), (7)-(10)) on a model SCF map rho -> F[V_eff[rho]] (Sec. II A)
# ---------------------------------------------------------------------------
def inner(a: np.ndarray, b: np.ndarray, grid: Grid) -> float:
    """<a, b>, the integral of a b over the cell (Sec. II A), as dv times the sum
    over grid points; for a spin-polarised pair the sum also runs over both
    channels (the direct-sum inner product of Sec. II D)."""
    return grid.dv * float(np.sum(a * b))


def lowrank_preconditioner(R: np.ndarray, apply_t, grid: Grid, s_tol: float, r_max: int):
    """drho_bar = P^lr_r R (Eq. (9)) with the rank r chosen adaptively (Eq. (10)).

    u_1 = R / ||R||.  For each direction u_i, t_i = apply_t(u_i) is the directional
    derivative of the residual along u_i (Eq. (7)).  With the t's so far,
    S_ij = <t_i, t_j>, c_j = <t_j, R>, y = S^{-1} c and
    s_rel = ||sum_i t_i y_i - R|| / ||R||.  Stop when s_rel < s_tol or r = r_max;
    otherwise the next direction is t_i minus its projections on u_1..u_i (all
    taken from t_i itself), normalised (Eq. (8)).

    Returns (drho_bar = sum_i y_i u_i, U [r][...], T [r][...], s_rel after each
    rank [r]).  A zero residual gives drho_bar = 0 and rank 0."""
    nR = np.sqrt(inner(R, R, grid))
    if nR == 0.0:
        return np.zeros_like(R), np.zeros((0,) + R.shape), np.zeros((0,) + R.shape), np.zeros(0)
    U = [R / nR]
    T = []
    hist = []
    while True:
        T.append(apply_t(U[-1]))
        r = len(T)
        S = np.array([[inner(T[i], T[j], grid) for j in range(r)] for i in range(r)])
        c = np.array([inner(T[j], R, grid) for j in range(r)])
        y = np.linalg.solve(S, c)
        fit = sum(y[i] * T[i] for i in range(r))
        hist.append(np.sqrt(inner(fit - R, fit - R, grid)) / nR)
        if hist[-1] < s_tol or r == r_max:
            break
        u = T[-1]
        u = u - sum(inner(u, U[k], grid) * U[k] for k in range(r))
        U.append(u / np.sqrt(inner(u, u, grid)))
    drho = sum(y[i] * U[i] for i in range(r))
    return drho, np.array(U), np.array(T), np.array(hist)


def lowrank_accumulate(R: np.ndarray, apply_t, grid: Grid, s_tol: float, U_prev, T_prev,
                       r_add_max: int):
    """The accumulated low-rank step of LRDMA (Sec. II B 1, Eq. (14)).

    U_prev, T_prev: directions and derivatives kept from earlier SCF steps (the u's
    orthonormal).  If they already fit R to s_rel < s_tol (Eq. (10)), nothing is
    added.  Otherwise new directions are added one at a time: the first is R with
    its projections on all earlier directions removed, normalised; each later one
    is the newest t with its projections on all directions removed, normalised
    (Eq. (8) against the whole history); each new t comes from apply_t at the
    current density.  Adding stops when s_rel < s_tol or r_add_max were added
    (r_add_max = 0: only the kept directions are fitted).  P^lr R (Eq. (9)) then
    uses every direction, kept and new.

    Returns (drho_bar, U, T, s_rel, added, fit) with fit = sum_i y_i t_i, the
    low-rank approximation of J applied to drho_bar (I_r^t R)."""
    U = [u for u in U_prev]
    T = [t for t in T_prev]
    nR = np.sqrt(inner(R, R, grid))

    def solve():
        r = len(T)
        S = np.array([[inner(T[i], T[j], grid) for j in range(r)] for i in range(r)])
        c = np.array([inner(T[j], R, grid) for j in range(r)])
        y = np.linalg.solve(S, c)
        fit = sum(y[i] * T[i] for i in range(r))
        return y, fit, np.sqrt(inner(fit - R, fit - R, grid)) / nR

    added = 0
    if T:
        y, fit, s_rel = solve()
        if s_rel < s_tol or r_add_max == 0:
            return sum(y[i] * U[i] for i in range(len(U))), np.array(U), np.array(T), s_rel, 0, fit
    v = R
    while True:
        u = v - sum(inner(v, U[k], grid) * U[k] for k in range(len(U)))
        U.append(u / np.sqrt(inner(u, u, grid)))
        T.append(apply_t(U[-1]))
        added += 1
        y, fit, s_rel = solve()
        if s_rel < s_tol or added == r_add_max:
            break
        v = T[-1]
    return sum(y[i] * U[i] for i in range(len(U))), np.array(U), np.array(T), s_rel, added, fit


def predicted_residual(R: np.ndarray, fit: np.ndarray, alpha: float) -> np.ndarray:
    """R_lin for the next step, R - alpha I_r^t R (Eq. (12)), from this step's
    residual, the low-rank fit I_r^t R = sum_i y_i t_i and the damping."""
    return R - alpha * fit


def linearity_indicator(norm_R_lin: float, norm_R: float) -> float:
    """beta = | ||R_lin|| / ||R|| - 1 | (Eq. (13)), with R_lin the residual the last
    step's low-rank model predicted for this step (Eq. (12))."""
    return abs(norm_R_lin / norm_R - 1.0)


def damping(norm_R: float, switched: bool = False, far: float = 0.1, near: float = 0.5,
            switch: float = 2.0) -> float:
    """alpha of the quasi-Newton step (Eq. (4)) by the schedule of Sec. III A:
    0.1 until ||R|| goes below 2.0, and 0.5 from then on.  `switched` tells
    whether an earlier SCF step already went below the threshold (the switch is
    made once and kept)."""
    return near if (switched or norm_R < switch) else far


def lrdma_event(has_history: bool, clear_pending: bool, beta, kept_s_rel, norm_R: float,
                s_tol: float = 0.3, beta_tol: float = 0.1, accumulate_below: float = 1.0) -> str:
    """The LRDMA decision of Sec. II B 1 with the gates of Sec. III A, in the
    order the text takes them: no history -> "fresh"; a clearing triggered at the
    last step (s_rel not reached) -> "CT"; beta > beta_tol -> "CL"; the kept
    approximation already fits R (kept_s_rel < s_tol) -> "reuse"; ||R|| not below
    accumulate_below -> "CR"; otherwise "accumulate"."""
    if not has_history:
        return "fresh"
    if clear_pending:
        return "CT"
    if beta > beta_tol:
        return "CL"
    if kept_s_rel < s_tol:
        return "reuse"
    if norm_R >= accumulate_below:
        return "CR"
    return "accumulate"


def effective_potential(V_ext: np.ndarray, rho: np.ndarray, grid: Grid, xc: bool = False):
    """V_eff[rho] = V_ext + V_H[rho] (Eq. (1)) with V_H = K_c applied to the total
    density; with xc also + V_xc,sigma of the LDA (lda_xc), one potential per
    channel.  rho: [nspin][nz][ny][nx] or [nz][ny][nx].  Returns [nz][ny][nx]
    without xc, [nspin][nz][ny][nx] with it."""
    rho = rho.reshape((-1,) + grid.shape)
    v = V_ext + hartree_kernel(rho.sum(axis=0), grid)
    if not xc:
        return v
    return v[None] + lda_xc(rho)[0]


def lowest_states(V: np.ndarray, grid: Grid, N: int):
    """The N lowest eigenpairs of H = -1/2 Lap_h + V by dense diagonalisation of
    the M x M matrix (tiny grids only).  Returns (eps [N], Psi [N][nz][ny][nx])."""
    M = grid.M
    Hd = hamiltonian_apply(np.eye(M).reshape((M,) + grid.shape), V, grid).reshape(M, M)
    w, Q = np.linalg.eigh(0.5 * (Hd + Hd.T))
    return w[:N], Q[:, :N].T.reshape((N,) + grid.shape).copy()


def scf_residual(rho: np.ndarray, V_ext: np.ndarray, grid: Grid, N: int, n_electrons: float,
                 kT: float, nspin: int = 1, xc: bool = False):
    """R[rho] = F[V_eff[rho]] - rho (Sec. II A, Sec. II D for two channels): the
    output density of the N lowest states of H[V_eff[rho]] in each channel minus
    the input.  Without the exchange-correlation term both channels see the same
    potential.  Returns (R [nspin][nz][ny][nx], Psi [nspin][N][...], eps [nspin][N])."""
    rho = rho.reshape((nspin,) + grid.shape)
    V = effective_potential(V_ext, rho, grid, xc)
    if not xc:
        V = np.stack([V] * nspin)
    states = [lowest_states(V[c], grid, N) for c in range(nspin)]
    eps = np.stack([e for e, _ in states])
    Psi = np.stack([p for _, p in states])
    rho_out, _ = density(Psi, eps, grid, n_electrons, kT, nspin)
    return rho_out - rho, Psi, eps


def lrdm_scf(rho0: np.ndarray, V_ext: np.ndarray, grid: Grid, N: int, n_electrons: float,
             kT: float, nspin: int = 1, s_tol: float = 0.3, r_max: int = 20,
             tol: float = 1e-9, max_iter: int = 50, xc: bool = False,
             alpha_switch: float = 2.0):
    """SCF by the damped quasi-Newton step rho <- rho - alpha P^lr_r R (Eq. (4),
    Sec. II B) with the directional derivatives of Eq. (7) from the subspace
    density response (K = K_c, plus the LDA kernel at rho with xc); alpha follows
    the schedule of Sec. III A (damping).  Returns (rho, [(||R||, rank, s_rel,
    alpha) per step])."""
    rho = rho0.reshape((nspin,) + grid.shape).copy()
    switched = False
    log = []
    for _ in range(max_iter):
        R, Psi, eps = scf_residual(rho, V_ext, grid, N, n_electrons, kT, nspin, xc)
        nR = np.sqrt(inner(R, R, grid))
        if nR < tol:
            log.append((nR, 0, 0.0, 0.0))
            break
        fxc = lda_xc(rho)[1] if xc else None

        def apply_t(u):
            return residual_derivative(Psi, eps, grid, n_electrons, kT, u[None], nspin,
                                       fxc)[0][0]

        drho, U, _, hist = lowrank_preconditioner(R, apply_t, grid, s_tol, r_max)
        switched = switched or nR < alpha_switch
        alpha = damping(nR, switched, switch=alpha_switch)
        rho = rho - alpha * drho
        log.append((nR, len(U), float(hist[-1]), alpha))
    return rho, log


def lrdma_scf(rho0: np.ndarray, V_ext: np.ndarray, grid: Grid, N: int, n_electrons: float,
              kT: float, nspin: int = 1, s_tol: float = 0.3, beta_tol: float = 0.1,
              r_iter_max: int = 5, accumulate_below: float = 1.0, r_max: int = 20,
              tol: float = 1e-9, max_iter: int = 50, xc: bool = False,
              alpha_switch: float = 2.0):
    """SCF with the accumulated low-rank step (LRDMA, Sec. II B 1).

    At each step, with R = R[rho]:
      * no history, or a clearing pending from the last step (CT): build afresh;
      * beta = |||R_lin|| / ||R|| - 1| > beta_tol: clear (CL) and build afresh;
      * else if the kept approximation fits R (s_rel < s_tol): use it as it is;
      * else if ||R|| >= accumulate_below: clear (CR) and build afresh (Sec. III A
        allows accumulation only while ||R|| < 1.0);
      * else accumulate up to r_iter_max new directions on the kept ones; if s_rel
        is still above s_tol, clear before the next step (CT).
    Building afresh is the LRDM step of Eqs. (8)-(10) (up to r_max directions);
    r_max also caps the accumulated rank (a full history is cleared, as CT).
    R_lin = R - alpha I_r^t R with I_r^t R = sum_i y_i t_i (Eq. (12)) is the
    residual this step's approximation and alpha predict for the next step.
    alpha follows the schedule of Sec. III A (damping), whose threshold (2.0) is
    not the accumulation gate (1.0).
    Returns (rho, log of (||R||, rank, added, event, s_rel, alpha, beta))."""
    rho = rho0.reshape((nspin,) + grid.shape).copy()
    switched = False
    U, T = [], []
    norm_R_lin = None
    clear_next = False
    log = []
    for _ in range(max_iter):
        R, Psi, eps = scf_residual(rho, V_ext, grid, N, n_electrons, kT, nspin, xc)
        nR = np.sqrt(inner(R, R, grid))
        if nR < tol:
            log.append((nR, len(U), 0, "done", 0.0, 0.0, None))
            break
        fxc = lda_xc(rho)[1] if xc else None

        def apply_t(u):
            return residual_derivative(Psi, eps, grid, n_electrons, kT, u[None], nspin,
                                       fxc)[0][0]

        beta = None if norm_R_lin is None else linearity_indicator(norm_R_lin, nR)
        if len(U) >= r_max:                          # no room to accumulate: start again
            clear_next = True
        kept_s_rel = np.inf
        if U and not clear_next and beta <= beta_tol:
            drho, U2, T2, kept_s_rel, added, fit = lowrank_accumulate(R, apply_t, grid, s_tol,
                                                                      U, T, 0)
        event = lrdma_event(bool(U), clear_next, beta, kept_s_rel, nR, s_tol, beta_tol,
                            accumulate_below)
        if event == "reuse":
            U, T, s_rel = list(U2), list(T2), kept_s_rel
        elif event == "accumulate":
            drho, U2, T2, s_rel, added, fit = lowrank_accumulate(
                R, apply_t, grid, s_tol, U, T, min(r_iter_max, r_max - len(U)))
            U, T = list(U2), list(T2)
            clear_next = s_rel >= s_tol
        if event in ("fresh", "CL", "CR", "CT"):
            drho, U2, T2, s_rel, added, fit = lowrank_accumulate(R, apply_t, grid, s_tol, [], [],
                                                                 r_max)
            U, T = list(U2), list(T2)
            clear_next = False
        switched = switched or nR < alpha_switch
        alpha = damping(nR, switched, switch=alpha_switch)
        rho = rho - alpha * drho
        R_lin = predicted_residual(R, fit, alpha)
        norm_R_lin = np.sqrt(inner(R_lin, R_lin, grid))
        log.append((nR, len(U), added if event != "reuse" else 0, event, s_rel, alpha, beta))
    return rho, log


# ---------------------------------------------------------------------------
# The paper's recursive Fermi-operator expansion (Eqs. (23)-(24))
# ---------------------------------------------------------------------------
def recursive_fermi_response(eps: np.ndarray, mu: float, kT: float, Hp: np.ndarray,
                             depth: int):
    """Response of the recursive expansion X_0 = 1/2 - 2^{-(T+2)} (D - mu)/kT,
    X_n = X_{n-1}^2 / (X_{n-1}^2 + (1 - X_{n-1})^2) along D + lam H' at fixed mu
    (Eqs. (23)-(24)), carried by first-order perturbation of each step:
        X_n + lam X_n' = (X^2 + lam (X X' + X' X)) (Y + lam Y')^{-1},
        Y = X^2 + (1 - X)^2,  Y' = 2 (X X' + X' X) - 2 X'  ... (first order).
    X stays diagonal, so the inverse of Y is a diagonal inversion.
    Returns (occupations diag(X_T), response matrix X_T')."""
    x = 0.5 - (2.0 ** (-(depth + 2))) * (np.asarray(eps) - mu) / kT
    xp = -(2.0 ** (-(depth + 2))) * Hp / kT
    for _ in range(depth):
        x2 = x * x
        y = x2 + (1.0 - x) ** 2
        # first-order pieces of X^2 and of Y = 2X^2 - 2X + 1 for diagonal X
        x2p = x[:, None] * xp + xp * x[None, :]
        yp = 2.0 * x2p - 2.0 * xp
        yinv = 1.0 / y
        # (A + lam A')(Y + lam Y')^{-1} = A Y^{-1} + lam (A' Y^{-1} - A Y^{-1} Y' Y^{-1})
        xp = x2p * yinv[None, :] - (x2 * yinv)[:, None] * yp * yinv[None, :]
        x = x2 * yinv
    return x, xp


def density_response_recursive(Psi: np.ndarray, eps: np.ndarray, grid: Grid,
                               n_electrons: float, kT: float, dV: np.ndarray, depth: int,
                               nspin: int = 1):
    """delta rho_k with the paper's recursive expansion of depth T in place of the
    exact Fermi-Dirac function (Eqs. (23)-(24)): the response of
    P_T(...P_0(D + lam H' - (mu + lam mu') I)) at lam = 0, i.e. the recursion's
    response to H' minus mu' times its response to the identity, with mu at the
    Fermi-Dirac electron count and mu' from the traceless condition (summed over
    both channels).  Shapes as for density_response; returns (drho, mu, dmu)."""
    Psi = Psi.reshape((nspin,) + Psi.shape[-4:])
    eps = np.asarray(eps, dtype=np.float64).reshape(nspin, -1)
    dV = dV.reshape((-1, nspin) + grid.shape)
    r = dV.shape[0]
    N = eps.shape[1]
    s = spin_factor(nspin)
    mu, _ = fermi_level(eps, n_electrons, kT, nspin)
    XI = [recursive_fermi_response(eps[c], mu, kT, np.eye(N), depth)[1] for c in range(nspin)]
    drho = np.empty_like(dV)
    dmu = np.empty(r)
    for k in range(r):
        XH = [recursive_fermi_response(eps[c], mu, kT,
                                       projected_perturbation(Psi[c], dV[k, c]), depth)[1]
              for c in range(nspin)]
        den = sum(np.trace(XI[c]) for c in range(nspin))
        dmu[k] = sum(np.trace(XH[c]) for c in range(nspin)) / den if abs(den) >= 1e-300 else 0.0
        for c in range(nspin):
            drho[k, c] = density_from_matrix(Psi[c], XH[c] - dmu[k] * XI[c], grid.dv, s)
    return drho, mu, dmu


# ---------------------------------------------------------------------------
# Adjoint of the subspace density response (vector-Jacobian product)
# ---------------------------------------------------------------------------
# The response delta rho = (s/dv) diag(Psi^T Gamma Psi), Gamma = F o H' - mu' diag(f')
# (Eq. (22)), H' = Psi diag(dV) Psi^T (Eq. (21)), mu' fixed by Tr Gamma = 0 and mu
# by the electron count (Eq. (1)), is differentiated here by hand.  With
# g = dL/d(delta rho):
#   A    = dL/dGamma = (s/dv) Psi diag(g) Psi^T
#   dH'  = dL/dH'    = F o A - nu diag(f'),  nu = sum f'_i A_ii / sum f'_i
#          (the same map as H' -> Gamma: the response is self-adjoint)
#   dL/ddV_p  = sum_ij Psi_ip dH'_ij Psi_jp
#   dL/dPsi   = 2 (s/dv) (Gamma Psi) o g + 2 (dH' Psi) o dV   (columns scaled)
#   dL/deps   through F (second divided differences), f' (f''), and mu(eps)
#             (dmu/deps_i = f'_i / sum f').
def fermi_derivatives(eps: np.ndarray, mu: float, kT: float):
    """d^k f / d eps^k for k = 1..4 at each eps, with a = f (1 - f):
    f' = -a/kT, f'' = a (1 - 2f)/kT^2, f''' = -a (1 - 6a)/kT^3,
    f'''' = a (1 - 2f)(1 - 12a)/kT^4 (a' = -(1 - 2f) a / kT)."""
    f, omf, _ = fermi_dirac(eps, mu, kT)
    a = f * omf
    d = omf - f                    # 1 - 2f without cancellation of f near 1/2
    return (-a / kT, a * d / kT ** 2, -a * (1.0 - 6.0 * a) / kT ** 3,
            a * d * (1.0 - 12.0 * a) / kT ** 4)


def second_divided_differences(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """D_ij = f[eps_i, eps_i, eps_j] = (F_ij - f'_i)/(eps_j - eps_i), with the limit
    f''_i / 2 at coincidence.  For |eps_j - eps_i| < 1e-3 kT the difference quotient
    would cancel; there the Taylor series about eps_i,
        f''/2 + f''' h/6 + f'''' h^2/24,   h = eps_j - eps_i,
    is used (next term ~ (h/kT)^3 relative)."""
    eps = np.asarray(eps, dtype=np.float64)
    F = divided_differences(eps, mu, kT)
    f1, f2, f3, f4 = fermi_derivatives(eps, mu, kT)
    h = eps[None, :] - eps[:, None]
    near = np.abs(h) < 1e-3 * kT
    D = np.empty_like(F)
    hs = np.where(near, 1.0, h)
    D[~near] = ((F - f1[:, None]) / hs)[~near]
    taylor = f2[:, None] / 2 + f3[:, None] * h / 6 + f4[:, None] * h * h / 24
    D[near] = taylor[near]
    return D


def density_response_vjp(Psi: np.ndarray, eps: np.ndarray, grid: Grid, n_electrons: float,
                         kT: float, dV: np.ndarray, g: np.ndarray, nspin: int = 1):
    """dL/ddV, dL/dPsi and dL/deps for L with dL/d(delta rho) = g, where delta rho =
    density_response(Psi, eps, grid, n_electrons, kT, dV, nspin).

    Psi [nspin][N][nz][ny][nx], eps [nspin][N], dV and g [r][nspin][nz][ny][nx].
    Returns (g_dV like dV, g_Psi like Psi, g_eps [nspin][N])."""
    Psi = Psi.reshape((nspin,) + Psi.shape[-4:])
    N = Psi.shape[1]
    eps = np.asarray(eps, dtype=np.float64).reshape(nspin, -1)
    dV = dV.reshape((-1, nspin) + grid.shape)
    g = g.reshape(dV.shape)
    r = dV.shape[0]
    s = spin_factor(nspin)
    c = s / grid.dv
    mu, _ = fermi_level(eps, n_electrons, kT, nspin)
    F = [divided_differences(eps[ch], mu, kT) for ch in range(nspin)]
    D = [second_divided_differences(eps[ch], mu, kT) for ch in range(nspin)]
    fd = [fermi_derivatives(eps[ch], mu, kT) for ch in range(nspin)]
    fp = [fd[ch][0] for ch in range(nspin)]
    S = float(sum(np.sum(x) for x in fp))
    P = [Psi[ch].reshape(N, -1) for ch in range(nspin)]          # N x M
    g_dV = np.zeros_like(dV)
    g_Psi = np.zeros((nspin, N, grid.M))
    Pm = [np.zeros((N, N)) for _ in range(nspin)]                # dL/dF
    q = [np.zeros(N) for _ in range(nspin)]                      # dL/df'
    for k in range(r):
        Hp = [projected_perturbation(Psi[ch], dV[k, ch]) for ch in range(nspin)]
        A = [c * projected_perturbation(Psi[ch], g[k, ch]) for ch in range(nspin)]
        dmu = fermi_shift(Hp, fp)
        nu = fermi_shift(A, fp)
        for ch in range(nspin):
            Gam = response_density_matrix(F[ch], Hp[ch], dmu, fp[ch])
            dH = response_density_matrix(F[ch], A[ch], nu, fp[ch])
            wv = dV[k, ch].reshape(-1)
            gv = g[k, ch].reshape(-1)
            g_dV[k, ch] = np.sum(P[ch] * (dH @ P[ch]), axis=0).reshape(grid.shape)
            g_Psi[ch] += 2.0 * c * (Gam @ P[ch]) * gv[None, :] + 2.0 * (dH @ P[ch]) * wv[None, :]
            Pm[ch] += A[ch] * Hp[ch]
            # dL/df'_i: the -mu' diag(f') term and mu' = sum f' H'_ii / sum f'
            q[ch] += -dmu * np.diag(A[ch]) - nu * (np.diag(Hp[ch]) - dmu)
    # eps with mu held fixed, then the chain through mu(eps)
    ge = np.stack([2.0 * np.sum(Pm[ch] * D[ch], axis=1) + q[ch] * fd[ch][1]
                   for ch in range(nspin)])
    dL_dmu = -float(np.sum(ge))
    if abs(S) >= 1e-300:
        ge = ge + np.stack(fp) / S * dL_dmu
    return g_dV, g_Psi.reshape(Psi.shape), ge


# ---------------------------------------------------------------------------
# Brillouin-zone sampling (Sec. II C, last paragraph, and its traceless
# condition integrated over the zone)
# ---------------------------------------------------------------------------
def bloch_hamiltonian_apply(Y: np.ndarray, V: np.ndarray, grid: Grid, kvec) -> np.ndarray:
    """H_k u for the cell-periodic part u of Bloch states e^{i k.x} u(x) with the
    7-point stencil of hamiltonian_apply: the link to the neighbour at +h_d
    carries the phase e^{i k_d h_d}, the link to -h_d its conjugate,
        (H_k u)_p = -1/2 sum_d (e^{i k_d h_d} u_{p+e_d} + e^{-i k_d h_d} u_{p-e_d}
                                - 2 u_p) / h_d^2 + V_p u_p.
    k = 0 is hamiltonian_apply.  Y: complex [..., nz, ny, nx]; kvec = (kx, ky, kz)."""
    Y = np.asarray(Y, dtype=np.complex128)
    lap = np.zeros_like(Y)
    for axis, hd, kd in ((-1, grid.h[0], kvec[0]), (-2, grid.h[1], kvec[1]),
                         (-3, grid.h[2], kvec[2])):
        ph = np.exp(1j * kd * hd)
        lap += (ph * np.roll(Y, -1, axis=axis) + np.conj(ph) * np.roll(Y, 1, axis=axis)
                - 2.0 * Y) / (hd * hd)
    return -0.5 * lap + V * Y


def chebyshev_filter_bloch(X: np.ndarray, V: np.ndarray, grid: Grid, kvec, degree: int,
                           a: float, b: float, a0: float) -> np.ndarray:
    """The scaled Chebyshev filter of chebyshev_filter with H_k in place of H, on a
    complex block (the ChFSI of each k-point's subspace, Sec. II C)."""
    return _chebyshev(np.asarray(X, dtype=np.complex128).copy(),
                      lambda Y: bloch_hamiltonian_apply(Y, V, grid, kvec), degree, a, b, a0)


def rayleigh_ritz_bloch(Y: np.ndarray, V: np.ndarray, grid: Grid, kvec):
    """rayleigh_ritz for H_k on a complex block: Householder QR, the Hermitian
    projected matrix and its eigenpairs.  Returns (eps [N], Psi_R complex [N][...])."""
    N = Y.shape[0]
    Psi_o, _ = np.linalg.qr(np.asarray(Y, dtype=np.complex128).reshape(N, -1).T)
    HPsi = bloch_hamiltonian_apply(Psi_o.T.reshape(Y.shape), V, grid, kvec).reshape(N, -1).T
    Hhat = Psi_o.conj().T @ HPsi
    Hhat = 0.5 * (Hhat + Hhat.conj().T)
    eps, Q = np.linalg.eigh(Hhat)
    return eps, (Psi_o @ Q).T.reshape(Y.shape).copy()


def lowest_bloch_states(V: np.ndarray, grid: Grid, kvec, N: int):
    """The N lowest eigenpairs of H_k by dense diagonalisation (tiny grids).
    Returns (eps [N], Psi complex [N][nz][ny][nx])."""
    M = grid.M
    Hd = bloch_hamiltonian_apply(np.eye(M, dtype=np.complex128).reshape((M,) + grid.shape), V,
                                 grid, kvec).reshape(M, M).T
    w, Q = np.linalg.eigh(0.5 * (Hd + Hd.conj().T))
    return w[:N], Q[:, :N].T.reshape((N,) + grid.shape).copy()


def fermi_level_bz(eps: np.ndarray, weights, n_electrons: float, kT: float, nspin: int = 1,
                   max_iter: int = 200):
    """mu solving s sum_sigma sum_k w_k sum_i f(eps_sigma,k,i, mu) = N_e (Eq. (1)
    with the zone average sum_k w_k, sum_k w_k = 1), by the bisection of
    fermi_level.  eps [nspin][nk][N].  Returns (mu, converged)."""
    w = np.asarray(weights, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64).reshape(nspin, len(w), -1)
    s = spin_factor(nspin)
    lo = float(eps.min()) - 50.0 * kT
    hi = float(eps.max()) + 50.0 * kT
    converged = False
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if hi - lo <= 2.0 * np.spacing(abs(mid)):
            converged = True
            break
        count = s * float(np.sum(w[None, :, None] * fermi_dirac(eps, mid, kT)[0]))
        if count > n_electrons:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi), converged


def projected_perturbation_complex(Psi: np.ndarray, dV: np.ndarray) -> np.ndarray:
    """H'_k = Psi_k^H diag(dV) Psi_k (Eq. (21) for a complex subspace); Psi [N][...]."""
    N = Psi.shape[0]
    P = Psi.reshape(N, -1).T                          # M x N
    return P.conj().T @ (dV.reshape(-1)[:, None] * P)


def density_from_matrix_complex(Psi: np.ndarray, Gamma: np.ndarray, dv: float,
                                s: float) -> np.ndarray:
    """(s/dv) diag(Psi Gamma Psi^H) with Psi the M x N matrix of the states as
    columns (real for Hermitian Gamma)."""
    N = Psi.shape[0]
    P = Psi.reshape(N, -1).T
    return ((s / dv) * np.real(np.sum((P @ Gamma) * P.conj(), axis=1))).reshape(Psi.shape[1:])


def density_response_bz(Psi: np.ndarray, eps: np.ndarray, weights, grid: Grid,
                        n_electrons: float, kT: float, dV: np.ndarray, nspin: int = 1):
    """delta rho for each perturbation dV_r with Brillouin-zone sampling (Sec. II C,
    last paragraph): each k-point's complex subspace responds as in Eq. (22),
        Gamma_k = F_k o H'_k - mu' diag(f'_k),
    with the common mu of the zone-averaged electron count and the common mu'
    of the zone-averaged traceless condition,
        mu' = sum_sigma sum_k w_k sum_i f'_ki H'_k,ii / sum_sigma sum_k w_k sum_i f'_ki,
    and delta rho = (s/dv) sum_k w_k diag(Psi_k Gamma_k Psi_k^H) per channel.
    Psi complex [nspin][nk][N][...], eps [nspin][nk][N], dV [r][nspin][...]
    (lattice-periodic, the same at every k).  Returns (drho [r][nspin][...], mu,
    dmu [r])."""
    w = np.asarray(weights, dtype=np.float64)
    nk = len(w)
    Psi = np.asarray(Psi).reshape((nspin, nk) + Psi.shape[-4:])
    eps = np.asarray(eps, dtype=np.float64).reshape(nspin, nk, -1)
    dV = dV.reshape((-1, nspin) + grid.shape)
    s = spin_factor(nspin)
    mu, _ = fermi_level_bz(eps, w, n_electrons, kT, nspin)
    fp = [[fermi_dirac(eps[c, k], mu, kT)[2] for k in range(nk)] for c in range(nspin)]
    Fm = [[divided_differences(eps[c, k], mu, kT) for k in range(nk)] for c in range(nspin)]
    r = dV.shape[0]
    drho = np.zeros_like(dV)
    dmu = np.empty(r)
    for q in range(r):
        Hp = [[projected_perturbation_complex(Psi[c, k], dV[q, c]) for k in range(nk)]
              for c in range(nspin)]
        num = sum(w[k] * np.sum(fp[c][k] * np.real(np.diag(Hp[c][k])))
                  for c in range(nspin) for k in range(nk))
        den = sum(w[k] * np.sum(fp[c][k]) for c in range(nspin) for k in range(nk))
        dmu[q] = 0.0 if abs(den) < 1e-300 else num / den
        for c in range(nspin):
            for k in range(nk):
                G = Fm[c][k] * Hp[c][k] - dmu[q] * np.diag(fp[c][k])
                drho[q, c] += w[k] * density_from_matrix_complex(Psi[c, k], G, grid.dv, s)
    return drho, mu, dmu

