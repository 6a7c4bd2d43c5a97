"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
notice each one: the pins have teeth."""
import numpy as np
import pytest

import oracle
import oracle.lrdm_oracle as L
from tests import pins as P


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(L, name, fn)
    monkeypatch.setattr(oracle, name, fn)


def _fails(check):
    try:
        return not check()
    except Exception:
        return True


ORIG = {k: getattr(L, k) for k in dir(L) if not k.startswith("__")}


def m_drop_dmu(mp):
    _patch(mp, "fermi_shift", lambda Hp, fp: 0.0)
    return lambda: P.invariants()["integral"] < 1e-13 and P.pin_response_subspace_fd() < 1e-8


def m_flip_F(mp):
    _patch(mp, "divided_differences", lambda e, mu, kT: -ORIG["divided_differences"](e, mu, kT))
    return lambda: P.invariants()["nsd"] == 0.0


def m_shift_F_index(mp):
    _patch(mp, "divided_differences", lambda e, mu, kT: ORIG["divided_differences"](np.roll(e, 1), mu, kT))
    return lambda: P.pin_response_subspace_fd() < 1e-8


def m_spin_factor(mp):
    _patch(mp, "spin_factor", lambda nspin: 1.0)
    return lambda: P.pin_response_full_space() < 1e-8


def m_laplacian_half(mp):
    def bad(Y, V, grid):
        return ORIG["hamiltonian_apply"](Y, V, grid) * 1.0 + 0.5 * (ORIG["hamiltonian_apply"](Y, 0 * V, grid))
    _patch(mp, "hamiltonian_apply", bad)
    return lambda: P.pin_plane_wave() < 1e-13


def m_cheb_sigma_sign(mp):
    def bad(X, V, grid, degree, a, b, a0):
        e, c0 = (b - a) / 2, (b + a) / 2
        s1 = e / (a0 - c0)
        yp = X.copy()
        y = (s1 / e) * (L.hamiltonian_apply(yp, V, grid) - c0 * yp)
        s = s1
        for _ in range(2, degree + 1):
            sn = 1.0 / (2.0 / s1 + s)
            yn = (2 * sn / e) * (L.hamiltonian_apply(y, V, grid) - c0 * y) - s * sn * yp
            yp, y, s = y, yn, sn
        return y
    _patch(mp, "chebyshev_filter", bad)
    return lambda: P.pin_filter_polynomial() < 1e-11


def m_hartree_no_4pi(mp):
    _patch(mp, "hartree_kernel", lambda u, g: ORIG["hartree_kernel"](u, g) / (4 * np.pi))
    return lambda: P.pin_hartree_plane_wave() < 1e-12


def m_projection_layout(mp):
    def bad(Psi, dV):
        N = Psi.shape[0]
        Pm = Psi.reshape(-1, N)                      # wrong layout: M x N read from N x M data
        return Pm.T @ (dV.reshape(-1)[:, None] * Pm)
    _patch(mp, "projected_perturbation", bad)
    return lambda: P.pin_response_subspace_fd() < 1e-8


def m_density_no_dv(mp):
    _patch(mp, "density_from_matrix", lambda Psi, G, dv, s: ORIG["density_from_matrix"](Psi, G, 1.0, s))
    return lambda: P.pin_response_full_space() < 1e-8


def m_rr_no_rotation(mp):
    def bad(Y, V, grid):
        N = Y.shape[0]
        Q, _ = np.linalg.qr(Y.reshape(N, -1).T)
        HQ = L.hamiltonian_apply(Q.T.reshape(Y.shape), V, grid).reshape(N, -1).T
        eps = np.linalg.eigvalsh(Q.T @ HQ)
        return eps, Q.T.reshape(Y.shape)
    _patch(mp, "rayleigh_ritz", bad)
    return lambda: P.pin_rr_generalized() < 1e-11


def m_bisection_direction(mp):
    def bad(eps, ne, kT, nspin=1, max_iter=200):
        eps = np.asarray(eps).reshape(nspin, -1)
        s = L.spin_factor(nspin)
        lo, hi = eps.min() - 50 * kT, eps.max() + 50 * kT
        for _ in range(max_iter):
            mid = 0.5 * (lo + hi)
            if s * np.sum(L.fermi_dirac(eps, mid, kT)[0]) > ne:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi), True
    _patch(mp, "fermi_level", bad)
    return lambda: P.pin_fermi_level() < 1e-12


def m_spin_channel_potential(mp):
    def bad(Psi, eps, grid, ne, kT, u, nspin=1):
        u = u.reshape((-1, nspin) + grid.shape)
        dV = np.stack([[L.hartree_kernel(u[k, c], grid) for c in range(nspin)] for k in range(u.shape[0])])
        drho, mu, dmu = L.density_response(Psi, eps, grid, ne, kT, dV, nspin)
        return drho - u, mu, dmu
    _patch(mp, "residual_derivative", bad)
    return lambda: P.pin_residual_derivative_spin() < 1e-14


def m_fermi_omf_subtraction_sign(mp):
    def bad(eps, mu, kT):
        f, omf, fp = ORIG["fermi_dirac"](eps, mu, kT)
        return f, omf, f * omf / kT                  # wrong sign of f'
    _patch(mp, "fermi_dirac", bad)
    return lambda: P.pin_divided_differences_decimal() < 1e-13 and P.pin_response_subspace_fd() < 1e-8


def _bad_lowrank(first=None, gs_sign=-1.0, use_solve=True):
    """The low-rank step with one planted change."""
    def bad(R, apply_t, grid, s_tol, r_max):
        nR = np.sqrt(L.inner(R, R, grid))
        U = [(first(R, apply_t) if first else R) / nR]
        U[0] = U[0] / np.sqrt(L.inner(U[0], U[0], grid))
        T, hist = [], []
        while True:
            T.append(apply_t(U[-1]))
            r = len(T)
            S = np.array([[L.inner(T[i], T[j], grid) for j in range(r)] for i in range(r)])
            c = np.array([L.inner(T[j], R, grid) for j in range(r)])
            y = np.linalg.solve(S, c) if use_solve else c
            fit = sum(y[i] * T[i] for i in range(r))
            hist.append(np.sqrt(L.inner(fit - R, fit - R, grid)) / nR)
            if hist[-1] < s_tol or r == r_max:
                break
            u = T[-1]
            u = u + gs_sign * sum(L.inner(u, U[k], grid) * U[k] for k in range(r))
            U.append(u / np.sqrt(L.inner(u, u, grid)))
        return sum(y[i] * U[i] for i in range(r)), np.array(U), np.array(T), np.array(hist)
    return bad


def m_lowrank_gs_sign(mp):
    _patch(mp, "lowrank_preconditioner", _bad_lowrank(gs_sign=+1.0))
    return lambda: P.pin_lowrank_krylov_lstsq() < 1e-11 and P.pin_lowrank_directions() < 1e-12


def m_lowrank_no_S_inverse(mp):
    _patch(mp, "lowrank_preconditioner", _bad_lowrank(use_solve=False))
    return lambda: P.pin_lowrank_krylov_lstsq() < 1e-11


def m_lowrank_first_direction(mp):
    _patch(mp, "lowrank_preconditioner", _bad_lowrank(first=lambda R, t: t(R)))
    return lambda: P.pin_lowrank_krylov_lstsq() < 1e-11


def m_hartree_sign_in_scf(mp):
    def bad(V_ext, rho, grid):
        return V_ext - L.hartree_kernel(rho.reshape((-1,) + grid.shape).sum(axis=0), grid)
    _patch(mp, "effective_potential", bad)
    return lambda: P.pin_scf_derivative_fd(1) < 1e-9



def m_recursion_drop_denominator_term(mp):
    def bad(eps, mu, kT, Hp, depth):
        x = 0.5 - (2.0 ** (-(depth + 2))) * (np.asarray(eps) - mu) / kT
        xp = -(2.0 ** (-(depth + 2))) * Hp / kT
        for _ in range(depth):
            x2 = x * x
            y = x2 + (1.0 - x) ** 2
            x2p = x[:, None] * xp + xp * x[None, :]
            xp = x2p / y[None, :]                    # the Y' term dropped
            x = x2 / y
        return x, xp
    _patch(mp, "recursive_fermi_response", bad)
    return lambda: P.pin_recursive_response_fd() < 1e-9



def m_accumulate_first_direction_not_orthogonalised(mp):
    orig = ORIG["lowrank_accumulate"]

    def bad(R, apply_t, grid, s_tol, U_prev, T_prev, r_add_max):
        if not U_prev:
            return orig(R, apply_t, grid, s_tol, U_prev, T_prev, r_add_max)
        # the history is fitted, but the new directions ignore it
        d, U, T, s, a, f = orig(R, apply_t, grid, s_tol, [], [], r_add_max)
        U = np.concatenate([np.array(U_prev), U])
        T = np.concatenate([np.array(T_prev), T])
        return d, U, T, s, a, f
    _patch(mp, "lowrank_accumulate", bad)
    return lambda: P.pin_accumulate_union_lstsq() < 1e-11


def m_predicted_residual_sign(mp):
    _patch(mp, "predicted_residual", lambda R, fit, alpha: R + alpha * fit)
    return lambda: P.pin_linear_prediction() < 1e-12



def m_pz81_constant(mp):
    bad = {k: dict(v) for k, v in L.PZ81.items()}
    bad["U"]["gamma"] = -0.1523
    mp.setattr(L, "PZ81", bad)
    return lambda: P.pin_pz81_continuity() < 2e-3


def m_residual_derivative_drops_xc(mp):
    orig = ORIG["residual_derivative"]
    _patch(mp, "residual_derivative",
           lambda Psi, eps, grid, ne, kT, u, nspin=1, fxc=None: orig(Psi, eps, grid, ne, kT, u, nspin))
    return lambda: P.pin_scf_derivative_fd_xc(1) < 1e-9


def m_damping_one_threshold(mp):
    """The schedule's switch merged with the accumulation gate at 1.0."""
    _patch(mp, "damping", lambda nR, switched=False, far=0.1, near=0.5, switch=2.0:
           ORIG["damping"](nR, switched, far, near, 1.0))
    return lambda: P.pin_damping_schedule()


def m_lrdma_gate_at_alpha_switch(mp):
    """Accumulation allowed below the damping switch (2.0) instead of below 1.0."""
    orig = ORIG["lrdma_event"]
    _patch(mp, "lrdma_event", lambda *a, **kw: orig(*a, **{**kw, "accumulate_below": 2.0}))
    return lambda: P.pin_lrdma_gates()


def m_bloch_phase_sign(mp):
    """The Bloch phase on the wrong link (H_{-k} in place of H_k)."""
    orig = ORIG["bloch_hamiltonian_apply"]
    _patch(mp, "bloch_hamiltonian_apply",
           lambda Y, V, grid, k: orig(Y, V, grid, tuple(-x for x in k)))
    return lambda: P.pin_bloch_plane_wave() < 1e-13


def m_bz_projection_without_conjugate(mp):
    """Psi^T dV Psi in place of Psi^H dV Psi for the complex subspaces."""
    def bad(Psi, dV):
        N = Psi.shape[0]
        Pm = Psi.reshape(N, -1).T
        return Pm.T @ (dV.reshape(-1)[:, None] * Pm)
    _patch(mp, "projected_perturbation_complex", bad)
    return lambda: P.pin_bz_subspace_fd(1) < 1e-9


def m_bz_count_without_weights(mp):
    """The zone-averaged electron count without the k-point weights."""
    orig = ORIG["fermi_level_bz"]
    _patch(mp, "fermi_level_bz",
           lambda eps, w, ne, kT, nspin=1, max_iter=200: orig(eps, [1.0 / len(w)] * len(w), ne, kT,
                                                                nspin, max_iter))
    return lambda: P.pin_bz_subspace_fd(1) < 1e-9


MUTANTS = [m_drop_dmu, m_flip_F, m_shift_F_index, m_spin_factor, m_laplacian_half,
           m_cheb_sigma_sign, m_hartree_no_4pi, m_projection_layout, m_density_no_dv,
           m_rr_no_rotation, m_bisection_direction, m_spin_channel_potential,
           m_fermi_omf_subtraction_sign, m_lowrank_gs_sign, m_lowrank_no_S_inverse,
           m_lowrank_first_direction, m_hartree_sign_in_scf,
           m_recursion_drop_denominator_term, m_accumulate_first_direction_not_orthogonalised,
           m_predicted_residual_sign, m_pz81_constant, m_residual_derivative_drops_xc,
           m_damping_one_threshold, m_lrdma_gate_at_alpha_switch, m_bloch_phase_sign,
           m_bz_projection_without_conjugate, m_bz_count_without_weights]


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m.__name__ for m in MUTANTS])
def test_planted_mistake_is_caught(mutant, monkeypatch):
    check = mutant(monkeypatch)
    assert _fails(check), f"pins did not notice {mutant.__name__}"
