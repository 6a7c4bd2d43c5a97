"""Pins of the oracle's low-rank step (Sec. II B, Eqs. (4), (7)-(10)) and of the
model SCF map it preconditions (Sec. II A)."""
import numpy as np
import pytest

import oracle as O
from tests import pins as P


def test_lowrank_step_is_krylov_least_squares():
    assert P.pin_lowrank_krylov_lstsq() < 1e-11


def test_lowrank_full_rank_is_newton_step():
    assert P.pin_lowrank_full_rank_newton() < 1e-11


def test_lowrank_directions_orthonormal_and_adaptive_rank():
    assert P.pin_lowrank_directions() < 1e-12


def test_lowrank_zero_residual():
    g = O.Grid((2, 2, 2), (1.0, 1.0, 1.0))
    drho, U, T, hist = O.lowrank_preconditioner(np.zeros(g.shape), lambda u: -u, g, 0.3, 5)
    assert not drho.any() and len(U) == 0 and len(hist) == 0


def test_lowrank_spin_pair_is_direct_sum():
    """A spin pair behaves as one vector of twice the length (Sec. II D)."""
    g, J, R, _ = P._linear_residual(n=(3, 2, 2), L=(1.5, 1.0, 1.0), seed=9)
    M = g.M // 2
    pair = R.reshape(2, M)

    def t_pair(u):
        return (J @ u.ravel()).reshape(u.shape)
    g2 = O.Grid((3, 2, 1), (1.5, 1.0, 0.5))                # same dv, half the points
    d2, _, _, h2 = O.lowrank_preconditioner(pair, t_pair, g2, 0.0, 4)
    d1, _, _, h1 = O.lowrank_preconditioner(R, t_pair, g, 0.0, 4)
    assert np.allclose(d2.ravel(), d1.ravel(), rtol=0, atol=1e-13)
    assert np.allclose(h1, h2, rtol=1e-13)


def test_damping_schedule_is_the_papers():
    """Sec. III A: alpha = 0.1 until ||R|| goes below 2.0, then 0.5 from that step
    on (values from the golden fixture, typed in from the paper)."""
    assert P.pin_damping_schedule()


def test_lrdma_gates_are_the_papers():
    """Sec. II B 1 with the gates of Sec. III A: accumulation only while ||R|| <
    1.0 (a CR clearing at 1.5, where alpha is already 0.5), beta_tol 0.1."""
    assert P.pin_lrdma_gates()


@pytest.mark.parametrize("nspin", [1, 2])
def test_residual_derivative_is_scf_residual_derivative(nspin):
    assert P.pin_scf_derivative_fd(nspin) < 1e-9


def test_lrdm_scf_reaches_the_mixing_fixed_point():
    diff, lrdm_steps, mix_steps, count, r_lrdm, r_mix = P.scf_fixed_points()
    assert r_lrdm < 1e-10 and r_mix < 1e-10
    assert diff < 1e-9
    assert count < 1e-12
    assert lrdm_steps < mix_steps / 3


def test_accumulated_step_is_least_squares_over_all_directions():
    assert P.pin_accumulate_union_lstsq() < 1e-11


def test_accumulated_step_without_history_is_the_lrdm_step():
    assert P.pin_accumulate_empty_history() < 1e-12


def test_linear_prediction_and_indicator():
    assert P.pin_linear_prediction() < 1e-12


def test_linearity_indicator_definition():
    assert O.linearity_indicator(1.2, 1.0) == pytest.approx(0.2)
    assert O.linearity_indicator(0.9, 1.0) == pytest.approx(0.1)


def test_lrdma_reaches_lrdm_fixed_point_with_fewer_directions():
    diff, dirs_a, dirs_l, events, final = P.lrdma_vs_lrdm()
    assert final < 1e-9 and diff < 1e-8
    assert dirs_a < dirs_l
    assert "accumulate" in events and "reuse" in events


def test_pz81_branches_join_at_rs_1():
    assert P.pin_pz81_continuity() < 2e-3


def test_lda_exchange_is_the_uniform_gas_value():
    assert P.pin_lda_exchange_uniform_gas() < 1e-14


def test_lda_potential_and_kernel_are_the_derivatives():
    assert P.pin_lda_derivatives_fd() < 1e-7


def test_lda_zero_below_density_threshold():
    V, f = O.lda_xc(np.array([[1e-13, 0.1], [0.2, 0.1]]))
    assert (V[:, 0] == 0).all() and (f[:, :, 0] == 0).all() and (V[:, 1] != 0).all()


@pytest.mark.parametrize("nspin", [1, 2])
def test_residual_derivative_with_lda_is_scf_residual_derivative(nspin):
    assert P.pin_scf_derivative_fd_xc(nspin) < 1e-9
