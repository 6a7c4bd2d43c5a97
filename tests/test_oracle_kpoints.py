"""Pins of the oracle's Brillouin-zone sampling (Sec. II C, last paragraph): the
Bloch Hamiltonian against plane waves, a hop-by-hop assembly and the folded
spectrum of a doubled cell; the zone-sampled response against the doubled cell's
dense-diagonalisation derivative, a Richardson difference of the zone-sampled
subspace density, the real path at k = 0, and its invariants."""
import numpy as np
import pytest

import oracle as O
from tests import pins as P


def test_bloch_plane_wave():
    assert P.pin_bloch_plane_wave() < 1e-13


def test_bloch_dense_matrix():
    assert P.pin_bloch_dense() < 1e-14


def test_bloch_supercell_spectrum():
    assert P.pin_bloch_supercell_spectrum() < 1e-12


def test_bz_response_is_the_doubled_cell_response():
    assert P.pin_bz_supercell_response() < 1e-8


@pytest.mark.parametrize("nspin", [1, 2])
def test_bz_response_is_the_subspace_derivative(nspin):
    assert P.pin_bz_subspace_fd(nspin) < 1e-9


def test_bz_gamma_point_is_the_real_path():
    assert P.pin_bz_gamma_is_the_real_path() < 1e-13


@pytest.mark.parametrize("nspin", [1, 2])
def test_bz_invariants(nspin):
    inv = P.bz_invariants(nspin)
    assert inv["integral"] < 1e-12 and inv["symmetry"] < 1e-12 and inv["nsd"] <= 1e-14


def test_bz_time_reversal():
    assert P.pin_bz_time_reversal() < 1e-13


def test_bloch_filter_and_rayleigh_ritz_reach_the_lowest_states():
    """ChFSI with H_k (filter and Rayleigh-Ritz passes) converges to the lowest
    eigenpairs of H_k found by dense diagonalisation."""
    g = O.Grid((5, 4, 4), (3.0, 2.5, 2.5))
    V = P.small_wells(g.n, g.L, 35)
    k = (0.3, -0.5, 0.2)
    N = 10
    e_ref, _ = O.lowest_bloch_states(V, g, k, 14)
    X = np.random.default_rng(5).standard_normal((14,) + g.shape) + 0j
    b = sum(2.0 / hd ** 2 for hd in g.h) + float(V.max())
    a, a0 = float(V.min()) + 0.25 * (b - float(V.min())), float(V.min()) - 0.1
    for _ in range(12):
        eps, X = O.rayleigh_ritz_bloch(O.chebyshev_filter_bloch(X, V, g, k, 12, a, b, a0), V, g, k)
        a, a0 = float(eps[-1]), float(eps[0]) - 0.1
    assert np.max(np.abs(eps[:N] - e_ref[:N])) < 1e-9
