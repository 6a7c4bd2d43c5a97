"""The oracle against closed forms, dense diagonalisation, finite differences,
decimal arithmetic and invariants (CPU only)."""
import pytest

from tests import pins as P


def test_stencil_plane_wave_closed_form():
    assert P.pin_plane_wave() < 1e-13


def test_stencil_matches_dense_matrix():
    assert P.pin_dense_stencil() < 1e-13


def test_filter_equals_chebyshev_polynomial_of_H():
    assert P.pin_filter_polynomial() < 1e-11


def test_filter_scalar_identity_on_eigenvector():
    assert P.pin_filter_scalar_identity() < 1e-9


def test_chfsi_reaches_exact_lowest_subspace():
    ritz_err, sin_max = P.pin_chfsi_exact_subspace()
    assert ritz_err < 1e-10
    assert sin_max < 1e-6


def test_rayleigh_ritz_exact_on_eigenvectors():
    assert P.pin_rr_exact_eigenvectors() < 1e-12


def test_rayleigh_ritz_matches_generalized_eigenproblem():
    assert P.pin_rr_generalized() < 1e-11


def test_fermi_level_counts_electrons():
    assert P.pin_fermi_level() < 1e-12


def test_fermi_level_in_gap():
    assert P.pin_fermi_gap() == 0.0


def test_divided_differences_50_digit_decimal():
    assert P.pin_divided_differences_decimal() < 1e-13


def test_divided_differences_plain_quotient_symmetric_nonpositive():
    assert P.pin_divided_differences_naive() < 1e-12


@pytest.mark.parametrize("nspin", [1, 2])
def test_response_subspace_richardson_fd(nspin):
    assert P.pin_response_subspace_fd(nspin) < 1e-8


def test_response_full_space_equals_dense_fd():
    assert P.pin_response_full_space() < 1e-8


def test_response_invariants():
    inv = P.invariants()
    assert inv["integral"] < 1e-13
    assert inv["symmetry"] < 1e-11
    assert inv["nsd"] == 0.0
    assert inv["constant"] < 1e-12
    assert inv["linearity"] < 1e-12
    assert inv["degenerate_rotation"] < 1e-12


def test_response_discrete_lindhard():
    assert P.pin_lindhard() < 1e-11


def test_hartree_plane_wave_multiplier():
    assert P.pin_hartree_plane_wave() < 1e-12


def test_hartree_inverts_stencil_laplacian():
    assert P.pin_hartree_poisson() < 1e-12


def test_residual_derivative_spin_pairs():
    assert P.pin_residual_derivative_spin() < 1e-14


def test_recursive_fermi_expansion_converges_to_divided_differences():
    errs = P.recursion_errors()
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-7


def test_recursive_expansion_response_matches_full_matrix_fd():
    """First-order perturbation of the recursion (Eqs. (23)-(24)) against central
    differences of the recursion run on full perturbed matrices."""
    assert P.pin_recursive_response_fd() < 1e-9


def test_recursive_density_response_traceless_and_convergent():
    integral, errs = P.pin_recursive_density_response()
    assert integral < 1e-13
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-9 and errs[3] < 1e-8
