"""Plain FP64 CPU oracle for the LRDM density-response hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs this code; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP path: it is written directly from the paper (Das & Gavini, "Accelerating
SCF iterations in Kohn-Sham DFT using a low rank approximation of the
dielectric matrix"), in NumPy, double precision, with no blocking or fusion.

Every function is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``
against something other than itself (closed forms, dense diagonalisation,
finite differences, 50-digit decimal arithmetic, invariants).
"""
from .lrdm_oracle import (  # noqa: F401
    Grid,
    hamiltonian_apply,
    chebyshev_filter,
    rayleigh_ritz,
    fermi_dirac,
    fermi_level,
    divided_differences,
    projected_perturbation,
    fermi_shift,
    response_density_matrix,
    density_from_matrix,
    density,
    density_response,
    hartree_kernel,
    residual_derivative,
    spin_factor,
    recursive_fermi_response,
    density_response_recursive,
    fermi_derivatives,
    second_divided_differences,
    density_response_vjp,
    inner,
    lowrank_preconditioner,
    damping,
    effective_potential,
    lowest_states,
    scf_residual,
    lrdm_scf,
    lowrank_accumulate,
    linearity_indicator,
    predicted_residual,
    lrdma_scf,
    lrdma_event,
    bloch_hamiltonian_apply,
    chebyshev_filter_bloch,
    rayleigh_ritz_bloch,
    lowest_bloch_states,
    fermi_level_bz,
    projected_perturbation_complex,
    density_from_matrix_complex,
    density_response_bz,
    lda_energy_density,
    lda_xc,
    pz81_eps_c,
)
