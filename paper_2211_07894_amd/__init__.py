"""MI355X-native hot path of the LRDM preconditioner (Das & Gavini): ChFSI
filter, Rayleigh-Ritz, subspace density response and residual derivative as
hand-written HIP kernels behind the C ABI of include/lrdm.h.

The Python layer only marshals torch device tensors into that ABI; see
``paper_2211_07894_amd.lrdm``.
"""
from .lrdm import (  # noqa: F401
    Grid,
    Occupation,
    LrdmError,
    library,
    context,
    hamiltonian_apply,
    fermi_occupations,
    projected_perturbation,
    hartree_kernel,
    chfsi_filter,
    subspace_rayleigh_ritz,
    density_response,
    density_response_bz,
    bloch_hamiltonian_apply,
    chfsi_filter_bloch,
    subspace_rayleigh_ritz_bloch,
    residual_derivative,
    density_response_backward,
    density_response_batched,
    DensityResponse,
    LowRankParams,
    density,
    effective_potential,
    lowrank_step,
    lda_xc,
    autotune,
)
from .scf import lrdm_scf, lrdma_scf  # noqa: F401,E402
