"""Model SCF driven by the LRDM step (Sec. II A-C): rho -> V_eff[rho] ->
ChFSI (filter + Rayleigh-Ritz) -> R[rho] = F[V_eff[rho]] - rho -> the low-rank
quasi-Newton update rho <- rho - alpha P^lr_r R.

Every step runs in the library's kernels (lrdm_effective_potential,
chfsi_filter, subspace_rayleigh_ritz, lrdm_density, lrdm_lowrank_step); this
module only holds the buffers and reads back the few scalars the loop decides
on (the potential's range for the filter's upper bound, the extreme Ritz values
for its other bounds, and the step's ||R||, rank and s_rel).
"""
from __future__ import annotations

import torch

from .lrdm import (Grid, LowRankParams, Occupation, chfsi_filter, density, effective_potential,
                   lowrank_step, subspace_rayleigh_ritz)


def lrdm_scf(grid: Grid, V_ext, X, occ: Occupation, degree: int, prec: str = "fp64",
             params: LowRankParams = LowRankParams(), rho0=None, tol: float = 1e-8,
             max_iter: int = 50, first_passes: int = 4):
    """Solve R[rho] = 0 for the model V_eff = V_ext + V_H[rho] (one channel).

    X [N][nz][ny][nx] is the starting block (double for fp64, float otherwise);
    it and one buffer like it alternate as filter input and output.  Each SCF step applies one
    Chebyshev filter of the given degree followed by Rayleigh-Ritz (the first
    step applies first_passes of them, degree 10 for the first), with the
    filter's bounds b = sum_d 2/h_d^2 + max V_eff (an upper bound of the
    spectrum), a = the largest and a0 = the smallest Ritz value minus 0.1.
    rho0 defaults to the uniform density N_e / volume.  Stops once the step
    reports ||R|| < tol (rho then carries that step's update too).

    Returns (rho [1][nz][ny][nx], eps [N], log, Psi): log holds one dict per
    step with norm_R, rank, s_rel and alpha; Psi [N][nz][ny][nx] is the last
    block of Ritz vectors (one of the two alternating buffers)."""
    if occ.nspin != 1:
        raise ValueError("the model SCF has no exchange-correlation term and runs one channel")
    dev = X.device
    N = X.shape[0]
    hx, hy, hz = (grid.L[d] / grid.n[d] for d in range(3))
    lap_top = 2.0 / hx ** 2 + 2.0 / hy ** 2 + 2.0 / hz ** 2
    vol = grid.L[0] * grid.L[1] * grid.L[2]
    shape = (1,) + grid.shape
    if rho0 is None:
        rho = torch.full(shape, occ.n_electrons / vol, dtype=torch.float64, device=dev)
    else:
        rho = rho0.reshape(shape).clone()
    V = torch.empty(grid.shape, dtype=torch.float64, device=dev)
    vr = torch.empty(2, dtype=torch.float64, device=dev)
    R = torch.empty(shape, dtype=torch.float64, device=dev)
    U = torch.empty((params.r_max,) + shape, dtype=torch.float64, device=dev)
    T = torch.empty_like(U)
    drho = torch.empty(shape, dtype=torch.float64, device=dev)
    eps = torch.empty(N, dtype=torch.float64, device=dev)
    Y = torch.empty_like(X)
    a = a0 = None
    log = []
    for it in range(max_iter):
        effective_potential(grid, V_ext, rho, out=V, vrange=vr)
        vmin, vmax = vr.tolist()
        b = lap_top + vmax
        if a is None:
            a0 = vmin - 0.1
            a = a0 + 0.25 * (b - a0)
        passes = first_passes if it == 0 else 1
        for p in range(passes):
            chfsi_filter(grid, V, X, 10 if (it == 0 and p == 0) else degree, a, b, a0, prec=prec,
                         out=Y)
            subspace_rayleigh_ritz(grid, V, Y, prec=prec, eps=eps)
            X, Y = Y, X
            lo, hi = eps[0].item(), eps[-1].item()
            a, a0 = hi, lo - 0.1
        density(grid, X, eps, occ, prec=prec, rho_in=rho, out=R)
        _, _, _, info = lowrank_step(grid, X, eps, occ, R, params, prec=prec, rho=rho, U=U, T=T,
                                     drho=drho)
        log.append(info)
        if info["norm_R"] < tol:
            break
    return rho, eps, log, X
