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


def lrdma_scf(grid: Grid, V_ext, X, occ: Occupation, degree: int, prec: str = "fp64",
              params: LowRankParams = LowRankParams(), beta_tol: float = 0.1, r_iter_max: int = 5,
              rho0=None, tol: float = 1e-8, max_iter: int = 50, first_passes: int = 4):
    """The model SCF of lrdm_scf with the accumulated low-rank step (LRDMA,
    Sec. II B 1).  At each SCF step, with R = R[rho]:
      * no kept directions, or a clearing pending (CT): build afresh;
      * beta = | ||R_lin|| / ||R|| - 1 | > beta_tol (Eq. (13)): clear (CL), afresh;
      * else if the kept directions fit R to s_rel < s_tol: reuse them;
      * else if ||R|| > r_switch: clear (CR), afresh;
      * else add at most r_iter_max directions to the kept ones; if s_rel stays
        at or above s_tol, clear before the next step (CT).
    Building afresh is the LRDM step (up to params.r_max directions); a full
    history (params.r_max kept) is cleared as CT.  R_lin is the residual the
    last step's approximation predicted (Eq. (12)), returned by the step.

    Returns (rho, eps, log, Psi): log holds one dict per step with norm_R, rank
    (directions in use), added, event, s_rel, alpha and beta."""
    if occ.nspin != 1:
        raise ValueError("the model SCF has no exchange-correlation term and runs one channel")
    dev = X.device
    N = X.shape[0]
    hx, hy, hz = (grid.L[d] / grid.n[d] for d in range(3))
    lap_top = 2.0 / hx ** 2 + 2.0 / hy ** 2 + 2.0 / hz ** 2
    vol = grid.L[0] * grid.L[1] * grid.L[2]
    shape = (1,) + grid.shape
    rho = (torch.full(shape, occ.n_electrons / vol, dtype=torch.float64, device=dev)
           if rho0 is None else rho0.reshape(shape).clone())
    V = torch.empty(grid.shape, dtype=torch.float64, device=dev)
    vr = torch.empty(2, dtype=torch.float64, device=dev)
    R = torch.empty(shape, dtype=torch.float64, device=dev)
    U = torch.empty((params.r_max,) + shape, dtype=torch.float64, device=dev)
    T = torch.empty_like(U)
    drho = torch.empty(shape, dtype=torch.float64, device=dev)
    eps = torch.empty(N, dtype=torch.float64, device=dev)
    Y = torch.empty_like(X)
    a = a0 = None
    kept = 0
    norm_R_lin = None
    clear_next = False
    log = []

    def step(r_keep, r_add_max, update):
        p = LowRankParams(s_tol=params.s_tol, r_max=params.r_max, alpha_far=params.alpha_far,
                          alpha_near=params.alpha_near, r_switch=params.r_switch,
                          r_add_max=r_add_max)
        return lowrank_step(grid, X, eps, occ, R, p, prec=prec, rho=rho if update else None,
                            U=U, T=T, drho=drho, r_keep=r_keep)[3]

    for it in range(max_iter):
        effective_potential(grid, V_ext, rho, out=V, vrange=vr)
        vmin, vmax = vr.tolist()
        b = lap_top + vmax
        if a is None:
            a0 = vmin - 0.1
            a = a0 + 0.25 * (b - a0)
        for p in range(first_passes if it == 0 else 1):
            chfsi_filter(grid, V, X, 10 if (it == 0 and p == 0) else degree, a, b, a0, prec=prec,
                         out=Y)
            subspace_rayleigh_ritz(grid, V, Y, prec=prec, eps=eps)
            X, Y = Y, X
            lo, hi = eps[0].item(), eps[-1].item()
            a, a0 = hi, lo - 0.1
        density(grid, X, eps, occ, prec=prec, rho_in=rho, out=R)
        if kept >= params.r_max:
            clear_next = True
        beta = None
        event = "fresh" if kept == 0 else ("CT" if clear_next else None)
        info = None
        if event is None:
            probe = step(kept, -1, False)            # the kept directions against this R
            if probe["norm_R"] < tol:
                log.append(dict(probe, event="done", beta=None, added=0))
                break
            beta = abs(norm_R_lin / probe["norm_R"] - 1.0)
            if beta > beta_tol:
                event = "CL"
            elif probe["s_rel"] < params.s_tol:
                event = "reuse"
                info = step(kept, -1, True)
            elif probe["norm_R"] > params.r_switch:
                event = "CR"
            else:
                event = "accumulate"
                info = step(kept, min(r_iter_max, params.r_max - kept), True)
                kept = info["rank"]
                clear_next = info["s_rel"] >= params.s_tol
        if info is None:
            info = step(0, 0, True)
            kept = info["rank"]
            clear_next = False
        norm_R_lin = info["norm_R_lin"]
        log.append(dict(info, event=event, beta=beta))
        if info["norm_R"] < tol:
            break
    return rho, eps, log, X
