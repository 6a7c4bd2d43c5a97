"""Model SCF driven by the LRDM step (Sec. II A-D): rho -> V_eff[rho] ->
ChFSI (filter + Rayleigh-Ritz, per channel) -> R[rho] = F[V_eff[rho]] - rho ->
the low-rank quasi-Newton update rho <- rho - alpha P^lr_r R.

Every step runs in the library's kernels (lrdm_effective_potential,
lrdm_lda_xc, chfsi_filter, subspace_rayleigh_ritz, lrdm_density,
lrdm_lowrank_step); this module only holds the buffers and reads back the few
scalars the loop decides on (the potential's range for the filter's upper
bound, the extreme Ritz values for its other bounds, and the step's ||R||,
rank, s_rel and predicted residual).
"""
from __future__ import annotations

import torch

from .lrdm import (Grid, LowRankParams, Occupation, chfsi_filter, density, effective_potential,
                   lda_xc, lowrank_step, subspace_rayleigh_ritz)


class _ModelSCF:
    """Buffers and the eigen-part of one SCF step of the model
    V_eff = V_ext + V_H[rho] (+ V_xc[rho] of the LDA with xc)."""

    def __init__(self, grid: Grid, V_ext, X, occ: Occupation, degree: int, prec: str, xc: bool,
                 rho0, r_max: int, first_passes: int):
        ns = occ.nspin
        if X.shape[0] != ns:
            raise ValueError("X must be [nspin][N][nz][ny][nx]")
        if ns == 2 and not xc:
            raise ValueError("two channels need the exchange-correlation term to differ")
        self.grid, self.V_ext, self.occ, self.degree, self.prec, self.xc = (
            grid, V_ext, occ, degree, prec, xc)
        self.first_passes = first_passes
        dev = X.device
        self.N = X.shape[1]
        hx, hy, hz = (grid.L[d] / grid.n[d] for d in range(3))
        self.lap_top = 2.0 / hx ** 2 + 2.0 / hy ** 2 + 2.0 / hz ** 2
        vol = grid.L[0] * grid.L[1] * grid.L[2]
        shape = (ns,) + grid.shape
        f64 = dict(dtype=torch.float64, device=dev)
        if rho0 is None:
            self.rho = torch.full(shape, occ.n_electrons / vol / ns, **f64)
        else:
            self.rho = rho0.reshape(shape).clone()
        self.V = torch.empty(shape if xc else grid.shape, **f64)
        self.vr = torch.empty(2, **f64)
        self.vxc = torch.empty(shape, **f64) if xc else None
        self.fxc = torch.empty((ns, ns) + grid.shape, **f64) if xc else None
        self.R = torch.empty(shape, **f64)
        self.U = torch.empty((r_max,) + shape, **f64)
        self.T = torch.empty_like(self.U)
        self.drho = torch.empty(shape, **f64)
        self.eps = torch.empty((ns, self.N), **f64)
        self.X = X
        self.Y = torch.empty_like(X)
        self.bounds = [None] * ns
        self.it = 0
        self.switched = False       # alpha has switched to alpha_near (Sec. III A)

    def residual(self):
        """V_eff, one ChFSI pass per channel (first_passes on the first step), and
        R = rho_out - rho into self.R; the LDA kernel at rho into self.fxc."""
        g, ns = self.grid, self.occ.nspin
        if self.xc:
            lda_xc(g, self.rho, vxc=self.vxc, fxc=self.fxc)
        effective_potential(g, self.V_ext, self.rho, out=self.V, vrange=self.vr, vxc=self.vxc)
        vmin, vmax = self.vr.tolist()
        b = self.lap_top + vmax
        for p in range(self.first_passes if self.it == 0 else 1):
            deg = 10 if (self.it == 0 and p == 0) else self.degree
            for c in range(ns):
                if self.bounds[c] is None:
                    a0 = vmin - 0.1
                    self.bounds[c] = (a0 + 0.25 * (b - a0), a0)
                a, a0 = self.bounds[c]
                Vc = self.V[c] if self.xc else self.V
                chfsi_filter(g, Vc, self.X[c], deg, a, b, a0, prec=self.prec, out=self.Y[c])
                subspace_rayleigh_ritz(g, Vc, self.Y[c], prec=self.prec, eps=self.eps[c])
                lo, hi = self.eps[c, 0].item(), self.eps[c, -1].item()
                self.bounds[c] = (hi, lo - 0.1)
            self.X, self.Y = self.Y, self.X
        self.it += 1
        density(g, self.X, self.eps, self.occ, prec=self.prec, rho_in=self.rho, out=self.R)

    def step(self, params: LowRankParams, r_keep: int, r_add_max: int, update: bool):
        """One low-rank step on self.R.  alpha follows the schedule of Sec. III A:
        alpha_far until ||R|| goes below alpha_switch, alpha_near from that step
        on (the switch is made once; later steps pass an infinite threshold)."""
        p = LowRankParams(s_tol=params.s_tol, r_max=params.r_max, alpha_far=params.alpha_far,
                          alpha_near=params.alpha_near,
                          alpha_switch=float("inf") if self.switched else params.alpha_switch,
                          r_add_max=r_add_max)
        info = lowrank_step(self.grid, self.X, self.eps, self.occ, self.R, p, prec=self.prec,
                            rho=self.rho if update else None, U=self.U, T=self.T,
                            drho=self.drho, r_keep=r_keep, fxc=self.fxc)[3]
        if update and info["norm_R"] < params.alpha_switch:
            self.switched = True
        return info


def lrdma_event(kept: int, clear_pending: bool, beta, kept_s_rel, norm_R: float, s_tol: float,
                beta_tol: float, accumulate_below: float) -> str:
    """What the accumulated step does at this SCF step (Sec. II B 1, gates of
    Sec. III A): "fresh" without kept directions, "CT" for a clearing left by the
    last step, "CL" when the linearity indicator beta exceeds beta_tol, "reuse"
    when the kept directions fit R to s_rel < s_tol, "CR" when ||R|| is not below
    accumulate_below, else "accumulate"."""
    if kept == 0:
        return "fresh"
    if clear_pending:
        return "CT"
    if beta > beta_tol:
        return "CL"
    if kept_s_rel < s_tol:
        return "reuse"
    return "CR" if norm_R >= accumulate_below else "accumulate"


def _block(X, occ):
    return X if X.dim() == 5 else X.reshape((occ.nspin,) + tuple(X.shape))


def lrdm_scf(grid: Grid, V_ext, X, occ: Occupation, degree: int, prec: str = "fp64",
             params: LowRankParams = LowRankParams(), rho0=None, tol: float = 1e-8,
             max_iter: int = 50, first_passes: int = 4, xc: bool = False):
    """Solve R[rho] = 0 for the model V_eff = V_ext + V_H[rho] (+ V_xc[rho], LDA,
    with xc) by the LRDM step (K = K_c, + K_xc with xc).

    X [N][nz][ny][nx] (one channel) or [nspin][N][nz][ny][nx] is the starting
    block (double for fp64, float otherwise); it and one buffer like it
    alternate as filter input and output.  Each SCF step applies, per channel,
    one Chebyshev filter of the given degree and Rayleigh-Ritz (the first step
    applies first_passes of them, degree 10 for the first), with the filter's
    bounds b = sum_d 2/h_d^2 + max V_eff (an upper bound of the spectrum), a =
    the largest and a0 = the smallest Ritz value minus 0.1.  rho0 defaults to
    the uniform density, split evenly over the channels.  Two channels need xc
    (without it they would not differ).  Stops once the step reports
    ||R|| < tol (rho then carries that step's update too).

    Returns (rho [nspin][nz][ny][nx], eps [nspin][N], log, Psi): log holds one
    dict per step with norm_R, rank, s_rel and alpha; Psi [nspin][N][...] is
    the last block of Ritz vectors (one of the two alternating buffers)."""
    m = _ModelSCF(grid, V_ext, _block(X, occ), occ, degree, prec, xc, rho0, params.r_max,
                  first_passes)
    log = []
    for _ in range(max_iter):
        m.residual()
        info = m.step(params, 0, 0, True)
        log.append(info)
        if info["norm_R"] < tol:
            break
    return m.rho, m.eps, log, m.X


def lrdma_scf(grid: Grid, V_ext, X, occ: Occupation, degree: int, prec: str = "fp64",
              params: LowRankParams = LowRankParams(), beta_tol: float = 0.1, r_iter_max: int = 5,
              rho0=None, tol: float = 1e-8, max_iter: int = 50, first_passes: int = 4,
              xc: bool = False, accumulate_below: float = 1.0):
    """The model SCF of lrdm_scf with the accumulated low-rank step (LRDMA,
    Sec. II B 1).  At each SCF step, with R = R[rho]:
      * no kept directions, or a clearing pending (CT): build afresh;
      * beta = | ||R_lin|| / ||R|| - 1 | > beta_tol (Eq. (13)): clear (CL), afresh;
      * else if the kept directions fit R to s_rel < s_tol: reuse them;
      * else if ||R|| >= accumulate_below: clear (CR), afresh (Sec. III A
        accumulates only while ||R|| < 1.0);
      * else add at most r_iter_max directions to the kept ones; if s_rel stays
        at or above s_tol, clear before the next step (CT).
    Building afresh is the LRDM step (up to params.r_max directions); a full
    history (params.r_max kept) is cleared as CT.  R_lin is the residual the
    last step's approximation predicted (Eq. (12)), returned by the step.

    Returns (rho, eps, log, Psi) as lrdm_scf; each log entry also has added,
    event and beta."""
    m = _ModelSCF(grid, V_ext, _block(X, occ), occ, degree, prec, xc, rho0, params.r_max,
                  first_passes)
    kept = 0
    norm_R_lin = None
    clear_next = False
    log = []
    for _ in range(max_iter):
        m.residual()
        if kept >= params.r_max:
            clear_next = True
        beta = None
        info = None
        if kept and not clear_next:
            probe = m.step(params, kept, -1, False)     # the kept directions against this R
            if probe["norm_R"] < tol:
                log.append(dict(probe, event="done", beta=None, added=0))
                break
            beta = abs(norm_R_lin / probe["norm_R"] - 1.0)
            event = lrdma_event(kept, False, beta, probe["s_rel"], probe["norm_R"],
                                params.s_tol, beta_tol, accumulate_below)
        else:
            event = lrdma_event(kept, clear_next, None, None, 0.0, params.s_tol, beta_tol,
                                accumulate_below)
        if event == "reuse":
            info = m.step(params, kept, -1, True)
        elif event == "accumulate":
            info = m.step(params, kept, min(r_iter_max, params.r_max - kept), True)
            kept = info["rank"]
            clear_next = info["s_rel"] >= params.s_tol
        if info is None:
            info = m.step(params, 0, 0, True)
            kept = info["rank"]
            clear_next = False
        norm_R_lin = info["norm_R_lin"]
        log.append(dict(info, event=event, beta=beta))
        if info["norm_R"] < tol:
            break
    return m.rho, m.eps, log, m.X
