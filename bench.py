"""Throughput of the LRDM density-response hot path on one MI355X.

One step = one pass of the whole path over the synthetic 64^3 / 1024-state
workload: chfsi_filter (degree 40) -> subspace_rayleigh_ritz ->
lrdm_residual_derivative for all 16 direction functions (Hartree kernel,
Fermi level, divided differences, projection, Fermi shift, back-projection,
t = drho - u).  The metric is directions per second, r / T_step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp64,...]

Prints ONE JSON line.  Inputs are resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "density-response directions/sec @64³ grid,1024 states vs FP64 path; rel err"
WORKLOAD = "c64_n1024_slab"
PEAK = {"hbm_GBs": 8000.0, "fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # TFLOP/s for contractions
FORM_DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="fp64,fp32,bf16x3")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--warm-passes", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the copy and GEMM measurements of the achievable peaks")
    ap.add_argument("--fermi-depths", default="6,8,10,12,16",
                    help="depths of the recursive Fermi expansion compared with the exact "
                         "divided differences on the FP64 form ('' to skip)")
    ap.add_argument("--scf-steps", type=int, default=40,
                    help="SCF steps of the model SCF run with the LRDM and the LRDMA step on "
                         "the headline form (0 to skip)")
    ap.add_argument("--grown", action="store_true",
                    help="also time the grown forms: 16 uneven batched systems (eager and "
                         "HIP-graph replay) and the 80^3 / 2048-state forward + adjoint")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default K-split counts of the projection contractions")
    ap.add_argument("--no-lrdm-step", action="store_true",
                    help="skip timing the low-rank step around the path")
    ap.add_argument("--cpu-protocol", action="store_true",
                    help="also time the oracle's median-of-3 full step on the 48^3 / 256-state "
                         "workload (about two minutes of host time)")
    ap.add_argument("--backproj-layout", type=int, choices=(0, 1), default=1,
                    help="BF16X3 back-projection layout: 1 = 256 points per workgroup (the "
                         "library default), 0 = 128 points")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run three 1 GiB device copies first: a kernel of known traffic for "
                         "scaling hardware byte counters")
    return ap.parse_args()


def kernel_source_hash(name: str) -> str:
    p = os.path.join(ROOT, "paper_2211_07894_amd", "csrc", name)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_record(kernel: str, workload: str, form: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken from the current kernel source; otherwise None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        recs = json.load(open(p))
    except Exception:
        return None
    for r in recs:
        if r.get("kernel") == kernel and r.get("workload") == workload and r.get("form") == form:
            if r.get("source_sha") == kernel_source_hash(r.get("source", "")):
                return r.get("bytes_per_launch")
    return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every box here has one MI355X and the path is "
              "not sharded across GPUs (see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2211_07894_amd as L
    from inputs import make_workload

    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = make_workload(args.workload)
    grid = L.Grid(tuple(wl.n), tuple(wl.L))
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    M, N, r, c = wl.M, wl.N, wl.rank, wl.degree
    hx, hy, hz = wl.h
    V = torch.from_numpy(wl.V[0]).to(dev)
    b_up = 2.0 / hx ** 2 + 2.0 / hy ** 2 + 2.0 / hz ** 2 + float(wl.V[0].max())
    log(f"workload {wl.name}: M={M} N={N} r={r} degree={c}")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)        # an elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 copies of 1 GiB")
    t0 = time.time()
    X = torch.empty((N,) + grid.shape, dtype=torch.float64, device=dev)
    chunk = 64
    for s in range(0, N, chunk):
        X[s:s + chunk] = torch.from_numpy(wl.block(states=range(s, min(N, s + chunk)))).to(dev)
    U = torch.from_numpy(wl.directions()).to(dev)          # [r][1][nz][ny][nx]
    log(f"inputs generated in {time.time() - t0:.1f}s")

    # ---- warm start: ChFSI passes (FP64 form) until the Ritz pair nearest mu has
    # a residual below 2e-3 or the pass budget is spent (untimed set-up)
    t0 = time.time()
    a0 = float(wl.V[0].min()) - 0.1
    a = a0 + 0.25 * (b_up - a0)
    Y = torch.empty_like(X)
    eps = None
    resid = float("nan")
    for p in range(args.warm_passes):
        deg = 10 if p == 0 else c
        L.chfsi_filter(grid, V, X, deg, a, b_up, a0, out=Y)
        eps = L.subspace_rayleigh_ritz(grid, V, Y)
        X, Y = Y, X
        a = float(eps[-1].item())
        a0 = float(eps[0].item()) - 0.2
        mu, _, _, _ = L.fermi_occupations(eps, occ, want_F=False)
        i = int(torch.argmin(torch.abs(eps - mu)).item())
        hpsi = L.hamiltonian_apply(grid, V, X[i:i + 1].contiguous())
        resid = float(torch.linalg.vector_norm(hpsi[0] - eps[i] * X[i]).item())
        log(f"warm pass {p}: degree {deg} residual(nearest mu) {resid:.2e} [{time.time() - t0:.1f}s]")
        if p > 0 and resid < 2e-3:
            break
    torch.cuda.synchronize()
    filt = (a, b_up, a0)

    results = {}
    ref = None      # FP64 form's Ritz pairs and t on them: the per-stage reference
    for form in forms:
        dt = torch.float64 if form == "fp64" else torch.float32
        Xf = X.to(dt).contiguous()
        Yf = torch.empty_like(Xf)
        t_out = torch.empty((r, 1) + grid.shape, dtype=torch.float64, device=dev)
        ctx = L.context()
        ctx.set_backproj_layout(args.backproj_layout)

        e_resp = torch.empty(N, dtype=torch.float64, device=dev)
        # K-split counts of the projection contractions for this form's shapes
        # (response, single direction, Gram), chosen by timing on this device
        tuned = None if args.no_autotune else L.autotune(grid, N, 1, r, prec=form)

        def step():
            L.chfsi_filter(grid, V, Xf, c, *filt, prec=form, out=Yf)
            e = L.subspace_rayleigh_ritz(grid, V, Yf, prec=form, eps=e_resp)
            L.residual_derivative(grid, Yf[None], e[None], occ, U, prec=form, out=t_out)
            return e

        try:
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
        except L.LrdmError as ex:
            log(f"form {form} unavailable: {ex}")
            continue
        ctx.profile(True)
        for k in ["cheb_step", "cheb_pair", "cheb_triple", "hpsi", "proj", "gram", "backproj", "nn", "eigh", "chol", "jac_sweep", "jac_solve", "jac_update", "hartree"]:
            ctx.profile_read(k)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        ctx.profile(False)
        kern = {k: ctx.profile_read(k) for k in
                ["cheb_step", "cheb_pair", "cheb_triple", "hpsi", "proj", "gram", "backproj", "nn", "eigh", "chol", "jac_sweep", "jac_solve", "jac_update", "hartree"]}
        ms_step = 1e3 * elapsed / args.steps
        # response only (r directions on this form's Ritz pairs): r / T_resp
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            L.residual_derivative(grid, Yf[None], e_resp[None], occ, U, prec=form, out=t_out)
        torch.cuda.synchronize()
        ms_resp = 1e3 * (time.perf_counter() - t0) / args.steps
        # errors in delta rho = t + u relative to the FP64 form: per stage (this
        # form's residual derivative on the FP64 Ritz pairs cast to its storage)
        # and end to end (its own filter and Rayleigh-Ritz)
        rel = rel_e2e = None
        if form == "fp64":
            e_last = step()
            torch.cuda.synchronize()
            ref = dict(Psi=Yf.clone(), eps=e_last.clone(), t=t_out.clone())
            rel = rel_e2e = 0.0
        elif ref is not None:
            drho_norm = torch.linalg.vector_norm(ref["t"] + U)
            t_stage = L.residual_derivative(grid, ref["Psi"].to(dt)[None], ref["eps"][None], occ, U,
                                            prec=form)
            rel = float((torch.linalg.vector_norm(t_stage - ref["t"]) / drho_norm).item())
            rel_e2e = float((torch.linalg.vector_norm(t_out - ref["t"]) / drho_norm).item())
        # the LRDM step around the path (Sec. II B): the model-SCF residual at a
        # uniform input density on this form's Ritz pairs, then low-rank steps with
        # the paper's parameters (one direction per response launch, adaptive rank)
        lrdm = None
        if not args.no_lrdm_step:
            vol = float(wl.L[0] * wl.L[1] * wl.L[2])
            rho_in = torch.full((1,) + grid.shape, wl.n_electrons / vol, dtype=torch.float64,
                                device=dev)
            Rres = torch.empty_like(rho_in)
            L.density(grid, Yf, e_resp, occ, prec=form, rho_in=rho_in, out=Rres)
            prm = L.LowRankParams()
            Ub = torch.empty((prm.r_max, 1) + grid.shape, dtype=torch.float64, device=dev)
            Tb = torch.empty_like(Ub)
            db = torch.empty_like(Rres)
            L.lowrank_step(grid, Yf, e_resp, occ, Rres, prm, prec=form, U=Ub, T=Tb, drho=db)
            torch.cuda.synchronize()
            keys = ["proj", "backproj", "hartree"]
            ctx.profile(True)
            for k in keys:
                ctx.profile_read(k)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, _, _, info = L.lowrank_step(grid, Yf, e_resp, occ, Rres, prm, prec=form, U=Ub,
                                               T=Tb, drho=db)
            torch.cuda.synchronize()
            ms_lr = 1e3 * (time.perf_counter() - t0) / args.steps
            ctx.profile(False)
            lr_kern = {k: ctx.profile_read(k) for k in keys}
            lrdm = dict(ms_per_step=round(ms_lr, 3), rank=info["rank"],
                        s_rel=round(info["s_rel"], 4), norm_R=round(info["norm_R"], 4),
                        alpha=info["alpha"],
                        ms_per_direction=round(ms_lr / max(info["rank"], 1), 3),
                        ms_per_direction_batched=round(ms_resp / r, 3),
                        kernel_ms_per_direction={k: round(v[0] / max(v[1], 1), 4)
                                                 for k, v in lr_kern.items() if v[1]})
            log(f"form {form}: LRDM step {ms_lr:.1f} ms, rank {info['rank']}, "
                f"s_rel {info['s_rel']:.3f}, ||R|| {info['norm_R']:.3f}")
            del Ub, Tb, db, Rres, rho_in
        # the model SCF around the path (Sec. II A-B) with the LRDM and the LRDMA
        # step, from the uniform density, on the headline form's warm block
        scf = None
        head_form = next(f for f in ("bf16x3", "fp32", "fp64") if f in forms)
        if form == head_form and args.scf_steps > 0:
            scf = {}
            for name, driver in (("lrdm", L.lrdm_scf), ("lrdma", L.lrdma_scf)):
                X0 = Yf.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, slog, _ = driver(grid, V, X0, occ, c, prec=form, tol=1e-6,
                                       max_iter=args.scf_steps, first_passes=1)
                torch.cuda.synchronize()
                dt_s = time.perf_counter() - t0
                dirs = sum(x["added"] if name == "lrdma" else x["rank"] for x in slog)
                scf[name] = dict(steps=len(slog), seconds=round(dt_s, 3), directions=dirs,
                                 norm_R=[round(x["norm_R"], 6) for x in slog],
                                 ranks=[x["rank"] for x in slog])
                if name == "lrdma":
                    scf[name]["events"] = [x["event"] for x in slog]
                log(f"model SCF ({name}, {form}): {len(slog)} steps in {dt_s:.2f}s, "
                    f"{dirs} directions, ||R|| {slog[0]['norm_R']:.3e} -> {slog[-1]['norm_R']:.3e}")
                del X0
        # the paper's recursive Fermi expansion against the exact divided
        # differences (Eqs. (23)-(24)), on the FP64 form so that the expansion error
        # is not hidden by storage rounding: relative error of delta rho = t + u
        expansion = None
        depths = [int(x) for x in args.fermi_depths.split(",") if x.strip()]
        if form == "fp64" and depths:
            expansion = {}
            t_exact = t_out.clone()
            drho_norm = torch.linalg.vector_norm(t_exact + U)
            t_rec = torch.empty_like(t_exact)
            try:
                for T in depths:
                    ctx.set_fermi_expansion(T)
                    L.residual_derivative(grid, Yf[None], e_resp[None], occ, U, prec=form,
                                          out=t_rec)
                    expansion[str(T)] = float(
                        (torch.linalg.vector_norm(t_rec - t_exact) / drho_norm).item())
            finally:
                ctx.set_fermi_expansion(0)
            log("recursive Fermi expansion, delta rho error vs exact: "
                + ", ".join(f"T={k} {v:.2e}" for k, v in expansion.items()))
            del t_exact, t_rec
        # the response's block mask on this form's Ritz values (the library drops the
        # blocks whose Fermi multiplier is at most 1e-14 of its largest entry):
        # counted here only to state the executed work
        _, _, _, Fm = L.fermi_occupations(e_resp, occ)
        nt = (N + 127) // 128
        bm = torch.zeros(nt, nt, dtype=torch.float64, device=dev)
        for I in range(nt):
            for J in range(I, nt):
                bm[I, J] = Fm[0, 128 * I:128 * I + 128, 128 * J:128 * J + 128].abs().max()
        active_blocks = int((bm > 1e-14 * bm.max()).sum().item())
        del Fm
        results[form] = dict(ms_per_step=ms_step, value=r * args.steps / elapsed, kernels=kern,
                             active_blocks=active_blocks,
                             lrdm_step=lrdm, fermi_expansion=expansion, model_scf=scf,
                             autotune=tuned,
                             rel_err_vs_fp64=rel, rel_err_end_to_end=rel_e2e,
                             ms_response=ms_resp, response_value=1e3 * r / ms_resp)
        log(f"form {form}: {ms_step:.1f} ms/step, {r * args.steps / elapsed:.2f} directions/s; "
            + ", ".join(f"{k} {v[0] / max(v[1], 1):.3f}ms x{v[1]}" for k, v in kern.items() if v[1]))
        del Xf, Yf

    if not results:
        log("no precision form ran")
        sys.exit(1)
    head = next(f for f in ("bf16x3", "fp32", "fp64") if f in results)
    hr = results[head]

    # ---- roofline of the dominant kernel (largest total time in the timed steps)
    s_bytes = 8 if head == "fp64" else 4
    per_launch = {
        # algorithmic work per launch, the method's own: the projection H' = Psi^T
        # diag(dV) Psi and the back-projection sum_ij Psi_i Gamma_ij Psi_j are
        # symmetric in (i, j), M N^2 flops per direction each (the dense
        # equivalent, 2 M N^2, is reported beside it); a filter step moves 3 M N s
        # bytes, two or three steps in one sweep 4 M N s bytes
        "backproj": ("mfma", r * 1.0 * M * N * N),
        "proj": ("mfma", r * 1.0 * M * N * N),
        "cheb_step": ("hbm", 3.0 * M * N * s_bytes + 8.0 * M),
        "cheb_pair": ("hbm", 4.0 * M * N * s_bytes + 8.0 * M),
        "cheb_triple": ("hbm", 4.0 * M * N * s_bytes + 8.0 * M),
    }
    dense_equiv = {"backproj": r * (2.0 * M * N * N + 2.0 * M * N), "proj": r * 2.0 * M * N * N}
    dom = max(per_launch, key=lambda k: hr["kernels"][k][0])
    ms_tot, launches = hr["kernels"][dom]
    bound, work = per_launch[dom]
    avg_s = ms_tot / 1e3 / max(launches, 1)
    if bound == "hbm":
        achieved, peak, unit = work / avg_s / 1e9, PEAK["hbm_GBs"], "GB/s"
    else:
        peak = PEAK["fp64"] if head == "fp64" else (PEAK["fp32"] if head == "fp32" else PEAK["bf16"])
        achieved, unit = work / avg_s / 1e12, "TFLOP/s"
    src = ("gemm.hip" if head == "fp64" else "gemm_lp.hip") if dom in ("backproj", "proj") \
        else "stencil.hip"
    # executed work: the contractions form only the upper triangle of 128 x 128
    # blocks, and of those only the active ones (blocks whose Fermi multiplier is
    # above 1e-14 of its largest entry); the BF16X3 form issues six BF16
    # products per FP32 product
    nt = (N + 127) // 128
    products = 6.0 if head == "bf16x3" else 1.0
    nblk = hr["active_blocks"]
    executed = {"backproj": products * r * (2.0 * M * 128 * 128 * nblk + 2.0 * M * N),
                "proj": products * r * 2.0 * M * 128 * 128 * nblk,
                "cheb_step": work, "cheb_pair": work, "cheb_triple": work}[dom]
    ex_rate = executed / avg_s / (1e9 if bound == "hbm" else 1e12)
    roofline = dict(kernel=dom, bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                    frac=round(achieved / peak, 4),
                    work_unit=("method's own flops: M N^2 per direction (symmetric in i, j)"
                               if bound == "mfma" else "algorithmic HBM bytes"),
                    executed_achieved=round(ex_rate, 3), executed_frac=round(ex_rate / peak, 4),
                    traffic=traffic_record(dom, WORKLOAD, head),
                    avg_launch_ms=round(1e3 * avg_s, 4), launches=launches,
                    work_per_launch=work, source=src,
                    active_blocks=f"{nblk} of {nt * (nt + 1) // 2}")
    if dom in dense_equiv:
        de = dense_equiv[dom] / avg_s / 1e12
        roofline["dense_equivalent_achieved"] = round(de, 3)
        roofline["dense_equivalent_frac"] = round(de / peak, 4)

    # ---- achievable peaks measured on this device (STREAM-style copy; large
    # library GEMMs on the matrix cores), so the fraction is stated both ways
    if not args.no_peaks:
        measured = measure_peaks(torch, dev)
        key = "hbm_GBs" if bound == "hbm" else {"fp64": "fp64", "fp32": "fp32"}.get(head, "bf16")
        roofline["measured_peak"] = measured.get(key)
        if roofline["measured_peak"]:
            roofline["frac_of_measured"] = round(achieved / roofline["measured_peak"], 4)
            roofline["executed_frac_of_measured"] = round(ex_rate / roofline["measured_peak"], 4)
        roofline["measured_peaks"] = measured

    grown = grown_forms(torch, L, dev) if args.grown else None

    # ---- CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, filt, full_c2=args.cpu_protocol)

    line = {
        "metric": METRIC,
        "value": round(hr["value"], 4),
        "unit": "directions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": FORM_DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: periodic 64^3 grid, 28 bohr cell, 256 Gaussian wells "
                               f"+ 20% slab at +0.5 Ha; 1024 states, 800 electrons, kT 0.005 Ha, "
                               f"Chebyshev degree 40, 16 GRF directions",
                   "form": head, "warm_start_residual": resid},
        "rel_err_vs_fp64": hr["rel_err_vs_fp64"],
        "rel_err_end_to_end": hr["rel_err_end_to_end"],
        "forms": {f: {"value": round(v["value"], 4), "ms_per_step": round(v["ms_per_step"], 3),
                      "response_value": round(v["response_value"], 3),
                      "ms_response": round(v["ms_response"], 3),
                      "rel_err_vs_fp64": v["rel_err_vs_fp64"],
                      "rel_err_end_to_end": v["rel_err_end_to_end"],
                      "lrdm_step": v["lrdm_step"],
                      "autotune_splits": (v["autotune"] or {}).get("splits"),
                      "active_blocks": v["active_blocks"],
                      "backproj_layout": ((v["autotune"] or {}).get("backproj_layout",
                                                                     args.backproj_layout)
                                          if f == "bf16x3" else None),
                      "kernel_ms": {k: round(x[0] / max(x[1], 1), 4) for k, x in v["kernels"].items() if x[1]}}
                  for f, v in results.items()},
        "fermi_expansion_rel_err": results.get("fp64", {}).get("fermi_expansion"),
        "model_scf": results[head].get("model_scf"),
        "grown_forms": grown,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def grown_forms(torch, L, dev, reps=5):
    """Times of the grown forms (FP32 storage; FP32 and BF16X3 arithmetic):
    * 16 uneven spin-polarised systems (grids 32^3..56^3, 64-512 states, 4-20
      directions) in one density_response_batched call, eager and replayed from
      one captured HIP graph (median of `reps`);
    * the 80^3 / 2048-state / 20-direction response, forward and adjoint
      (density_response, density_response_backward with all three gradients).
    Inputs: per system an orthonormalised seeded Gaussian block (QR on the GPU),
    sorted seeded energies, dV = K_c(u_up + u_down) of the GRF directions."""
    import numpy as np
    from inputs import batched_systems, grf_directions, make_workload

    def ms_of(fn):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        return float(np.median(ts))

    systems, directions = [], 0
    for wl in batched_systems(16):
        grid = L.Grid(tuple(wl.n), tuple(wl.L))
        blocks = []
        for c in range(2):
            X = torch.from_numpy(wl.block(channel=c)).to(dev).reshape(wl.N, wl.M)
            Q, _ = torch.linalg.qr(X.T)
            blocks.append(Q.T.contiguous())
        Psi = torch.stack(blocks).reshape((2, wl.N) + grid.shape).float().contiguous()
        rng = np.random.default_rng(wl.system_id)
        eps = np.sort(rng.uniform(-2.0, 0.5, (2, wl.N)), axis=1)
        eps[1] += 0.01
        u = torch.from_numpy(grf_directions(wl.system_id, wl.n, wl.L, wl.rank, nspin=2)).to(dev)
        dV = L.hartree_kernel(grid, (u[:, 0] + u[:, 1]).contiguous())
        systems.append(dict(grid=grid, Psi=Psi, eps=torch.from_numpy(eps).to(dev),
                            occ=L.Occupation(2, wl.kT, wl.n_electrons),
                            dV=torch.stack([dV, dV], dim=1).contiguous()))
        directions += wl.rank
    outs = [(torch.empty((si["dV"].shape[0], 2) + si["grid"].shape, dtype=torch.float64,
                         device=dev),
             torch.empty(1, dtype=torch.float64, device=dev),
             torch.empty(si["dV"].shape[0], dtype=torch.float64, device=dev)) for si in systems]
    side = torch.cuda.Stream()
    batched = {}
    for form in ("fp32", "bf16x3"):
        with torch.cuda.stream(side):
            L.density_response_batched(systems, prec=form, outs=outs)     # sizes the workspace
            side.synchronize()

            def eager():
                L.density_response_batched(systems, prec=form, outs=outs)
            eager_ms = ms_of(eager)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=side):
                L.density_response_batched(systems, prec=form, outs=outs)
            replay_ms = ms_of(graph.replay)
        del graph
        log(f"batched 16 systems ({directions} directions x 2 channels, {form}): eager "
            f"{eager_ms:.1f} ms, graph replay {replay_ms:.1f} ms")
        batched[form] = dict(systems=16, directions=directions, eager_ms=round(eager_ms, 3),
                             graph_replay_ms=round(replay_ms, 3),
                             directions_per_s=round(1e3 * directions / replay_ms, 2))
    del systems, outs

    wl = make_workload("c80_n2048")
    grid, occ = L.Grid(tuple(wl.n), tuple(wl.L)), L.Occupation(1, wl.kT, wl.n_electrons)
    gen = torch.Generator(device=dev).manual_seed(2211)
    Psi = torch.randn((wl.N,) + grid.shape, dtype=torch.float32, device=dev, generator=gen)
    Psi /= torch.linalg.vector_norm(Psi.reshape(wl.N, -1), dim=1).reshape(wl.N, 1, 1, 1)
    eps = torch.sort(torch.rand(wl.N, dtype=torch.float64, device=dev, generator=gen) * 3 - 2)[0]
    U = torch.from_numpy(grf_directions(wl.system_id, wl.n, wl.L, wl.rank)).to(dev)
    dV = L.hartree_kernel(grid, U.reshape((wl.rank,) + grid.shape).contiguous())
    dV = dV.reshape((wl.rank, 1) + grid.shape).contiguous()
    G = torch.from_numpy(grf_directions(wl.system_id + 100, wl.n, wl.L, wl.rank)).to(dev)
    adjoint = {}
    for form in ("fp32", "bf16x3"):
        fwd_ms = ms_of(lambda: L.density_response(grid, Psi, eps, occ, dV, prec=form))
        bwd_ms = ms_of(lambda: L.density_response_backward(grid, Psi, eps, occ, dV, G, prec=form))
        log(f"80^3 / 2048 states / 20 directions ({form}): forward {fwd_ms:.1f} ms, "
            f"adjoint {bwd_ms:.1f} ms")
        adjoint[form] = dict(N=wl.N, M=wl.M, r=wl.rank, forward_ms=round(fwd_ms, 2),
                             backward_ms=round(bwd_ms, 2))
    del Psi, eps, U, dV, G
    return dict(batched=batched["fp32"], batched_bf16x3=batched["bf16x3"],
                adjoint_c80=adjoint["fp32"], adjoint_c80_bf16x3=adjoint["bf16x3"],
                kpoints_c48=kpoint_forms(torch, L, dev, ms_of))


def kpoint_forms(torch, L, dev, ms_of):
    """Brillouin-zone sampling on the 48^3 / 256-state cell: four k-points (Gamma,
    two zone-face midpoints along x and y, and the body diagonal's midpoint; weights
    1/8, 3/8, 3/8, 1/8).  Set-up (untimed): three real ChFSI passes (degree 10, then
    30) from the seeded block give a Gamma subspace; each k-point starts from it,
    takes one Bloch filter pass and the complex Rayleigh-Ritz.  Timed (median of
    the repetitions): one ChFSI pass of each k-point (Bloch filter, degree 30, and
    the complex Rayleigh-Ritz, FP64), and the zone-sampled response of the eight
    GRF directions (density_response_bz) in the three forms."""
    import numpy as np
    from inputs import grf_directions, make_workload
    wl = make_workload("c48_n256")
    grid = L.Grid(tuple(wl.n), tuple(wl.L))
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    N = wl.N
    V = torch.from_numpy(np.ascontiguousarray(wl.V[0])).to(dev)
    b_up = sum(2.0 / hd ** 2 for hd in wl.h) + float(wl.V[0].max())
    X = torch.from_numpy(wl.block()).to(dev).reshape((N,) + grid.shape).contiguous()
    Y = torch.empty_like(X)
    a0 = float(wl.V[0].min()) - 0.1
    a = a0 + 0.25 * (b_up - a0)
    for p in range(3):
        L.chfsi_filter(grid, V, X, 10 if p == 0 else wl.degree, a, b_up, a0, out=Y)
        e = L.subspace_rayleigh_ritz(grid, V, Y)
        X, Y = Y, X
        a, a0 = float(e[-1].item()), float(e[0].item()) - 0.2
    kx, ky, kz = (np.pi / L_ for L_ in wl.L)
    ks = [(0.0, 0.0, 0.0), (0.5 * kx, 0.0, 0.0), (0.0, 0.5 * ky, 0.0),
          (0.5 * kx, 0.5 * ky, 0.5 * kz)]
    weights = torch.tensor([0.125, 0.375, 0.375, 0.125], dtype=torch.float64, device=dev)
    nk = len(ks)
    Psi = torch.zeros((1, nk, 2, N) + grid.shape, dtype=torch.float64, device=dev)
    eps = torch.empty((1, nk, N), dtype=torch.float64, device=dev)
    Yk = torch.empty((2, N) + grid.shape, dtype=torch.float64, device=dev)
    bounds = []
    for q, k in enumerate(ks):
        Psi[0, q, 0] = X
        L.chfsi_filter_bloch(grid, V, Psi[0, q], k, wl.degree, a, b_up, a0, out=Yk)
        eps[0, q] = L.subspace_rayleigh_ritz_bloch(grid, V, Yk, k)
        Psi[0, q].copy_(Yk)
        bounds.append((float(eps[0, q, -1].item()), b_up, float(eps[0, q, 0].item()) - 0.2))

    def chfsi_pass(q):
        L.chfsi_filter_bloch(grid, V, Psi[0, q], ks[q], wl.degree, *bounds[q], out=Yk)
        L.subspace_rayleigh_ritz_bloch(grid, V, Yk, ks[q])

    pass_ms = [ms_of(lambda q=q: chfsi_pass(q)) for q in range(nk)]
    u = torch.from_numpy(grf_directions(wl.system_id, wl.n, wl.L, wl.rank)).to(dev)
    dV = L.hartree_kernel(grid, u.reshape((wl.rank,) + grid.shape).contiguous())
    dV = dV.reshape((wl.rank, 1) + grid.shape).contiguous()
    response = {}
    drho64 = None
    for form in ("fp64", "fp32", "bf16x3"):
        P = Psi if form == "fp64" else Psi.float()
        ms = ms_of(lambda: L.density_response_bz(grid, P, eps, weights, occ, dV, prec=form))
        drho, _, _ = L.density_response_bz(grid, P, eps, weights, occ, dV, prec=form)
        if drho64 is None:
            drho64 = drho.clone()
        err = float((torch.linalg.vector_norm(drho - drho64) /
                     torch.linalg.vector_norm(drho64)).item())
        response[form] = dict(ms=round(ms, 3), directions_per_s=round(1e3 * wl.rank / ms, 2),
                              rel_err_vs_fp64=err)
        log(f"zone sampling 48^3 / 256 states / 4 k-points / {wl.rank} directions ({form}): "
            f"response {ms:.2f} ms, rel err vs fp64 {err:.1e}")
    log("zone sampling: ChFSI pass per k-point (Bloch filter degree "
        f"{wl.degree} + complex Rayleigh-Ritz) " + ", ".join(f"{t:.1f}" for t in pass_ms) + " ms")
    return dict(grid=list(wl.n), N=N, nk=nk, weights=[0.125, 0.375, 0.375, 0.125],
                directions=wl.rank, chfsi_pass_ms_per_k=[round(t, 2) for t in pass_ms],
                response=response)


def measure_peaks(torch, dev):
    """Achievable rates on this device, for stating each roofline fraction against
    both the nominal and the measured peak: a 1 GiB device-to-device copy (2 GiB of
    traffic, STREAM copy), and large square GEMMs (torch.matmul, the vendor library)
    in BF16, FP32 and FP64 on the matrix cores.  Measurement infrastructure only."""
    out = {}

    def rate(fn, work, reps=5):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return work / (e0.elapsed_time(e1) / 1e3 / reps)

    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    out["hbm_GBs"] = round(rate(lambda: b.copy_(a), 8.0 * n) / 1e9, 1)
    del a, b
    for key, dt, k in (("bf16", torch.bfloat16, 8192), ("fp32", torch.float32, 8192),
                       ("fp64", torch.float64, 8192)):
        x = torch.randn(k, k, device=dev).to(dt)
        y = torch.randn(k, k, device=dev).to(dt)
        out[key] = round(rate(lambda: torch.matmul(x, y), 2.0 * k ** 3, reps=3) / 1e12, 1)
        del x, y
    torch.cuda.synchronize()
    log("measured peaks: " + ", ".join(f"{k} {v}" for k, v in out.items()))
    return out


def host_info():
    """CPU model, core counts and the BLAS the oracle's NumPy calls."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            blas.append(dict(api=i.get("internal_api"), version=i.get("version"),
                             threads=i.get("num_threads"), user_api=i.get("user_api")))
    except Exception:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = None
    return dict(cpu_model=model, nproc=os.cpu_count(), affinity_cores=affinity, blas=blas)


def _oracle_step(O, wl, X, filt, U):
    """One step of the oracle: the degree-c filter, Rayleigh-Ritz, and the
    residual derivative of every direction.  Returns the seconds taken."""
    g = O.Grid(wl.n, wl.L)
    t0 = time.perf_counter()
    Y = O.chebyshev_filter(X, wl.V[0], g, wl.degree, *filt)
    eps, Psi = O.rayleigh_ritz(Y, wl.V[0], g)
    O.residual_derivative(Psi[None], eps[None], g, wl.n_electrons, wl.kT, U, 1)
    return time.perf_counter() - t0


def _cold_bounds(wl):
    g = (wl.L[0] / wl.n[0], wl.L[1] / wl.n[1], wl.L[2] / wl.n[2])
    b = sum(2.0 / hd ** 2 for hd in g) + float(wl.V[0].max())
    a0 = float(wl.V[0].min()) - 0.1
    return a0 + 0.25 * (b - a0), b, a0


def _per_direction_single_core(O, wl, reps=3):
    """Median seconds of one direction of the residual derivative with one BLAS
    thread, on an orthonormal block of the workload's size (the cost does not
    depend on the values)."""
    from threadpoolctl import threadpool_limits
    g = O.Grid(wl.n, wl.L)
    Q, _ = np.linalg.qr(wl.block().reshape(wl.N, -1).T)
    Psi = Q.T.reshape((wl.N,) + g.shape).copy()
    del Q
    eps = np.sort(np.random.default_rng(0).uniform(-2.0, 1.0, wl.N))
    u = wl.directions(rank=1)
    ts = []
    with threadpool_limits(limits=1):
        for _ in range(reps):
            t0 = time.perf_counter()
            O.residual_derivative(Psi[None], eps[None], g, wl.n_electrons, wl.kT, u, 1)
            ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_baseline(wl, filt, full_c2=False):
    """The FP64 oracle timed on the host, following the protocol of the baseline
    plan: the host's CPU model, cores and BLAS; on the 24^3 / 32-state workload
    the median of three full steps (filter, Rayleigh-Ritz, all directions) with
    all cores; one-thread seconds per direction on the 24^3 and 48^3 workloads;
    with full_c2 also the median of three full steps on 48^3 / 256 states.  The
    headline value is the 64^3 / 1024-state step estimated from a bounded
    sample: the filter on 4 of 1024 states (scaled by N/4), Rayleigh-Ritz on 128
    states of the same grid (scaled by (N/128)^2, its leading M N^2 terms), and
    one full-size direction of the residual derivative (scaled by r)."""
    import oracle as O
    from inputs import make_workload
    info = host_info()
    cores = max([b.get("threads") or 1 for b in info["blas"]] + [1])
    out = {"host": info}
    c1 = make_workload("c24_n32")
    ts = [_oracle_step(O, c1, c1.block(), _cold_bounds(c1), c1.directions()) for _ in range(3)]
    out["c24_n32"] = dict(median_step_s=round(float(np.median(ts)), 4),
                          steps_s=[round(t, 4) for t in ts],
                          directions_per_s=round(c1.rank / float(np.median(ts)), 3),
                          single_core_s_per_direction=round(_per_direction_single_core(O, c1), 4))
    c2 = make_workload("c48_n256")
    out["c48_n256"] = dict(single_core_s_per_direction=round(_per_direction_single_core(O, c2), 3))
    if full_c2:
        ts = [_oracle_step(O, c2, c2.block(), _cold_bounds(c2), c2.directions())
              for _ in range(3)]
        out["c48_n256"].update(median_step_s=round(float(np.median(ts)), 2),
                               steps_s=[round(t, 2) for t in ts],
                               directions_per_s=round(c2.rank / float(np.median(ts)), 4))
    log(f"cpu oracle protocol: {out}")

    g = O.Grid(wl.n, wl.L)
    V = wl.V[0]
    N, r = wl.N, wl.rank
    t0 = time.perf_counter()
    Xs = wl.block(states=range(4))
    O.chebyshev_filter(Xs, V, g, wl.degree, *filt)
    t_filter = (time.perf_counter() - t0) * N / 4
    Ys = wl.block(states=range(128))
    t0 = time.perf_counter()
    O.rayleigh_ritz(Ys, V, g)
    t_rr = (time.perf_counter() - t0) * (N / 128) ** 2
    del Ys
    Psi = wl.block()
    Psi /= np.sqrt(g.M)
    eps = np.sort(np.random.default_rng(0).uniform(-2.0, 1.0, N))
    u = wl.directions(rank=1)
    t0 = time.perf_counter()
    O.residual_derivative(Psi[None], eps[None], g, wl.n_electrons, wl.kT, u, 1)
    t_dir = time.perf_counter() - t0
    del Psi
    t_step = t_filter + t_rr + r * t_dir
    log(f"cpu oracle: filter {t_filter:.1f}s (scaled), RR {t_rr:.1f}s (scaled), direction {t_dir:.2f}s")
    out.update({"value": round(r / t_step, 5), "unit": "directions/s", "cores": cores,
                "kind": "oracle",
                "sample": "FP64 NumPy oracle: filter on 4 of 1024 states (x256), Rayleigh-Ritz on "
                          "128 states (x64), one full-size residual-derivative direction (x16); "
                          f"estimated step {t_step:.1f}s",
                "c64_n1024_estimate_s": dict(filter=round(t_filter, 2), rayleigh_ritz=round(t_rr, 2),
                                             per_direction=round(t_dir, 3))})
    return out


if __name__ == "__main__":
    main()
