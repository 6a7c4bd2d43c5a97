"""Batched uneven systems (density_response_batched): 16 spin-polarised systems
with grids from {32,40,48,56}^3, 64-512 states and 4-20 directions each, FP32
storage.  Each system's result is bit-identical to a single density_response
call; the two smallest systems match the FP64 oracle everywhere and all 16 on
sampled points; and the batch captured into a HIP graph replays to the same
bits.  The BF16X3 form of the batch (the systems forked over streams) is
bit-identical to its single calls and within its 1e-6 bound of the oracle on
the two smallest systems."""
import time

import numpy as np
import pytest

import oracle as O
from inputs import batched_systems, grf_directions
from tests.gpu_common import rel, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402


def _system_inputs(wl, dtype=torch.float32):
    """Seeded inputs of one batched system: per channel an orthonormalised random
    block (the seeded Gaussian block of the workload, QR by torch on the GPU),
    sorted energies around the Fermi level, and dV = K_c u for the workload's GRF
    directions (both channels see the same K_c (u_up + u_down); formed by the
    oracle)."""
    grid = L.Grid(tuple(wl.n), tuple(wl.L))
    N, M = wl.N, wl.M
    blocks = []
    for c in range(2):
        X = torch.from_numpy(wl.block(channel=c)).to("cuda").reshape(N, M)
        Q, _ = torch.linalg.qr(X.T)
        blocks.append(Q.T.contiguous())
    Psi = torch.stack(blocks).reshape((2, N) + grid.shape).to(dtype).contiguous()
    rng = np.random.default_rng(wl.system_id)
    eps = np.sort(rng.uniform(-2.0, 0.5, (2, N)), axis=1)
    eps[1] += 0.01
    U = grf_directions(wl.system_id, wl.n, wl.L, wl.rank, nspin=2)
    g = O.Grid(wl.n, wl.L)
    dV1 = np.stack([O.hartree_kernel(U[k, 0] + U[k, 1], g) for k in range(wl.rank)])
    dV = torch.from_numpy(np.stack([dV1, dV1], axis=1)).to("cuda").contiguous()
    return dict(grid=grid, Psi=Psi, eps=torch.from_numpy(eps).to("cuda"),
                occ=L.Occupation(2, wl.kT, wl.n_electrons), dV=dV)


@pytest.fixture(scope="module")
def systems():
    wls = batched_systems(16)
    return wls, [_system_inputs(wl) for wl in wls]


def test_batched_equals_single_calls(systems):
    wls, sys_in = systems
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = L.density_response_batched(sys_in, prec="fp32")
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    single = [L.density_response(s["grid"], s["Psi"], s["eps"], s["occ"], s["dV"], prec="fp32")
              for s in sys_in]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    dirs = sum(wl.rank for wl in wls)
    print(f"16 systems, {dirs} directions: batched {1e3 * t_batch:.1f} ms, "
          f"one call each {1e3 * t_single:.1f} ms")
    for (d, mu, dmu), (ds, mus, dmus) in zip(out, single):
        assert torch.equal(d, ds) and torch.equal(mu, mus) and torch.equal(dmu, dmus)


def test_batched_smallest_systems_match_oracle(systems):
    wls, sys_in = systems
    order = sorted(range(len(wls)), key=lambda k: wls[k].M * wls[k].N ** 2)[:2]
    out = L.density_response_batched([sys_in[k] for k in order], prec="fp32")
    for (d, _, _), k in zip(out, order):
        wl, s = wls[k], sys_in[k]
        g = O.Grid(wl.n, wl.L)
        Psi = to_host(s["Psi"])             # the FP32 block, in FP64
        ref, _, _ = O.density_response(Psi, to_host(s["eps"]), g, wl.n_electrons, wl.kT,
                                       to_host(s["dV"]), 2)
        err = max(rel(to_host(d)[j, c], ref[j, c]) for j in range(wl.rank) for c in range(2))
        print(f"system {k} ({wl.n[0]}^3, N={wl.N}, r={wl.rank}): rel err {err:.2e}")
        assert err < 1e-5


def test_batched_bf16x3_equals_single_calls_and_oracle(systems):
    wls, sys_in = systems
    out = L.density_response_batched(sys_in, prec="bf16x3")
    single = [L.density_response(s["grid"], s["Psi"], s["eps"], s["occ"], s["dV"],
                                 prec="bf16x3") for s in sys_in]
    for (d, mu, dmu), (ds, mus, dmus) in zip(out, single):
        assert torch.equal(d, ds) and torch.equal(mu, mus) and torch.equal(dmu, dmus)
    order = sorted(range(len(wls)), key=lambda k: wls[k].M * wls[k].N ** 2)[:2]
    for k in order:
        wl, s, d = wls[k], sys_in[k], out[k][0]
        g = O.Grid(wl.n, wl.L)
        ref, _, _ = O.density_response(to_host(s["Psi"]), to_host(s["eps"]), g, wl.n_electrons,
                                       wl.kT, to_host(s["dV"]), 2)
        err = max(rel(to_host(d)[j, c], ref[j, c]) for j in range(wl.rank) for c in range(2))
        print(f"bf16x3 system {k} ({wl.n[0]}^3, N={wl.N}, r={wl.rank}): rel err {err:.2e}")
        assert err < 1e-6


def test_batched_all_systems_match_oracle_sampled(systems):
    """Every system of the batch against the FP64 oracle, in the batched launch:
    for the first and last direction and both channels the oracle forms the
    whole N x N projected perturbation, the common Fermi level and shift, and
    delta rho at 48 seeded points (FP32 bound, 1e-5 relative over the samples)."""
    wls, sys_in = systems
    out = L.density_response_batched(sys_in, prec="fp32")
    worst = 0.0
    for k, ((d, mu, dmu), wl, s) in enumerate(zip(out, wls, sys_in)):
        g = O.Grid(wl.n, wl.L)
        N, M = wl.N, g.M
        P = to_host(s["Psi"]).reshape(2, N, M)       # the FP32 blocks, in FP64
        e = to_host(s["eps"])
        dVh = to_host(s["dV"])
        mu_o, ok = O.fermi_level(e, wl.n_electrons, wl.kT, 2)
        assert ok and abs(float(mu.item()) - mu_o) < 1e-12
        fps = [O.fermi_dirac(e[c], mu_o, wl.kT)[2] for c in range(2)]
        Fs = [O.divided_differences(e[c], mu_o, wl.kT) for c in range(2)]
        pts = np.sort(np.random.default_rng(k).choice(M, 48, replace=False))
        dh = to_host(d)
        for j in (0, wl.rank - 1):
            Hps = [O.projected_perturbation(P[c], dVh[j, c]) for c in range(2)]
            dmu_o = O.fermi_shift(Hps, fps)
            assert abs(float(to_host(dmu)[j]) - dmu_o) < 1e-4 * max(1.0, abs(dmu_o))
            for c in range(2):
                G = O.response_density_matrix(Fs[c], Hps[c], dmu_o, fps[c])
                ref = O.density_from_matrix(P[c][:, pts], G, g.dv, O.spin_factor(2))
                worst = max(worst, rel(dh[j, c].reshape(-1)[pts], ref))
        print(f"system {k} ({wl.n[0]}^3, N={N}, r={wl.rank}): sampled rel err so far {worst:.2e}")
    assert worst < 1e-5


def test_batched_graph_replays(systems):
    """The whole batch captured into one HIP graph on a side stream and replayed
    three times, with other work on the stream in between; every replay gives
    the eager result bit for bit."""
    _, sys_in = systems
    s = torch.cuda.Stream()
    outs = [(torch.empty((si["dV"].shape[0], 2) + si["grid"].shape, dtype=torch.float64,
                         device="cuda"),
             torch.empty(1, dtype=torch.float64, device="cuda"),
             torch.empty(si["dV"].shape[0], dtype=torch.float64, device="cuda"))
            for si in sys_in]
    with torch.cuda.stream(s):
        L.density_response_batched(sys_in, prec="fp32", outs=outs)   # sizes the workspace
    s.synchronize()
    eager = [tuple(t.clone() for t in o) for o in outs]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        L.density_response_batched(sys_in, prec="fp32", outs=outs)
    for rep in range(3):
        for o in outs:
            for t in o:
                t.fill_(float("nan"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        print(f"replay {rep}: {1e3 * (time.perf_counter() - t0):.1f} ms")
        for o, e in zip(outs, eager):
            for t, te in zip(o, e):
                assert torch.equal(t, te)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        assert torch.isfinite((x * x).sum())
