"""density_response_noalloc through the C ABI: the same results as
density_response on two calls in a row (the second smaller), in the three
forms, without growing the context's workspace; a problem beyond the fixed
scratch is rejected before any launch."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402
from paper_2211_07894_amd import lrdm as B  # noqa: E402

BOUND = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-6}


def _case(n, box, N, nspin, r, seed):
    g = L.Grid(n, box)
    M = n[0] * n[1] * n[2]
    rng = np.random.default_rng(seed)
    Psi = np.empty((nspin, N, M))
    for c in range(nspin):
        Q, _ = np.linalg.qr(rng.standard_normal((M, N)))
        Psi[c] = Q.T
    eps = np.sort(rng.uniform(-1.5, 0.8, (nspin, N)), axis=1)
    dV = rng.standard_normal((r, nspin, M))
    return g, Psi, eps, dV, L.Occupation(nspin, 0.01, 0.39 * 2 * N)


def _noalloc(ctx, g, Psi, eps, N, occ, dV, r, prec):
    ns = occ.nspin
    drho = torch.empty((r, ns, g.M), dtype=torch.float64, device="cuda")
    mu = torch.empty(1, dtype=torch.float64, device="cuda")
    dmu = torch.empty(r, dtype=torch.float64, device="cuda")
    gc, oc = g.c(), occ.c()
    st = ctx.lib.density_response_noalloc(
        ctx.ptr, ctypes.byref(gc), ctypes.c_void_p(Psi.data_ptr()),
        ctypes.c_void_p(eps.data_ptr()), N, ctypes.byref(oc), ctypes.c_void_p(dV.data_ptr()), r,
        B.PREC[prec], ctypes.c_void_p(drho.data_ptr()), ctypes.c_void_p(mu.data_ptr()),
        ctypes.c_void_p(dmu.data_ptr()))
    return st, drho, mu, dmu


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_density_response(prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    stream = torch.cuda.current_stream().cuda_stream
    fresh = B.Context(torch.cuda.current_device(), stream)      # its own, empty workspace
    try:
        for n, box, N, nspin, r, seed in (((20, 18, 13), (8.0, 7.2, 5.2), 150, 2, 3, 1),
                                          ((12, 10, 8), (5.0, 4.2, 3.4), 40, 1, 2, 2)):
            g, Psi, eps, dV, occ = _case(n, box, N, nspin, r, seed)
            Pd, ed, dd = to_dev(Psi, dt), to_dev(eps), to_dev(dV)
            st, drho, mu, dmu = _noalloc(fresh, g, Pd, ed, N, occ, dd, r, prec)
            assert st == 0, fresh.lib.lrdm_last_error(fresh.ptr).decode()
            torch.cuda.synchronize()
            assert fresh.lib.lrdm_workspace_bytes(fresh.ptr) == 0
            ref, mu_r, dmu_r = L.density_response(g, Pd, ed, occ, dd.reshape(r, nspin, *g.shape),
                                                  prec=prec)
            err = rel(to_host(drho), to_host(ref))
            print(f"{prec} N={N} nspin={nspin}: noalloc vs density_response {err:.2e}")
            assert err < BOUND[prec]
            assert float(mu.item()) == float(mu_r.item())
            assert rel(to_host(dmu), to_host(dmu_r)) < BOUND[prec]
    finally:
        fresh.close()


def test_noalloc_rejects_a_problem_beyond_its_scratch():
    """64^3 / 1024 states in FP32 storage: the back-projection's transposed copy of
    Psi alone is 1 GiB."""
    g = L.Grid((64, 64, 64), (28.0, 28.0, 28.0))
    N, r = 1024, 16
    Psi = torch.zeros((N, g.M), dtype=torch.float32, device="cuda")
    eps = torch.linspace(-1, 1, N, dtype=torch.float64, device="cuda")
    dV = torch.zeros((r, 1, g.M), dtype=torch.float64, device="cuda")
    ctx = L.context()
    before = ctx.lib.lrdm_workspace_bytes(ctx.ptr)
    st, _, _, _ = _noalloc(ctx, g, Psi, eps, N, L.Occupation(1, 0.01, 800.0), dV, r, "fp32")
    assert st == -1
    assert "bytes of scratch" in ctx.lib.lrdm_last_error(ctx.ptr).decode()
    assert ctx.lib.lrdm_workspace_bytes(ctx.ptr) == before
