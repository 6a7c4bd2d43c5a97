"""Chebyshev filter where two or three recurrence steps run in one sweep (a
block owns a whole z column: short columns, or 1024 states and more), against
the FP64 oracle: small grids with degrees that leave every mix of three-step,
two-step and single sweeps, the shortest columns the sweeps take (nz = 4 for
two steps, 8 for three), and the 64^3 / 1024-state workload in the launch
configuration the bench times, on sampled states (the filter acts on each
state alone, so the oracle filters only those)."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import filter_bounds, rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402


@pytest.mark.parametrize("n,box,N", [((24, 20, 10), (10.0, 8.3, 4.2), 7),
                                     ((12, 8, 8), (5.2, 3.5, 3.5), 4),
                                     ((16, 8, 4), (7.0, 3.5, 1.8), 3)])
@pytest.mark.parametrize("degree", [2, 3, 4, 8, 9, 10])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_filter_sweeps_small(n, box, N, degree, prec):
    g = O.Grid(n, box)
    rng = np.random.default_rng(degree + 10 * N)
    V = rng.uniform(-1.0, 0.0, g.shape)
    X = rng.standard_normal((N,) + g.shape)
    a, b, a0 = filter_bounds(V, g)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd = to_dev(X, dt)
    Y = to_host(L.chfsi_filter(L.Grid(g.n, g.L), to_dev(V), Xd, degree, a, b, a0, prec=prec))
    ref = O.chebyshev_filter(to_host(Xd).astype(np.float64), V, g, degree, a, b, a0)
    err = rel(Y, ref)
    print(f"{prec} grid {n} N={N} degree {degree}: rel err {err:.2e}")
    assert err < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("degree", [5, 40])
def test_filter_sweeps_full_size_sampled(degree):
    """FP32 block of 1024 states on the 64^3 grid; states 0, 1, 517 and 1023
    against the oracle's filter of the same FP32-rounded states."""
    n, box, N = (64, 64, 64), (28.0, 28.0, 28.0), 1024
    g = O.Grid(n, box)
    rng = np.random.default_rng(64)
    V = rng.uniform(-1.0, 0.0, g.shape)
    gen = torch.Generator(device="cuda").manual_seed(517)
    Xd = torch.randn((N,) + g.shape, dtype=torch.float32, device="cuda", generator=gen)
    Xd /= torch.linalg.vector_norm(Xd.reshape(N, -1), dim=1).reshape(N, 1, 1, 1)
    a, b, a0 = filter_bounds(V, g)
    Y = L.chfsi_filter(L.Grid(g.n, g.L), to_dev(V), Xd, degree, a, b, a0, prec="fp32")
    torch.cuda.synchronize()
    pick = [0, 1, 517, 1023]
    Ys = to_host(Y[pick])
    ref = O.chebyshev_filter(to_host(Xd[pick]).astype(np.float64), V, g, degree, a, b, a0)
    for k in range(len(pick)):
        err = rel(Ys[k], ref[k])
        print(f"degree {degree} state {pick[k]}: rel err {err:.2e}")
        assert err < 1e-5
