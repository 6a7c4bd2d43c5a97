"""The 48^3 / 256-state workload (degree 30, 8 directions): the FP64 path and
FP32 storage against the oracle on identical inputs, stage by stage.  The input
subspace is the oracle's after two ChFSI passes from the seeded block (degrees
8 and 30); from it the GPU runs one more step: the filter (against the oracle's
three-term recurrence), Rayleigh-Ritz on its own filtered block (Ritz values
against the oracle's Householder QR and dense eigh of the oracle's filtered
block), and the residual derivative on the oracle's Ritz pairs (FP32: cast to
FP32 storage).  Bounds: FP64 1e-12 (filter), 1e-10 (Ritz values), 1e-9 (t);
FP32 1e-5 relative for every stage."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import filter_bounds, oracle_subspace, rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402

BOUND = {"fp64": (1e-12, 1e-10, 1e-9), "fp32": (1e-5, 1e-5, 1e-5)}


@pytest.fixture(scope="module")
def c48():
    wl, g, V, eps, Psi = oracle_subspace("c48_n256", passes=2)
    a, b, a0 = filter_bounds(V, g, eps)
    Y_ref = O.chebyshev_filter(Psi, V, g, wl.degree, a, b, a0)
    e_ref, Psi_ref = O.rayleigh_ritz(Y_ref, V, g)
    U = wl.directions()
    t_ref, _, _ = O.residual_derivative(Psi_ref[None], e_ref[None], g, wl.n_electrons, wl.kT,
                                        U, 1)
    return wl, g, V, Psi, (a, b, a0), Y_ref, e_ref, Psi_ref, U, t_ref


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_c48_step_against_oracle(c48, form):
    wl, g, V, Psi, filt, Y_ref, e_ref, Psi_ref, U, t_ref = c48
    grid = L.Grid(tuple(g.n), tuple(g.L))
    dt = torch.float64 if form == "fp64" else torch.float32
    b_f, b_e, b_t = BOUND[form]
    Vd = to_dev(V)
    Y = L.chfsi_filter(grid, Vd, to_dev(Psi, dt), wl.degree, *filt, prec=form)
    err_f = rel(to_host(Y), Y_ref)
    e = to_host(L.subspace_rayleigh_ritz(grid, Vd, Y, prec=form))
    err_e = float(np.max(np.abs(e - e_ref)) / np.max(np.abs(e_ref)))
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    t = L.residual_derivative(grid, to_dev(Psi_ref[None], dt), to_dev(e_ref[None]), occ,
                              to_dev(U), prec=form)
    err_t = rel(to_host(t), t_ref)
    print(f"c48 {form}: filter {err_f:.2e}, Ritz values {err_e:.2e}, t {err_t:.2e}")
    assert err_f < b_f and err_e < b_e and err_t < b_t
