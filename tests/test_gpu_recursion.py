"""The paper's recursive Fermi expansion (Eqs. (23)-(24)) as the response
multiplier, against the oracle's first-order perturbation of the recursion
(matrix form, diagonal shortcut taken only for the inversion): delta rho and mu'
for several depths, one and two channels, and the BF16X3 form."""
import numpy as np
import pytest

import oracle as O
from inputs import grf_directions
from tests.gpu_common import oracle_subspace, rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402


@pytest.fixture(scope="module")
def c24():
    return oracle_subspace("c24_n32", passes=2)


@pytest.fixture
def expansion():
    """Sets the depth on the shared context and always restores the exact form."""
    ctx = L.context()
    yield ctx.set_fermi_expansion
    ctx.set_fermi_expansion(0)


def _system(c24, nspin, r=2):
    wl, g, V, eps, Psi = c24
    Psi2 = np.stack([Psi] * nspin)
    eps2 = np.stack([eps + 0.003 * c for c in range(nspin)])
    dV = grf_directions(wl.system_id, wl.n, wl.L, r, nspin=nspin)
    return wl, g, Psi2, eps2, dV


@pytest.mark.parametrize("nspin", [1, 2])
@pytest.mark.parametrize("depth", [4, 8, 10, 16])
def test_recursive_response_fp64(c24, expansion, nspin, depth):
    wl, g, Psi2, eps2, dV = _system(c24, nspin)
    occ = L.Occupation(nspin, wl.kT, wl.n_electrons)
    grid = L.Grid(tuple(g.n), tuple(g.L))
    expansion(depth)
    drho, mu, dmu = L.density_response(grid, to_dev(Psi2), to_dev(eps2), occ, to_dev(dV))
    ref, mu_o, dmu_o = O.density_response_recursive(Psi2, eps2, g, wl.n_electrons, wl.kT, dV,
                                                    depth, nspin)
    exact, _, _ = O.density_response(Psi2, eps2, g, wl.n_electrons, wl.kT, dV, nspin)
    print(f"T={depth} nspin={nspin}: vs oracle {rel(to_host(drho), ref):.2e}, "
          f"expansion error {rel(ref, exact):.2e}")
    assert rel(to_host(drho), ref) < 1e-10
    assert np.abs(to_host(dmu) - dmu_o).max() < 1e-10 * max(1.0, np.abs(dmu_o).max())
    assert abs(float(to_host(mu)[0]) - mu_o) < 1e-12


def test_recursive_response_bf16x3_and_step(c24, expansion):
    """The low-precision form with the expansion, and the low-rank step built on it."""
    wl, g, Psi2, eps2, dV = _system(c24, 1)
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    grid = L.Grid(tuple(g.n), tuple(g.L))
    Psi_f = to_dev(Psi2, torch.float32)
    expansion(10)
    drho, _, _ = L.density_response(grid, Psi_f, to_dev(eps2), occ, to_dev(dV), prec="bf16x3")
    ref, _, _ = O.density_response_recursive(to_host(Psi_f), eps2, g, wl.n_electrons, wl.kT,
                                             dV, 10, 1)
    assert rel(to_host(drho), ref) < 1e-6
    # the step uses the same multiplier through the residual derivative
    R = 0.5 * dV[0]
    _, _, _, info = L.lowrank_step(grid, to_dev(Psi2), to_dev(eps2), occ, to_dev(R),
                                   L.LowRankParams(s_tol=0.0, r_max=3))

    def apply_t(u):
        d, _, _ = O.density_response_recursive(Psi2, eps2, g, wl.n_electrons, wl.kT,
                                               O.hartree_kernel(u, g)[None], 10, 1)
        return d[0] - u
    _, _, _, hist = O.lowrank_preconditioner(R, apply_t, g, 0.0, 3)
    assert info["rank"] == 3 and abs(info["s_rel"] - hist[-1]) < 1e-10


def test_backward_rejects_recursive_form(c24, expansion):
    wl, g, Psi2, eps2, dV = _system(c24, 1)
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    grid = L.Grid(tuple(g.n), tuple(g.L))
    expansion(8)
    with pytest.raises(L.LrdmError, match="EUNSUPPORTED"):
        L.density_response_backward(grid, to_dev(Psi2), to_dev(eps2), occ, to_dev(dV),
                                    to_dev(np.ones_like(dV)))
    with pytest.raises(L.LrdmError, match="depth must be in 0..64"):
        L.context().set_fermi_expansion(65)
