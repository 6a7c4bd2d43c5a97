"""The density response at the full size of the 64^3 / 1024-state / 16-direction
workload, in the launch configuration the bench times (all 16 directions in one
call), against the FP64 oracle on sampled outputs: for two directions the oracle
forms the whole N x N projected perturbation, the Fermi quantities and Gamma,
and evaluates delta rho at 64 seeded grid points.  Each form is compared on its
own storage of Psi (the FP32 forms' rounded block, in FP64, for the oracle).
Bounds: FP64 1e-10, FP32 1e-5, BF16X3 1e-6 relative (l2 over the samples)."""
import numpy as np
import pytest

import oracle as O
from inputs import make_workload
from tests.gpu_common import rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402

BOUND = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-6}


@pytest.fixture(scope="module")
def c64():
    """Seeded unit-norm block (the response formula does not need orthonormal
    rows), sorted energies across the Fermi level, and dV = K_H u for the
    workload's 16 GRF directions (formed by the oracle; the same dV feeds both
    sides)."""
    wl = make_workload("c64_n1024_slab")
    g = O.Grid(wl.n, wl.L)
    grid = L.Grid(tuple(wl.n), tuple(wl.L))
    N = wl.N
    gen = torch.Generator(device="cuda").manual_seed(1024)
    Psi = torch.randn((N,) + grid.shape, dtype=torch.float64, device="cuda", generator=gen)
    Psi /= torch.linalg.vector_norm(Psi.reshape(N, -1), dim=1).reshape(N, 1, 1, 1)
    eps = torch.sort(torch.rand(N, dtype=torch.float64, device="cuda", generator=gen) * 3.0
                     - 2.0)[0]
    u = wl.directions()                                       # [r][1][nz][ny][nx]
    dV = to_dev(np.stack([O.hartree_kernel(u[k, 0], g)[None] for k in range(len(u))]))
    return wl, g, grid, Psi, eps, dV


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_density_response_full_size_sampled(c64, prec):
    wl, g, grid, Psi64, eps, dV = c64
    N, M, r = wl.N, g.M, wl.rank
    Psi = Psi64 if prec == "fp64" else Psi64.float().contiguous()
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    drho, mu, dmu = L.density_response(grid, Psi, eps, occ, dV, prec=prec)
    drho = to_host(drho)
    P = to_host(Psi).reshape(N, M)            # the form's input, in FP64
    e = to_host(eps)
    dVh = to_host(dV)
    mu_o, ok = O.fermi_level(e, wl.n_electrons, wl.kT, 1)
    assert ok
    _, _, fp = O.fermi_dirac(e, mu_o, wl.kT)
    F = O.divided_differences(e, mu_o, wl.kT)
    pts = np.sort(np.random.default_rng(64).choice(M, 64, replace=False))
    errs = []
    for k in (0, r - 1):
        Hp = O.projected_perturbation(P, dVh[k, 0])
        dmu_o = O.fermi_shift([Hp], [fp])
        G = O.response_density_matrix(F, Hp, dmu_o, fp)
        ref = O.density_from_matrix(P[:, pts], G, g.dv, O.spin_factor(1))
        got = drho[k, 0].reshape(-1)[pts]
        errs.append(rel(got, ref))
        assert abs(float(to_host(dmu)[k]) - dmu_o) < 10 * BOUND[prec] * max(1.0, abs(dmu_o))
        del Hp, G
    assert abs(float(to_host(mu).ravel()[0]) - mu_o) < 1e-12
    print(f"{prec}: sampled delta rho rel err {max(errs):.2e} (directions 0 and {r - 1})")
    assert max(errs) < BOUND[prec]
