"""Single-precision storage forms (FP32, BF16X3) of the HIP path against the FP64
oracle.  Per stage, on identical inputs: the oracle's Ritz pairs are cast to the
form's FP32 storage and the response density is compared with the oracle's FP64
result on the uncast pairs.  Bounds: FP32 <= 1e-5 and BF16X3 <= 1e-6 relative
(l2, max over directions and channels)."""
import numpy as np
import pytest

import oracle as O
from inputs import grf_directions
from tests.gpu_common import filter_bounds, oracle_subspace, rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402

BOUND = {"fp32": 1e-5, "bf16x3": 1e-6}
FORMS = ["fp32", "bf16x3"]


def _grid(g: O.Grid):
    return L.Grid(tuple(g.n), tuple(g.L))


def f32(x):
    return to_dev(x, torch.float32)


@pytest.fixture(scope="module")
def c24():
    return oracle_subspace("c24_n32", passes=2)


def _random_subspace(n, box, N, nspin, seed):
    g = O.Grid(n, box)
    rng = np.random.default_rng(seed)
    Psi = np.stack([np.linalg.qr(rng.standard_normal((g.M, N)))[0].T.reshape((N,) + g.shape)
                    for _ in range(nspin)])
    eps = np.sort(rng.uniform(-1.0, 0.5, (nspin, N)), axis=1)
    return g, Psi, eps, rng


@pytest.mark.parametrize("form", FORMS)
def test_density_response_c24(c24, form):
    wl, g, V, eps, Psi = c24
    U = grf_directions(wl.system_id, wl.n, wl.L, wl.rank)
    dV = np.stack([O.hartree_kernel(U[k, 0], g)[None] for k in range(wl.rank)])
    drho, mu, dmu = L.density_response(_grid(g), f32(Psi[None]), to_dev(eps[None]),
                                       L.Occupation(1, wl.kT, wl.n_electrons), to_dev(dV),
                                       prec=form)
    ref, mu_o, dmu_o = O.density_response(Psi[None], eps[None], g, wl.n_electrons, wl.kT, dV, 1)
    errs = [rel(to_host(drho)[k], ref[k]) for k in range(wl.rank)]
    print(f"{form} c24 drho rel err {max(errs):.3e}")
    assert max(errs) < BOUND[form]
    assert abs(float(mu.item()) - mu_o) < 1e-12      # FP64 from eps alone
    assert np.max(np.abs(to_host(dmu) - dmu_o)) < BOUND[form] * np.max(np.abs(dmu_o))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("nspin", [1, 2])
def test_density_response_ragged_multitile(form, nspin):
    """N = 150 (two 128-row tiles, ragged) on a ragged grid with a random
    orthonormal subspace and energies spanning mu."""
    g, Psi, eps, rng = _random_subspace((20, 18, 13), (8.0, 7.2, 5.2), 150, nspin, 5)
    ne = 0.8 * 150
    dV = rng.standard_normal((3, nspin) + g.shape)
    drho, _, _ = L.density_response(_grid(g), f32(Psi), to_dev(eps), L.Occupation(nspin, 0.02, ne),
                                    to_dev(dV), prec=form)
    ref, _, _ = O.density_response(Psi, eps, g, ne, 0.02, dV, nspin)
    errs = [rel(to_host(drho)[k, c], ref[k, c]) for k in range(3) for c in range(nspin)]
    print(f"{form} nspin {nspin} drho rel err {max(errs):.3e}")
    assert max(errs) < BOUND[form]


@pytest.mark.parametrize("nspin", [1, 2])
def test_bf16x3_backproj_layouts(nspin):
    """Both BF16X3 back-projection layouts (256 and 128 points per workgroup)
    against the oracle: N = 300 (three row blocks, the last ragged), 4680 grid
    points (18 whole 256-point blocks and a ragged one), kT = 0.005 so that the
    occupied-occupied block drops out, and the two layouts within 1e-6 of each
    other."""
    g, Psi, eps, rng = _random_subspace((20, 18, 13), (8.0, 7.2, 5.2), 300, nspin, 21)
    ne = 0.6 * 300
    dV = rng.standard_normal((4, nspin) + g.shape)
    ref, _, _ = O.density_response(Psi, eps, g, ne, 0.005, dV, nspin)
    ctx = L.context()
    got = {}
    try:
        for layout in (1, 0):
            ctx.set_backproj_layout(layout)
            drho, _, _ = L.density_response(_grid(g), f32(Psi), to_dev(eps),
                                            L.Occupation(nspin, 0.005, ne), to_dev(dV),
                                            prec="bf16x3")
            got[layout] = to_host(drho)
            errs = [rel(got[layout][k, c], ref[k, c]) for k in range(4) for c in range(nspin)]
            print(f"layout {layout} nspin {nspin}: drho rel err {max(errs):.3e}")
            assert max(errs) < BOUND["bf16x3"]
    finally:
        ctx.set_backproj_layout(1)
    d = max(rel(got[1][k, c], got[0][k, c]) for k in range(4) for c in range(nspin))
    print(f"layouts differ by {d:.2e}")
    assert d < 1e-6


@pytest.mark.parametrize("form", FORMS)
def test_density_response_three_tiles_odd(form):
    """N = 300 (three tiles, the last ragged) and an odd grid of 7 x 9 x 11."""
    g, Psi, eps, rng = _random_subspace((7, 9, 11), (3.5, 4.5, 5.5), 300, 1, 9)
    ne = 0.7 * 300
    dV = rng.standard_normal((2, 1) + g.shape)
    drho, _, _ = L.density_response(_grid(g), f32(Psi), to_dev(eps), L.Occupation(1, 0.05, ne),
                                    to_dev(dV), prec=form)
    ref, _, _ = O.density_response(Psi, eps, g, ne, 0.05, dV, 1)
    for k in range(2):
        assert rel(to_host(drho)[k], ref[k]) < BOUND[form]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("nspin", [1, 2])
def test_residual_derivative(c24, form, nspin):
    wl, g, V, eps, Psi = c24
    U = grf_directions(wl.system_id, wl.n, wl.L, 3, nspin=nspin)
    Psi2 = np.stack([Psi] * nspin)
    eps2 = np.stack([eps + 0.003 * c for c in range(nspin)])
    ne = wl.n_electrons
    t = L.residual_derivative(_grid(g), f32(Psi2), to_dev(eps2), L.Occupation(nspin, wl.kT, ne),
                              to_dev(U), prec=form)
    ref, _, _ = O.residual_derivative(Psi2, eps2, g, ne, wl.kT, U, nspin)
    for k in range(3):
        # bound on delta rho = t + u
        err = np.linalg.norm(to_host(t)[k] - ref[k]) / np.linalg.norm(ref[k] + U[k])
        assert err < BOUND[form]


@pytest.mark.parametrize("form", FORMS)
def test_projected_perturbation(form):
    g, Psi, _, rng = _random_subspace((20, 18, 13), (8.0, 7.2, 5.2), 150, 1, 3)
    dV = rng.standard_normal((2, 1) + g.shape)
    Hp = to_host(L.projected_perturbation(_grid(g), f32(Psi), to_dev(dV), nspin=1, prec=form))
    P = Psi[0].reshape(150, -1)
    for k in range(2):
        ref = O.projected_perturbation(Psi[0], dV[k, 0])
        assert np.max(np.abs(Hp[k, 0] - ref)) < 1e-6 * np.max(np.abs(ref))
        assert np.array_equal(Hp[k, 0], Hp[k, 0].T)
    del P


def test_hamiltonian_apply_fp32():
    g = O.Grid((20, 18, 13), (8.0, 7.2, 5.2))
    rng = np.random.default_rng(1)
    V = rng.uniform(-2, 0, g.shape)
    X = rng.standard_normal((5,) + g.shape).astype(np.float32)
    HX = to_host(L.hamiltonian_apply(_grid(g), to_dev(V), f32(X), prec="fp32"))
    ref = O.hamiltonian_apply(X.astype(np.float64), V, g)
    assert rel(HX, ref) < 1e-6


@pytest.mark.parametrize("degree", [1, 2, 20])
def test_chfsi_filter_fp32(c24, degree):
    wl, g, V, eps, Psi = c24
    a, b, a0 = filter_bounds(V, g, eps)
    X = Psi.astype(np.float32)
    Y = to_host(L.chfsi_filter(_grid(g), to_dev(V), f32(X), degree, a, b, a0, prec="fp32"))
    ref = O.chebyshev_filter(X.astype(np.float64), V, g, degree, a, b, a0)
    # block-wise: FP32 rounding made at step k in the directions of the lowest
    # states is amplified like the polynomial itself, so a strongly damped state
    # carries a larger error relative to its own (tiny) norm
    print(f"filter fp32 degree {degree}: block rel err {rel(Y, ref):.2e}, worst state "
          f"{max(rel(Y[i], ref[i]) for i in range(wl.N)):.2e}")
    assert rel(Y, ref) < 1e-5


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("degree", [20, 40])
def test_rayleigh_ritz(c24, form, degree):
    """FP32 storage: Ritz values within 1e-5 of the spectral radius of the FP64
    oracle's, vectors orthonormal to 1e-5, and the response built on them (end
    to end through this form) within 1e-4 of the oracle's.  At degree 40 the
    filtered columns span about ten orders of magnitude, as at the 64^3 /
    1024-state workload: the Gram matrix there is beyond FP32 products."""
    wl, g, V, eps, Psi = c24
    a, b, a0 = filter_bounds(V, g, eps)
    Y = O.chebyshev_filter(Psi, V, g, degree, a, b, a0)
    norms = np.linalg.norm(Y.reshape(wl.N, -1), axis=1)
    print(f"degree {degree}: filtered column norms {norms.min():.2e} .. {norms.max():.2e}")
    eps_o, Psi_o = O.rayleigh_ritz(Y, V, g)
    Yd = f32(Y)
    e = to_host(L.subspace_rayleigh_ritz(_grid(g), to_dev(V), Yd, prec=form))
    scale = b
    assert np.max(np.abs(e - eps_o)) < 1e-5 * scale
    P = to_host(Yd).reshape(wl.N, -1)
    assert np.max(np.abs(P @ P.T - np.eye(wl.N))) < 1e-5
    dV = grf_directions(wl.system_id, wl.n, wl.L, 2)
    d_gpu, _, _ = O.density_response(P.reshape((1, wl.N) + g.shape), e[None], g, wl.n_electrons,
                                     wl.kT, dV, 1)
    d_ref, _, _ = O.density_response(Psi_o[None], eps_o[None], g, wl.n_electrons, wl.kT, dV, 1)
    print(f"{form} RR end-to-end drho rel err {rel(d_gpu, d_ref):.3e}")
    assert rel(d_gpu, d_ref) < 1e-4


@pytest.mark.parametrize("form", FORMS)
def test_rayleigh_ritz_multitile(form):
    g = O.Grid((20, 18, 13), (8.0, 7.2, 5.2))
    rng = np.random.default_rng(6)
    V = rng.uniform(-1, 0, g.shape)
    N = 150
    Y = rng.standard_normal((N,) + g.shape).astype(np.float32)
    eps_o, _ = O.rayleigh_ritz(Y.astype(np.float64), V, g)
    Yd = f32(Y)
    e = to_host(L.subspace_rayleigh_ritz(_grid(g), to_dev(V), Yd, prec=form))
    assert np.max(np.abs(e - eps_o)) < 1e-5 * np.max(np.abs(eps_o))
    P = to_host(Yd).reshape(N, -1)
    assert np.max(np.abs(P @ P.T - np.eye(N))) < 1e-5


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3"])
def test_autotune_keeps_the_response(c24, form):
    """The tuned K-split counts change only the order of the partial sums: the
    response after tuning matches the one before to rounding, and the oracle to
    the form's bound."""
    wl, g, V, eps, Psi = c24
    grid = L.Grid(tuple(g.n), tuple(g.L))
    occ = L.Occupation(1, wl.kT, wl.n_electrons)
    dV = grf_directions(wl.system_id, wl.n, wl.L, 4)
    dt = torch.float64 if form == "fp64" else torch.float32
    P = to_dev(Psi[None], dt)
    before, _, _ = L.density_response(grid, P, to_dev(eps[None]), occ, to_dev(dV), prec=form)
    before = to_host(before)
    tuned = L.autotune(grid, wl.N, 1, 4, prec=form)
    print(f"{form}: splits {tuned['splits']}, layouts {tuned['variants']}, ms {tuned['ms']}, "
          f"back-projection layout {tuned['backproj_layout']} ({tuned['backproj_ms']} ms)")
    after, _, _ = L.density_response(grid, P, to_dev(eps[None]), occ, to_dev(dV), prec=form)
    after = to_host(after)
    assert rel(after, before) < (1e-13 if form == "fp64" else 1e-6)
    ref, _, _ = O.density_response(to_host(P), eps[None], g, wl.n_electrons, wl.kT, dV, 1)
    assert rel(after, ref) < (1e-10 if form == "fp64" else BOUND[form])
    assert all(s >= 1 for s in tuned["splits"])
    if form == "bf16x3":
        assert tuned["backproj_layout"] in (0, 1) and min(tuned["backproj_ms"]) > 0.0
        L.context().set_backproj_layout(1)     # the library default, for the tests after this one
    else:
        assert tuned["backproj_ms"] == [0.0, 0.0]


def test_rayleigh_ritz_bf16x3_fresh_context_two_passes():
    """A context whose first call is a BF16X3 Rayleigh-Ritz of a block with
    dependent rows (copies and a combination: a second orthonormalisation pass
    over the explicit residuals, with the split rotation between the passes):
    the workspace sized for that call alone must hold the rotation's split
    operands and then the second Gram product.  The Ritz vectors come out
    orthonormal, spanning the independent rows and diagonalising H there."""
    g = O.Grid((32, 32, 32), (12.0, 12.0, 12.0))
    rng = np.random.default_rng(77)
    V = rng.uniform(-1, 0, g.shape)
    N = 256
    Y = rng.standard_normal((N,) + g.shape)
    Y[200] = Y[7]
    Y[201] = 2.0 * Y[30] - Y[31]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):                  # a new stream: a fresh context
        Yd = to_dev(Y, torch.float32)
        e = to_host(L.subspace_rayleigh_ritz(L.Grid(g.n, g.L), to_dev(V), Yd, prec="bf16x3"))
        side.synchronize()
    P = to_host(Yd).reshape(N, -1)
    assert np.all(np.isfinite(e))
    assert np.max(np.abs(P @ P.T - np.eye(N))) < 1e-5
    keep = [i for i in range(N) if i not in (200, 201)]
    Yk = to_host(to_dev(Y, torch.float32)).reshape(N, -1)[keep]
    assert np.linalg.norm(Yk - (Yk @ P.T) @ P) / np.linalg.norm(Yk) < 1e-5
    HP = O.hamiltonian_apply(P.reshape((N,) + g.shape), V, g).reshape(N, -1)
    assert np.max(np.abs(P @ HP.T - np.diag(e))) < 1e-4 * np.max(np.abs(e))
