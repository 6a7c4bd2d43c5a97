"""Brillouin-zone sampling of the response (density_response_bz) against the
FP64 oracle: complex k-point subspaces (the lowest Bloch states of a small cell,
and random orthonormal complex blocks spanning several 128-row tiles), unequal
weights, one and two channels, the three precision forms; and k = 0 with real
states against the real path.  Every oracle input comes from the oracle or the
seeded generators."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import rel, to_dev, to_host
from tests.pins import small_wells

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402

BOUND = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-6}


def _grid(g: O.Grid):
    return L.Grid(tuple(g.n), tuple(g.L))


def _realified(Psi):
    """[nspin][nk][N][...] complex -> [nspin][nk][2][N][...] real (Re rows, Im rows)."""
    return np.stack([Psi.real, Psi.imag], axis=2)


def _bloch_case(nspin):
    g = O.Grid((10, 9, 8), (5.0, 4.6, 4.1))
    V = small_wells(g.n, g.L, 51, nwells=3)
    ks = [(0.0, 0.0, 0.0), (0.5, -0.3, 0.2), (-0.9, 0.4, 0.7)]
    w = np.array([0.2, 0.5, 0.3])
    N = 40
    rng = np.random.default_rng(52)
    Psi, eps = [], []
    for c in range(nspin):
        Vc = V + 0.05 * c * rng.standard_normal(g.shape)
        st = [O.lowest_bloch_states(Vc, g, k, N) for k in ks]
        eps.append(np.stack([e for e, _ in st]))
        Psi.append(np.stack([p for _, p in st]))
    ne = 0.6 * N * 2.0
    return g, np.stack(Psi), np.stack(eps), w, ne, 0.02


def _random_case(nspin, N=150, nk=2, seed=53):
    """Random orthonormal complex subspaces (the realified rows span 300 > 2 tiles)
    on a ragged grid, sorted energies across mu."""
    g = O.Grid((20, 18, 13), (8.0, 7.2, 5.2))
    rng = np.random.default_rng(seed)
    Psi = np.empty((nspin, nk, N) + g.shape, dtype=np.complex128)
    eps = np.empty((nspin, nk, N))
    for c in range(nspin):
        for k in range(nk):
            Z = rng.standard_normal((g.M, N)) + 1j * rng.standard_normal((g.M, N))
            Q, _ = np.linalg.qr(Z)
            Psi[c, k] = Q.T.reshape((N,) + g.shape)
            eps[c, k] = np.sort(rng.uniform(-1.5, 0.8, N))
    w = rng.uniform(0.5, 1.5, nk)
    return g, Psi, eps, w / w.sum(), 0.39 * 2 * N, 0.01


@pytest.mark.parametrize("nspin", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["bloch", "random"])
def test_density_response_bz(case, prec, nspin):
    g, Psi, eps, w, ne, kT = _bloch_case(nspin) if case == "bloch" else _random_case(nspin)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Pd = to_dev(_realified(Psi), dt)
    Ph = to_host(Pd)                                  # the form's storage, in FP64
    Psi_form = Ph[:, :, 0] + 1j * Ph[:, :, 1]
    dV = np.random.default_rng(54).standard_normal((3, nspin) + g.shape)
    occ = L.Occupation(nspin, kT, ne)
    drho, mu, dmu = L.density_response_bz(_grid(g), Pd, to_dev(eps), to_dev(w), occ, to_dev(dV),
                                          prec=prec)
    ref, mu_o, dmu_o = O.density_response_bz(Psi_form, eps, w, g, ne, kT, dV, nspin)
    err = max(rel(to_host(drho)[q, c], ref[q, c]) for q in range(3) for c in range(nspin))
    print(f"{case} {prec} nspin {nspin}: delta rho rel err {err:.2e}")
    assert abs(float(mu.item()) - mu_o) < 1e-12
    assert np.max(np.abs(to_host(dmu) - dmu_o)) < 10 * BOUND[prec] * max(1.0, np.max(np.abs(dmu_o)))
    assert err < BOUND[prec]
    # the zone-averaged traceless condition: delta rho integrates to zero (to the
    # orthonormality of the stored states: about 1e-7 for FP32 storage)
    tol = 1e-9 if prec == "fp64" else 1e-6
    for q in range(3):
        total = g.dv * float(to_host(drho)[q].sum())
        assert abs(total) < tol * g.dv * float(np.abs(to_host(drho)[q]).sum())


def test_density_response_bz_gamma_is_the_real_path():
    """One k-point at k = 0 with real states (imaginary rows zero) gives the
    real density_response."""
    g, Psi, eps, w, ne, kT = _random_case(1, N=130, nk=1, seed=55)
    Q, _ = np.linalg.qr(np.random.default_rng(56).standard_normal((g.M, 130)))
    R = Q.T.reshape((130,) + g.shape)
    dV = np.random.default_rng(57).standard_normal((2, 1) + g.shape)
    occ = L.Occupation(1, kT, ne)
    a, mu_a, dmu_a = L.density_response(_grid(g), to_dev(R[None]), to_dev(eps[0]), occ, to_dev(dV))
    Pbz = np.stack([R, np.zeros_like(R)])[None, None]
    b, mu_b, dmu_b = L.density_response_bz(_grid(g), to_dev(Pbz), to_dev(eps), to_dev([1.0]), occ,
                                           to_dev(dV))
    assert rel(to_host(b), to_host(a)) < 1e-12
    assert abs(float(mu_a.item()) - float(mu_b.item())) < 1e-13
