"""Oracle comparisons at the sizes the bench runs, in its launch configurations:
the Hartree kernel on whole 64^3 and 80^3 grids (the LDS axis path at 64 points,
the direct path above), the FP64 Chebyshev filter of the whole 64^3 / 1024-state
block at degree 40 on sampled states, Rayleigh-Ritz of a 64^3 / 1024-state block
(Ritz values against the oracle's Householder QR and dense eigh), and the
response with the Fermi level in a gap.  Every oracle input comes from the seeded input
generators and the oracle itself."""
import numpy as np
import pytest

import oracle as O
from inputs import grf_directions, make_workload
from tests.gpu_common import rel, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2211_07894_amd as L  # noqa: E402


def _grid(g: O.Grid):
    return L.Grid(tuple(g.n), tuple(g.L))


# ------------------------------------------------------------------ a9 Hartree kernel
@pytest.mark.parametrize("name,r", [("c64_n1024_slab", 16), ("c80_n2048", 20)])
def test_hartree_kernel_full_size(name, r):
    """K_c of the workload's GRF directions (Eq. (3)), all directions in one call
    as the residual derivative launches it: 64 points per axis take the LDS-staged
    axis passes, 80 the direct ones.  Element-wise 1e-12 relative per direction."""
    wl = make_workload(name)
    g = O.Grid(wl.n, wl.L)
    U = grf_directions(wl.system_id, wl.n, wl.L, r)[:, 0]
    dV = to_host(L.hartree_kernel(_grid(g), to_dev(U)))
    errs = [rel(dV[k], O.hartree_kernel(U[k], g)) for k in range(r)]
    print(f"{name}: Hartree rel err max {max(errs):.2e} over {r} directions")
    assert max(errs) < 1e-12


# ------------------------------------------------------------------ a2 filter, FP64, 64^3 / 1024
def test_chfsi_filter_fp64_full_size_sampled():
    """The FP64 filter of degree 40 on the whole 1024-state block (the bench's
    launch), against the oracle's three-term recurrence on six sampled states
    (the filter acts on each state alone)."""
    wl = make_workload("c64_n1024_slab")
    g = O.Grid(wl.n, wl.L)
    V = wl.V[0]
    b = sum(2.0 / hd ** 2 for hd in g.h) + float(V.max())
    a0 = float(V.min()) - 0.1
    a = a0 + 0.25 * (b - a0)
    N = wl.N
    X = torch.empty((N,) + g.shape, dtype=torch.float64, device="cuda")
    for s in range(0, N, 128):
        X[s:s + 128] = to_dev(wl.block(states=range(s, s + 128)))
    Y = L.chfsi_filter(_grid(g), to_dev(V), X, wl.degree, a, b, a0)
    idx = [0, 1, 257, 600, 1022, 1023]
    ref = O.chebyshev_filter(wl.block(states=idx), V, g, wl.degree, a, b, a0)
    got = to_host(Y[idx])
    errs = [rel(got[k], ref[k]) for k in range(len(idx))]
    print(f"FP64 filter 64^3/1024 degree {wl.degree}: sampled rel err max {max(errs):.2e}")
    assert max(errs) < 1e-12


# ------------------------------------------------------------------ a3 Rayleigh-Ritz, 64^3 / 1024
def test_rayleigh_ritz_fp64_full_size():
    """Rayleigh-Ritz of a 1024-state block on the 64^3 workload: the seeded
    Gaussian block with row norms graded over eight orders of magnitude (as a
    filtered block's are), so the column scaling and the block Jacobi
    eigensolver run at full size.  Ritz values within 1e-10 relative of the
    oracle's (Householder QR, dense eigh); Ritz vectors orthonormal and with the
    oracle's Ritz residual property."""
    wl = make_workload("c64_n1024_slab")
    g = O.Grid(wl.n, wl.L)
    V = wl.V[0]
    N = wl.N
    Y = wl.block()
    Y *= (10.0 ** (-8.0 * np.arange(N) / (N - 1)))[:, None, None, None]
    e_ref, _ = O.rayleigh_ritz(Y, V, g)
    Yd = to_dev(Y)
    del Y
    e = to_host(L.subspace_rayleigh_ritz(_grid(g), to_dev(V), Yd))
    err = float(np.max(np.abs(e - e_ref)) / np.max(np.abs(e_ref)))
    P = Yd.reshape(N, -1)
    orth = float(torch.max(torch.abs(P @ P.T - torch.eye(N, dtype=P.dtype, device="cuda"))))
    print(f"RR 64^3/1024: Ritz value rel err {err:.2e}, orthonormality {orth:.2e}")
    assert err < 1e-10
    assert orth < 1e-12
    # Ritz property on sampled vectors: H psi_i - e_i psi_i orthogonal to the subspace
    idx = [0, 511, 1023]
    Hpsi = L.hamiltonian_apply(_grid(g), to_dev(V), Yd[idx].contiguous()).reshape(len(idx), -1)
    Rz = Hpsi - torch.from_numpy(e[idx]).to("cuda")[:, None] * P[idx]
    assert float(torch.max(torch.abs(P @ Rz.T))) < 1e-10 * float(np.max(np.abs(e_ref)))


# ------------------------------------------------------------------ a7 mu' with mu in a gap
@pytest.mark.parametrize("nspin", [1, 2])
def test_density_response_mu_in_gap(nspin):
    """A gapped spectrum (occupied band [-2, -1] Ha, empty band [1, 2] Ha) at kT
    = 1e-3: mu lies in the gap, every occupation is 0 or 1 to rounding, and the
    sums of the traceless condition come from the band edges only (sum f' of
    order 1e-11).  The bisection ends where the count first reaches N_e, about
    35 kT below the empty band, so f' there never underflows and mu' is the
    ratio of those tiny sums on both sides (the zero branch for a vanishing sum
    guards a case the bisection cannot produce).  mu is not unique there: the
    count reaches N_e to rounding over a range whose end depends on the order
    of the sum, so mu is checked by its electron count and its place in the
    gap, and mu' against the oracle's shift at the same mu.  delta rho comes from
    the occupied-empty divided differences and must match the oracle's."""
    g = O.Grid((20, 18, 13), (8.0, 7.2, 5.2))
    N = 150
    rng = np.random.default_rng(77)
    Q, _ = np.linalg.qr(rng.standard_normal((g.M, N)))
    Psi = np.stack([Q.T.reshape((N,) + g.shape)] * nspin)
    n_occ = 60
    eps = np.concatenate([np.sort(rng.uniform(-2.0, -1.0, n_occ)),
                          np.sort(rng.uniform(1.0, 2.0, N - n_occ))])
    eps = np.stack([eps + 0.01 * c for c in range(nspin)])
    ne = 2.0 * n_occ          # one channel: two per state; two channels: one each
    kT = 1e-3
    dV = rng.standard_normal((3, nspin) + g.shape)
    occ = L.Occupation(nspin, kT, ne)
    drho, mu, dmu = L.density_response(_grid(g), to_dev(Psi), to_dev(eps), occ, to_dev(dV))
    ref, mu_o, dmu_o = O.density_response(Psi, eps, g, ne, kT, dV, nspin)
    _, _, fp = O.fermi_dirac(eps, mu_o, kT)
    print(f"mu in gap, nspin {nspin}: mu {float(mu.item()):.6f}, sum f' {fp.sum():.2e}")
    mu_g = float(mu.item())
    assert eps[:, n_occ - 1].max() < mu_g < eps[:, n_occ].min()
    s = O.spin_factor(nspin)
    assert abs(s * float(np.sum(O.fermi_dirac(eps, mu_g, kT)[0])) - ne) < 1e-12 * ne
    fp_g = [O.fermi_dirac(eps[c], mu_g, kT)[2] for c in range(nspin)]
    for k in range(3):
        Hps = [O.projected_perturbation(Psi[c], dV[k, c]) for c in range(nspin)]
        dmu_at_g = O.fermi_shift(Hps, fp_g)
        assert abs(float(to_host(dmu)[k]) - dmu_at_g) < 1e-9 * max(1.0, abs(dmu_at_g))
    err = max(rel(to_host(drho)[k, c], ref[k, c]) for k in range(3) for c in range(nspin))
    print(f"mu in gap, nspin {nspin}: delta rho rel err {err:.2e}")
    assert err < 1e-10
