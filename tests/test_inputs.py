"""The seeded workload generators: reproducible, shaped as documented, and the
Gaussian wells equal a direct 27-image sum."""
import itertools

import numpy as np

from inputs import SYSTEMS, batched_systems, gaussian_wells, grf_directions, make_workload, random_block


def test_wells_equal_direct_image_sum():
    n, L = (5, 4, 6), (3.0, 2.0, 3.5)
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 1, (3, 3)) * np.asarray(L)
    d = rng.uniform(1, 3, 3)
    w = rng.uniform(0.8, 1.5, 3)
    V = gaussian_wells(n, L, d, w, pos)
    ref = np.zeros((n[2], n[1], n[0]))
    for z, y, x in itertools.product(range(n[2]), range(n[1]), range(n[0])):
        p = np.array([x * L[0] / n[0], y * L[1] / n[1], z * L[2] / n[2]])
        for a in range(3):
            for m in itertools.product((-1, 0, 1), repeat=3):
                r = p - pos[a] + np.array(m) * np.asarray(L)
                ref[z, y, x] -= d[a] * np.exp(-r @ r / (2 * w[a] ** 2))
    assert np.max(np.abs(V - ref)) < 1e-12


def test_block_states_independent_and_reproducible():
    full = random_block(7, 6, (4, 5, 3))
    part = random_block(7, 6, (4, 5, 3), states=[4, 1])
    assert np.array_equal(part[0], full[4]) and np.array_equal(part[1], full[1])
    assert np.array_equal(random_block(7, 6, (4, 5, 3)), full)


def test_grf_directions_orthonormal_zero_mean():
    n, L = (8, 8, 8), (4.0, 4.0, 4.0)
    dv = (L[0] / 8) ** 3
    for nspin in (1, 2):
        U = grf_directions(3, n, L, 5, nspin=nspin)
        G = dv * np.einsum("ksxyz,lsxyz->kl", U, U)
        assert np.max(np.abs(G - np.eye(5))) < 1e-12
        assert np.max(np.abs(U.reshape(5, nspin, -1).sum(-1))) < 1e-10


def test_named_systems_shapes():
    wl = make_workload("c24_n32")
    assert wl.V.shape == (1, 24, 24, 24) and wl.N == 32 and wl.rank == 4
    assert set(SYSTEMS) >= {"c24_n32", "c48_n256", "c64_n1024_slab", "c80_n2048"}
    bs = batched_systems(4)
    for s in bs:
        assert s.nspin == 2 and s.V.shape[0] == 2 and 64 <= s.N <= 512
        assert s.n[0] in (32, 40, 48, 56) and 4 <= s.rank <= 20
