"""Seeded generators for the synthetic periodic systems the hot path runs on.

The paper benchmarks real materials (Pt nanoparticles, metal/semiconductor/
insulator stacks, doped oxide films; Sec. III).  Their structures and
pseudopotentials are not available here, so the workloads are stand-ins with
the same character: a local potential made of Gaussian wells (metal-like
attractive regions), optionally a slab with a constant offset (an
insulator-like region), a Gaussian random trial block and Gaussian random
field direction functions.

Every array is float64 in the "x fastest" layout ``[..., nz, ny, nx]``.
Random streams come from ``np.random.SeedSequence([221107894, system_id,
stream_id, ...])`` so that each piece (and each state of the trial block) can
be regenerated on its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

ROOT_SEED = 221107894

# stream ids
_S_WELLS = 0
_S_SLAB = 1
_S_BLOCK = 2
_S_GRF = 3
_S_SPIN = 4
_S_BATCH = 5


def _rng(system_id: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([ROOT_SEED, system_id, stream, *extra])))


# --------------------------------------------------------------------------
# named systems (sizes and physical parameters of the benchmark workloads)
# --------------------------------------------------------------------------
SYSTEMS = {
    # 24^3 grid, 10 bohr cell, 8 wells, 32 states / 24 electrons, degree 20, 4 directions
    "c24_n32": dict(system_id=1, n=24, L=10.0, nwells=8, N=32, n_electrons=24.0,
                    kT=0.01, degree=20, rank=4, slab=False, nspin=1),
    # 48^3 grid, 20 bohr, 64 wells, 256 states / 200 electrons, degree 30, 8 directions
    "c48_n256": dict(system_id=2, n=48, L=20.0, nwells=64, N=256, n_electrons=200.0,
                     kT=0.01, degree=30, rank=8, slab=False, nspin=1),
    # 64^3 grid, 28 bohr, 256 wells + 20%-volume slab at +0.5 Ha, 1024 states /
    # 800 electrons, kT 0.005, degree 40, 16 directions (the headline workload)
    "c64_n1024_slab": dict(system_id=3, n=64, L=28.0, nwells=256, N=1024,
                           n_electrons=800.0, kT=0.005, degree=40, rank=16,
                           slab=True, nspin=1),
    # 80^3 grid, 34 bohr, 512 wells, 2048 states / 1600 electrons, 20 directions
    "c80_n2048": dict(system_id=5, n=80, L=34.0, nwells=512, N=2048,
                      n_electrons=1600.0, kT=0.01, degree=40, rank=20, slab=False,
                      nspin=1),
}

WELL_DEPTH = (1.0, 3.0)      # Ha, uniform
WELL_WIDTH = (0.8, 1.5)      # bohr, uniform
SLAB_FRACTION = 0.2          # of the cell along z
SLAB_OFFSET = 0.5            # Ha
GRF_CORR_LENGTH = 1.5        # bohr
SPIN_DEPTH_SPREAD = 0.1      # down-channel well depths differ by U(-0.1, 0.1) relative


@dataclass
class Workload:
    name: str
    system_id: int
    n: tuple            # (nx, ny, nz)
    L: tuple            # (Lx, Ly, Lz) bohr
    N: int
    n_electrons: float
    kT: float
    degree: int
    rank: int
    nspin: int
    V: np.ndarray       # [nspin][nz][ny][nx]
    wells: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def h(self) -> tuple:
        return tuple(self.L[d] / self.n[d] for d in range(3))

    @property
    def dv(self) -> float:
        h = self.h
        return h[0] * h[1] * h[2]

    def block(self, states=None, dtype=np.float64, channel: int = 0) -> np.ndarray:
        return random_block(self.system_id, self.N, self.n, states=states,
                            dtype=dtype, channel=channel)

    def directions(self, rank: Optional[int] = None) -> np.ndarray:
        return grf_directions(self.system_id, self.n, self.L,
                              self.rank if rank is None else rank, nspin=self.nspin)


def _axis_images(coord: np.ndarray, centre: np.ndarray, width: np.ndarray, L: float):
    """exp(-(x - R + mL)^2 / (2 w^2)) summed over m in {-1, 0, 1}: [nwells, n]."""
    d = coord[None, :] - centre[:, None]
    out = np.zeros_like(d)
    for m in (-1.0, 0.0, 1.0):
        out += np.exp(-((d + m * L) ** 2) / (2.0 * width[:, None] ** 2))
    return out


def gaussian_wells(n, L, depth, width, pos) -> np.ndarray:
    """V(x) = -sum_a depth_a exp(-|x - R_a|^2 / (2 width_a^2)) over the 27 nearest
    periodic images of each well (a product of three per-axis image sums)."""
    nx, ny, nz = n
    Lx, Ly, Lz = L
    gx = _axis_images(np.arange(nx) * (Lx / nx), pos[:, 0], width, Lx)
    gy = _axis_images(np.arange(ny) * (Ly / ny), pos[:, 1], width, Ly)
    gz = _axis_images(np.arange(nz) * (Lz / nz), pos[:, 2], width, Lz)
    V = np.zeros((nz, ny, nx))
    for a in range(len(depth)):
        V -= depth[a] * (gz[a][:, None, None] * gy[a][None, :, None] * gx[a][None, None, :])
    return V


def slab_offset(n, L, z0: float, fraction=SLAB_FRACTION, offset=SLAB_OFFSET) -> np.ndarray:
    """+offset on the periodic slab z in [z0, z0 + fraction*Lz)."""
    nx, ny, nz = n
    Lz = L[2]
    z = np.arange(nz) * (Lz / nz)
    inside = np.mod(z - z0, Lz) < fraction * Lz
    V = np.zeros((nz, ny, nx))
    V[inside, :, :] = offset
    return V


def random_block(system_id: int, N: int, n, states=None, dtype=np.float64,
                 channel: int = 0) -> np.ndarray:
    """Gaussian trial block X [len(states)][nz][ny][nx]; state i uses its own stream,
    so any subset of states can be drawn without drawing the rest."""
    nx, ny, nz = n
    idx = range(N) if states is None else states
    idx = list(idx)
    out = np.empty((len(idx), nz, ny, nx), dtype=dtype)
    for row, i in enumerate(idx):
        out[row] = _rng(system_id, _S_BLOCK, channel, int(i)).standard_normal((nz, ny, nx))
    return out


def _inner(a, b, dv):
    return dv * float(np.dot(a.ravel(), b.ravel()))


def grf_directions(system_id: int, n, L, rank: int, nspin: int = 1,
                   ell: float = GRF_CORR_LENGTH) -> np.ndarray:
    """Direction functions u_k [rank][nspin][nz][ny][nx]: Gaussian random fields with
    covariance exp(-r^2 / (2 ell^2)), zero mean, orthonormal under
    <f, g> = dv * sum f g (summed over both channels for spin pairs)."""
    nx, ny, nz = n
    Lx, Ly, Lz = L
    dv = (Lx / nx) * (Ly / ny) * (Lz / nz)
    qx = 2 * np.pi * np.fft.fftfreq(nx, d=Lx / nx)
    qy = 2 * np.pi * np.fft.fftfreq(ny, d=Ly / ny)
    qz = 2 * np.pi * np.fft.fftfreq(nz, d=Lz / nz)
    q2 = qz[:, None, None] ** 2 + qy[None, :, None] ** 2 + qx[None, None, :] ** 2
    amp = np.exp(-q2 * ell * ell / 4.0)
    amp[0, 0, 0] = 0.0
    rng = _rng(system_id, _S_GRF)
    U = np.empty((rank, nspin, nz, ny, nx))
    for k in range(rank):
        for s in range(nspin):
            w = rng.standard_normal((nz, ny, nx))
            U[k, s] = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
            U[k, s] -= U[k, s].mean()
    # modified Gram-Schmidt in the (direct-sum) inner product
    for k in range(rank):
        for j in range(k):
            c = _inner(U[k], U[j], dv)
            U[k] -= c * U[j]
        U[k] /= np.sqrt(_inner(U[k], U[k], dv))
    return U


def make_workload(name: str) -> Workload:
    cfg = SYSTEMS[name]
    return _build(name, **cfg)


def _build(name, system_id, n, L, nwells, N, n_electrons, kT, degree, rank, slab,
           nspin, spin_spread=SPIN_DEPTH_SPREAD):
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    LL = (L, L, L) if np.isscalar(L) else tuple(L)
    rng = _rng(system_id, _S_WELLS)
    pos = rng.uniform(0.0, 1.0, size=(nwells, 3)) * np.asarray(LL)[None, :]
    depth = rng.uniform(*WELL_DEPTH, size=nwells)
    width = rng.uniform(*WELL_WIDTH, size=nwells)
    V0 = gaussian_wells(nn, LL, depth, width, pos)
    if slab:
        z0 = _rng(system_id, _S_SLAB).uniform(0.0, LL[2])
        V0 = V0 + slab_offset(nn, LL, z0)
    V = [V0]
    wells = dict(pos=pos, depth=depth, width=width)
    if nspin == 2:
        s = _rng(system_id, _S_SPIN).uniform(-spin_spread, spin_spread, size=nwells)
        V1 = gaussian_wells(nn, LL, depth * (1.0 + s), width, pos)
        if slab:
            V1 = V1 + slab_offset(nn, LL, z0)
        V.append(V1)
        wells["spin_scale"] = 1.0 + s
    return Workload(name=name, system_id=system_id, n=nn, L=LL, N=N,
                    n_electrons=float(n_electrons), kT=kT, degree=degree, rank=rank,
                    nspin=nspin, V=np.stack(V), wells=wells)


def batched_systems(count: int = 16, batch_id: int = 4) -> list:
    """Uneven spin-polarised systems: grids from {32,40,48,56}^3 with spacing
    0.4375 bohr, 64..512 states, 16..128 wells, 4..20 directions,
    N_e = 2 round(0.39 N)."""
    rng = _rng(batch_id, _S_BATCH)
    out = []
    for i in range(count):
        n = int(rng.choice([32, 40, 48, 56]))
        N = int(rng.integers(64, 513))
        nwells = int(rng.integers(16, 129))
        rank = int(rng.integers(4, 21))
        ne = 2.0 * round(0.39 * N)
        out.append(_build(f"batch{i}_n{n}_N{N}", system_id=1000 + i, n=n, L=0.4375 * n,
                          nwells=nwells, N=N, n_electrons=ne, kT=0.01, degree=30,
                          rank=rank, slab=False, nspin=2))
    return out
