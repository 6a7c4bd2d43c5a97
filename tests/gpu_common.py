"""Shared helpers of the GPU parity tests: seeded systems whose oracle-side
inputs (Ritz pairs, filter bounds) are produced by the oracle only, then copied
to the device for the HIP path."""
from __future__ import annotations

import numpy as np
import torch

import oracle as O
from inputs import make_workload

DEV = "cuda"


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


def to_host(t):
    return t.detach().double().cpu().numpy()


def filter_bounds(V, g: O.Grid, eps=None):
    """Upper bound of the spectrum (Gershgorin: sum 2/h^2 + max V) and, from a
    previous Rayleigh-Ritz, a = largest Ritz value and a0 = below the smallest."""
    b = sum(2.0 / hd ** 2 for hd in g.h) + float(V.max())
    if eps is None:
        a0 = float(V.min()) - 0.1
        a = a0 + 0.25 * (b - a0)
    else:
        a = float(eps[-1])
        a0 = float(eps[0]) - 0.2
    return a, b, a0


def oracle_subspace(name, passes=2, degrees=(8, None), states=None):
    """Ritz pairs of the named workload after a few oracle ChFSI passes from the
    seeded Gaussian block (a low first degree keeps the block well conditioned)."""
    wl = make_workload(name)
    g = O.Grid(wl.n, wl.L)
    V = wl.V[0]
    X = wl.block() if states is None else wl.block(states=range(states))
    eps = None
    for p in range(passes):
        deg = degrees[p] if p < len(degrees) and degrees[p] else wl.degree
        a, b, a0 = filter_bounds(V, g, eps)
        Y = O.chebyshev_filter(X, V, g, deg, a, b, a0)
        eps, X = O.rayleigh_ritz(Y, V, g)
    return wl, g, V, eps, X
