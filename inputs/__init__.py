"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and bench.py.

This package only *draws* inputs (potentials, trial blocks, direction
functions).  It holds none of the method's arithmetic: no Hamiltonian, no
filter, no occupations, no response.  Both the oracle and the HIP path receive
the arrays it returns.
"""
from .gen import (  # noqa: F401
    Workload,
    SYSTEMS,
    make_workload,
    gaussian_wells,
    slab_offset,
    random_block,
    grf_directions,
    batched_systems,
)
