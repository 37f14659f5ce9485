"""Seeded synthetic systems (atoms, contracted GTO shells, lattice, density).

This package builds the inputs that both the HIP path and the CPU oracle
consume.  It holds none of the exchange-build arithmetic: no integrals, no
normalisation, no screening, no pair lists.  Every random number is drawn
either from ``numpy.random.Generator(PCG64(seed))`` in a documented order or
from a counter-based hash (SplitMix64) keyed by the quantity it belongs to.
"""
from .generate import (  # noqa: F401
    System,
    molecule8,
    diamond_cell,
    cluster_k4,
    cluster_batch,
    request_stream,
    random_cluster,
    diamond_supercell,
    density_blocks,
    density_series,
    perturb_density,
    splitmix64,
    hash_uniform,
    nfunc,
    nao_radial,
    nao_basis,
)
