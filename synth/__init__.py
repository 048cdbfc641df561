"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package only builds atomic structures (lattices, noise, strain, species
assignment, random packings) and draws seeded random numbers. It contains none
of the potential's arithmetic: no descriptors, basis functions, networks,
forces or losses.
"""

from .structures import (  # noqa: F401
    Batch,
    make_batch,
    bcc_structure,
    fcc_structure,
    random_packing,
    pack,
)
from .workloads import WORKLOADS, Workload, workload_batch, draw_theta, random_targets  # noqa: F401
