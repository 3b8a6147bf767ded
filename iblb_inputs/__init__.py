"""Seeded synthetic inputs (meshes, boxes, workloads) shared by the oracle
tests and the GPU library's tests and benchmark.  Holds none of the method's
arithmetic."""
from . import configs, mesh  # noqa: F401
from .configs import (  # noqa: F401
    BF16DEV, F16DEV, F32, F64, Z_PERIODIC, Z_WALLS, Box, Droplet, Workload,
)
