"""MI355X (gfx950) immersed boundary - lattice Boltzmann wetting step.

The compute path is libiblb.so (HIP kernels behind the C ABI of
include/iblb.h); this package only marshals arguments to it.
"""
from .binding import (  # noqa: F401
    EXPORTS, IBLB_BF16DEV, IBLB_BIT_BAND, IBLB_BIT_JUMP, IBLB_BIT_MACH, IBLB_BIT_RHO, IBLB_BIT_WALL,
    IBLB_E_DEVICE, IBLB_E_INVAL, IBLB_E_MESH, IBLB_E_STATE, IBLB_E_UNSTABLE, IBLB_E_WORKSPACE,
    IBLB_F16DEV, IBLB_F32, IBLB_F64, IBLB_FLAG_AUTOTUNE, IBLB_FLAG_FULL_U, IBLB_OK,
    IBLB_FLAG_GRAPH, IblbError, Simulation, band_tile, load, make_config, velocity_set, workspace_size,
)
