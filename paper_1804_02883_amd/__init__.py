"""MI355X-native hybrid Lattice Boltzmann / External Potential Dynamics step.

The simulation runs in libepdlb.so (HIP kernels for gfx950 behind a C ABI,
declared in include/epdlb.h); `binding` exposes that ABI to Python.
"""
from .binding import (  # noqa: F401
    Simulation, Batch, Trainer, Fluid3D, Densities3D, make_params, mrt_gammas, load_library, LIB_PATH, EpdlbError, EPDLB_NN_PARAMS,
    EPDLB_STAGE_ADVECT_UPDATE, EPDLB_STAGE_DENSITIES, EPDLB_STAGE_FORCE, EPDLB_STAGE_LB,
    EPDLB_AUX_STILDE, EPDLB_AUX_S, EPDLB_AUX_FORCE,
)
