"""MI355X-native immersed-boundary lattice Boltzmann hot path (arXiv 2609.02298).

The compute path is ``libib_lbm.so`` (hand-written gfx950 HIP kernels behind
the C ABI of ``include/ib_lbm.h`` and ``include/ib_lbm_server.h``); this
package holds the thin ctypes binding, the build script, the autotuner and
the client-side drivers of the serving loop.
"""
from .ib_lbm import (  # noqa: F401
    Batch, Server, Sim, IbLbmError, PENDING, load_library, footprint, stream_copy, LIB_PATH, EXPORTS,
    FP64, FP32_SHIFTED, BGK, TRT, CMMRT, PERIODIC, BOUNCE_BACK, VEL_PARABOLIC, VEL_UNIFORM,
    ZERO_GRADIENT, ZOU_HE, DF, MDF, DFC, HAT, PESKIN4, FIXED, PRESCRIBED_SIN, FREE, IM_NONE, IM_FENG,
    SPREAD_GATHER, SPREAD_ATOMIC, VERLET, EULER_A1, UD_RIGID, UD_TAYLOR_GREEN,
)
