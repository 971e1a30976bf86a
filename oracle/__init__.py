"""CPU FP64 oracle of the IB-LBM time step (arXiv 2609.02298).

TEST INFRASTRUCTURE ONLY.  The product path never imports this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library.
"""
from .oracle import (  # noqa: F401
    OracleSim,
    build_oracle,
    lib,
    phi,
    equilibrium,
    collide_node,
    dense_A,
    interp,
    spread,
    dfc_lambda,
    body_half_kick,
    body_full_kick,
    body_euler,
    BGK, TRT, CMMRT,
    PERIODIC, BOUNCE_BACK, VEL_PARABOLIC, VEL_UNIFORM, ZERO_GRADIENT, ZOU_HE,
    DF, MDF, DFC, HAT, PESKIN4, FIXED, PRESCRIBED_SIN, FREE, IM_NONE, IM_FENG,
    VERLET, EULER_A1, UD_RIGID, UD_TAYLOR_GREEN,
)
