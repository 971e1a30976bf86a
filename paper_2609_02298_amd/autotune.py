"""Launch-shape autotuner for the collide-stream kernel.

Times candidate tile shapes through the C ABI (HIP events around each
collide-stream launch on the library's stream) on a body-free lattice of the
same size, collision model and precision as the workload, and keeps the
fastest.  Results are cached in memory and, optionally, in a JSON file keyed
by (precision, collision, nx, ny).
"""
from __future__ import annotations

import itertools
import json
import os

from . import ib_lbm as ib

DEFAULT_CANDIDATES = [
    dict(block_x=bx, block_y=by, rows_per_thread=rpt, xcd_remap=1)
    for bx, by, rpt in itertools.product((64, 128, 256), (1, 2, 4), (1, 2, 4))
    if bx * by <= 1024
]

_cache: dict = {}


def _key(nx, ny, collision, precision):
    return f"p{precision}-c{collision}-{nx}x{ny}"


def load_cache(path: str) -> None:
    try:
        with open(path) as fh:
            _cache.update(json.load(fh))
    except (OSError, ValueError):
        pass


def save_cache(path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(_cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_shape(nx, ny, collision, precision, shape, steps=40, stream=None) -> float:
    """Average collide-stream launch time in microseconds."""
    case = dict(nx=nx, ny=ny, collision=collision, tau=0.8, bc=(ib.PERIODIC,) * 4)
    s = ib.Sim(case, precision=precision, stream=stream)
    try:
        s.set_launch(**shape)
        s.step(4)
        s.sync()
        s.timing(True)
        s.step(steps)
        ms, n = s.timing_read(0)
    finally:
        s.close()
    return ms / max(n, 1) * 1e3


def tune(nx, ny, collision, precision, candidates=None, steps=40, stream=None) -> dict:
    """Best launch shape for this lattice (cached)."""
    k = _key(nx, ny, collision, precision)
    if k in _cache:
        return dict(_cache[k]["shape"])
    best = None
    for sh in candidates or DEFAULT_CANDIDATES:
        t = time_shape(nx, ny, collision, precision, sh, steps, stream)
        if best is None or t < best[0]:
            best = (t, sh)
    _cache[k] = {"shape": best[1], "us": best[0]}
    return dict(best[1])
