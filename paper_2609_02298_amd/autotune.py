"""Launch-shape autotuner for the collide-stream kernel and the IB pass.

Times candidate tile shapes through the C ABI (HIP events around each
collide-stream launch on the library's stream) on a body-free lattice of the
same size, collision model and precision as the workload, and keeps the
fastest.  Results are cached in memory and in a JSON table keyed by
(precision, collision, nx, ny); the table shipped with the package
(launch_table.json, written on an MI355X by ``python -m
paper_2609_02298_amd.autotune --write PATH``) is loaded first, so tuned
workloads start without re-tuning.

The IB pass runs one workgroup per body; its size (256, 512 or 1024
threads) is tuned per body description and precision by timing the pass on
the workload itself (``tune_ib``).  For a workload with bodies the tile
shape is then chosen by the time of whole steps (``tune_step``): the tiles
that wait for the IB pass in a pipelined step are whole tiles, so wide tiles
can lengthen the step.  ``--ib`` tunes both for the benchmark's workloads.
"""
from __future__ import annotations

import itertools
import json
import os

from . import ib_lbm as ib

DEFAULT_CANDIDATES = [
    dict(block_x=bx, block_y=by, rows_per_thread=rpt, xcd_remap=remap)
    for remap, bx, by, rpt in itertools.product((1, 0), (64, 128, 256, 512, 1024), (1, 2, 4), (1, 2, 4))
    if bx * by <= 1024
]

REFINE = 6  # candidates timed again before the choice

_cache: dict = {}
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "launch_table.json")


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


def lookup(nx, ny, collision, precision):
    """The tuned shape for this lattice from the shipped table or an earlier
    tune() in this process, or None."""
    if not _cache:
        load_cache(TABLE)
    e = _cache.get(_key(nx, ny, collision, precision))
    return dict(e["shape"]) if e else None


def tune(nx, ny, collision, precision, candidates=None, steps=40, stream=None) -> dict:
    """Best launch shape for this lattice (from the table, else timed)."""
    k = _key(nx, ny, collision, precision)
    if not _cache:
        load_cache(TABLE)
    if k in _cache:
        return dict(_cache[k]["shape"])
    # one timing of every candidate, then the fastest few again, longer and
    # three times each: single timings of near-equal shapes differ by a few
    # per cent from run to run
    first = sorted(((time_shape(nx, ny, collision, precision, sh, steps, stream), i)
                    for i, sh in enumerate(candidates or DEFAULT_CANDIDATES)))
    cands = candidates or DEFAULT_CANDIDATES
    best = None
    for _, i in first[:REFINE]:
        ts = sorted(time_shape(nx, ny, collision, precision, cands[i], 3 * steps, stream)
                    for _ in range(3))
        if best is None or ts[1] < best[0]:
            best = (ts[1], cands[i])
    _cache[k] = {"shape": best[1], "us": best[0]}
    return dict(best[1])


IB_CANDIDATES = (256, 512, 1024)


def _ib_key(case, precision):
    """IB-pass entries are keyed by what the pass's work depends on: the
    body (scheme, kernel, markers, MDF bounds) and the precision."""
    parts = []
    for b in case.get("bodies", []):
        nb = int(b.get("n_markers", 0)) or int(round(3.141592653589793 * b["diameter"]))
        parts.append(f"s{b.get('scheme', 0)}k{b.get('kernel', 0)}n{nb}"
                     f"m{b.get('mdf_iters', 5)}t{b.get('mdf_tol', 0.0):g}")
    return f"ib-p{precision}-" + "-".join(parts)


def time_ib(case, precision, threads, steps=40, shape=None) -> float:
    """Average IB-pass duration in microseconds (HIP events around each pass
    of plain, unpipelined steps) with the given workgroup size."""
    s = ib.Sim(case, precision=precision)
    try:
        s.set_launch(**dict(shape or {}, ib_threads=threads))
        s.set_overlap(False)
        s.step(4)
        s.sync()
        s.timing(True)
        s.step(steps)
        ms, n = s.timing_read(1)
    finally:
        s.close()
    return ms / max(n, 1) * 1e3


def tune_ib(case, precision, candidates=IB_CANDIDATES, steps=40) -> int:
    """Best IB workgroup size for the case's bodies (from the table, else
    timed on this case)."""
    if not case.get("bodies"):
        return 0
    k = _ib_key(case, precision)
    if not _cache:
        load_cache(TABLE)
    if k in _cache:
        return int(_cache[k]["ib_threads"])
    shape = tune(case["nx"], case["ny"], case["collision"], precision)
    best = None
    for t in candidates:
        us = time_ib(case, precision, t, steps, shape)
        if best is None or us < best[0]:
            best = (us, t)
    _cache[k] = {"ib_threads": best[1], "us": best[0]}
    return best[1]


# Shapes tried for whole pipelined steps: the kernel's best shape plus
# narrow tiles, which keep the rectangle of tiles that wait for the IB pass
# (rounded to whole tiles) small.
STEP_CANDIDATES = [
    dict(block_x=bx, block_y=by, rows_per_thread=rpt, xcd_remap=1)
    for bx, by, rpt in ((64, 1, 1), (64, 1, 2), (64, 2, 1), (64, 2, 2), (64, 4, 1), (128, 1, 1),
                        (128, 1, 2), (128, 2, 1), (256, 1, 1), (256, 1, 2))
]


def time_step(case, precision, shape, steps=100, warmup=20) -> float:
    """Wall-clock microseconds per step of the workload itself (its bodies,
    faces and pipelining), with the given launch shape."""
    import time
    s = ib.Sim(case, precision=precision)
    try:
        s.set_launch(**shape)
        s.step(warmup)
        s.sync()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        return (time.perf_counter() - t0) / steps * 1e6
    finally:
        s.close()


def tune_step(case, precision, steps=100) -> dict:
    """Launch shape and IB workgroup size for a workload with bodies, chosen
    by whole-step time: in a pipelined step the tiles that wait for the IB
    pass are whole tiles, so the shape that is fastest for the collide-stream
    alone can lengthen the step."""
    base = dict(tune(case["nx"], case["ny"], case["collision"], precision))
    if not case.get("bodies"):
        return base
    ibt = tune_ib(case, precision)
    k = "step-" + _key(case["nx"], case["ny"], case["collision"], precision) + "-" + _ib_key(case, precision)
    if k in _cache:
        return dict(_cache[k]["shape"], ib_threads=ibt)
    cands = [base] + [c for c in STEP_CANDIDATES if c != base]
    best = None
    for sh in cands:
        sh = dict(sh, ib_threads=ibt)
        t = sorted(time_step(case, precision, sh, steps) for _ in range(2))[0]
        if best is None or t < best[0]:
            best = (t, sh)
    _cache[k] = {"shape": {n: v for n, v in best[1].items() if n != "ib_threads"}, "us_per_step": best[0]}
    return dict(best[1])


def _bench_cases():
    """The bodies the benchmark steps: the headline cylinder with fixed and
    adaptive MDF, and the largest sweep case."""
    import ib_cases
    head = ib_cases.unsteady_cylinder(scheme="MDF", kernel="P4", collision="TRT", re=100.0)
    adapt = ib_cases.unsteady_cylinder(scheme="MDF", kernel="P4", collision="TRT", re=100.0)
    adapt["bodies"][0].update(ib_cases.ADAPTIVE_MDF)
    sweep = ib_cases.sweep_cases(256, seed=0)
    big = max(sweep, key=lambda c: c["nx"] * c["ny"])
    return [head, adapt, big]


def _main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune the collide-stream launch shape of workloads")
    ap.add_argument("--write", required=True, help="JSON table to write")
    ap.add_argument("lattices", nargs="*", default=["2000x800", "4096x4096"],
                    help="NXxNY entries, tuned for every collision model and precision")
    ap.add_argument("--fresh", action="store_true",
                    help="time every entry again instead of starting from the shipped table")
    ap.add_argument("--ib", action="store_true",
                    help="also tune the IB-pass workgroup size of the benchmark's bodies")
    args = ap.parse_args(argv)
    ib.load_library()
    if args.fresh:
        _cache.clear()
        _cache["_fresh"] = True  # keeps the shipped table from being loaded on lookup
    for spec in args.lattices:
        nx, ny = (int(v) for v in spec.lower().split("x"))
        for prec in (ib.FP32_SHIFTED, ib.FP64):
            for col in (ib.BGK, ib.TRT, ib.CMMRT):
                sh = tune(nx, ny, col, prec)
                print(f"{nx}x{ny} precision {prec} collision {col}: {sh} "
                      f"{_cache[_key(nx, ny, col, prec)]['us']:.1f} us", flush=True)
    if args.ib:
        for case in _bench_cases():
            for prec in (ib.FP32_SHIFTED, ib.FP64):
                t = tune_ib(case, prec)
                k = _ib_key(case, prec)
                print(f"{case['name']} IB {k}: {t} threads {_cache[k]['us']:.1f} us", flush=True)
                sh = tune_step(case, prec)
                ks = "step-" + _key(case["nx"], case["ny"], case["collision"], prec) + "-" + k
                print(f"{case['name']} step {ks}: {sh} {_cache[ks]['us_per_step']:.2f} us per step",
                      flush=True)
    _cache.pop("_fresh", None)
    save_cache(args.write)


if __name__ == "__main__":
    _main()
