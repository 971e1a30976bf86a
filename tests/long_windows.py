"""Whole-step parity over long windows: the benchmark configurations 2-4 at
full size for 2,000 steps, the GPU against the FP64 oracle.

Too long for the test suite (the single-threaded oracle takes 0.3-1 s per
full-size step), so it runs in two halves:

    python tests/long_windows.py gpu --out DIR      # on an MI355X: GPU runs
    python tests/long_windows.py compare --gpu DIR  # anywhere: oracle runs, comparison
    python tests/long_windows.py table --gpu DIR    # the comparison again, from the kept runs

The GPU half stores, for every case, the body states every 100 steps and, at
the end, the density and velocity on every fourth node in x and y (full
precision) with the field norms over all nodes.  The compare half runs the
oracle on the same seeded cases (one process per case), keeps its histories
and fields beside the GPU files (working output, regenerated on every run,
nothing committed) and prints the largest differences.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import ib_cases  # noqa: E402

STEPS = 2000
EVERY = 100
SUB = 4
KEYS = ("fx", "fy", "torque", "xc", "yc", "vx", "vy", "slip_mean")


def cases():
    """(name, case, GPU precisions): configurations 2, 3 and 4 (single body
    and pair) with their stated schemes and lattices."""
    return [
        ("config2-unsteady-cylinder-MDF-P4-TRT",
         ib_cases.unsteady_cylinder(scheme="MDF", kernel="P4", collision="TRT", re=100.0), ("fp64", "fp32")),
        ("config3-oscillating-cylinder", ib_cases.oscillating_cylinder(), ("fp64",)),
        ("config4-sedimentation-single", ib_cases.sedimentation(pair=False), ("fp64",)),
        ("config4-sedimentation-pair", ib_cases.sedimentation(pair=True), ("fp64",)),
    ]


def summarise(rho, ux, uy):
    sub = (slice(None, None, SUB), slice(None, None, SUB))
    speed = np.hypot(ux, uy)
    return dict(rho_sub=rho[sub], ux_sub=ux[sub], uy_sub=uy[sub],
                norms=np.array([np.abs(rho - 1.0).max(), speed.max(), np.sqrt((speed ** 2).mean())]))


def run_gpu(out):
    import paper_2609_02298_amd as ib
    os.makedirs(out, exist_ok=True)
    for name, case, precs in cases():
        for pname in precs:
            prec = ib.FP64 if pname == "fp64" else ib.FP32_SHIFTED
            t0 = time.time()
            sim = ib.Sim(case, precision=prec)
            nb = len(case["bodies"])
            hist = []
            for t in range(EVERY, STEPS + 1, EVERY):
                sim.step(t - sim.steps_done)
                hist.append([[sim.forces(b, check=False)[k] for k in KEYS] for b in range(nb)])
            rho, ux, uy = sim.fields()
            d = summarise(rho, ux, uy)
            np.savez(os.path.join(out, f"{name}-{pname}.npz"), hist=np.array(hist), **d)
            print(f"{name} {pname}: {STEPS} steps in {time.time() - t0:.1f} s, "
                  f"fused {sim.fused()}, pipelined {sim.overlap()[0]}", flush=True)
            sim.close()


def oracle_case(arg):
    name, case = arg
    import oracle
    t0 = time.time()
    ref = oracle.OracleSim(case)
    for b in case["bodies"]:
        ref.add_body(b)
    nb = len(case["bodies"])
    hist = []
    for t in range(EVERY, STEPS + 1, EVERY):
        ref.step(t - ref.steps_done)
        hist.append([[ref.body_state(b)[k] for k in KEYS] for b in range(nb)])
        print(f"  {name}: oracle step {t} ({time.time() - t0:.0f} s)", flush=True)
    rho, ux, uy = ref.fields()
    ref.close()
    return name, np.array(hist), summarise(rho, ux, uy)


def compare(gpu_dir, procs):
    from multiprocessing import Pool
    todo = [(name, case) for name, case, _ in cases()]
    with Pool(min(procs, len(todo))) as pool:
        results = pool.map(oracle_case, todo)
    for name, hist, d in results:
        np.savez(os.path.join(gpu_dir, f"oracle-{name}.npz"), hist=hist, **d)
    table(gpu_dir)


def table(gpu_dir):
    """The largest differences over the window, per case and precision:
    drag is the force component with the larger magnitude in the oracle's
    history (x for the cylinders in a stream, y for settling particles),
    relative at every sampled step; force is max |F_gpu - F_oracle| over
    max |F_oracle| (vectors); position and velocity are absolute, in
    lattice units; field is the largest velocity difference on the
    subsampled nodes over the largest oracle speed component."""
    print(f"\n{'case':38s} {'prec':5s} {'drag (max rel)':>15s} {'force':>10s} "
          f"{'position':>10s} {'velocity':>10s} {'field':>10s}")
    for name, case, precs in cases():
        r = np.load(os.path.join(gpu_dir, f"oracle-{name}.npz"))
        hist_r = r["hist"]
        for pname in precs:
            g = np.load(os.path.join(gpu_dir, f"{name}-{pname}.npz"))
            hist_g = g["hist"]
            c = int(np.abs(hist_r[:, :, 1]).max() > np.abs(hist_r[:, :, 0]).max())
            drag = (np.abs(hist_g[:, :, c] - hist_r[:, :, c]) / np.abs(hist_r[:, :, c])).max()
            force = np.hypot(*(hist_g[:, :, :2] - hist_r[:, :, :2]).transpose(2, 0, 1)).max() \
                / np.hypot(hist_r[:, :, 0], hist_r[:, :, 1]).max()
            pos = np.abs(hist_g[:, :, 3:5] - hist_r[:, :, 3:5]).max()
            vel = np.abs(hist_g[:, :, 5:7] - hist_r[:, :, 5:7]).max()
            scale = max(np.abs(r["ux_sub"]).max(), np.abs(r["uy_sub"]).max())
            field = max(np.abs(g["ux_sub"] - r["ux_sub"]).max(), np.abs(g["uy_sub"] - r["uy_sub"]).max()) / scale
            print(f"{name:38s} {pname:5s} {drag:15.3e} {force:10.3e} {pos:10.3e} {vel:10.3e} {field:10.3e}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["gpu", "compare", "table"])
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out", "long_windows"))
    ap.add_argument("--gpu", default=os.path.join(ROOT, "gpurun_out", "long_windows"))
    ap.add_argument("--procs", type=int, default=4)
    a = ap.parse_args()
    if a.mode == "gpu":
        run_gpu(a.out)
    elif a.mode == "compare":
        compare(a.gpu, a.procs)
    else:
        table(a.gpu)


if __name__ == "__main__":
    main()
