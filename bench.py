#!/usr/bin/env python3
"""Throughput benchmark of the IB-LBM hot path on one MI355X.

One "step" is one full IB-LBM time step of the workload: fused collide +
stream over the lattice, then the immersed-boundary pass (interpolation,
scheme update, spreading, FP64 force/torque reductions, body update).

Default workload: the unsteady fixed cylinder on the 2000 x 800 lattice,
D = 80 (251 markers), Re = 100, MDF (k = 5) with the Peskin 4-point kernel
and TRT collision, FP32 shifted populations (FP64 reductions).  The line
also carries the FP64 run of the same workload, the collide-stream
roofline (achieved GB/s of algorithmic bytes from HIP events on the
library's stream), and the FP64 oracle timed on the host on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--extra]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def kernel_source_hash() -> str:
    """Hash of what the collide-stream kernels are built from: their source,
    the shared collide-stream device code, and the shared definitions
    (structs, helpers) ahead of the launcher declarations in the internal
    header."""
    csrc = os.path.join(ROOT, "paper_2609_02298_amd", "csrc")
    h = hashlib.sha256()
    for name in ("lbm_kernels.hip", "lbm_device.h"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "ib_lbm_internal.h"), "rb") as fh:
        head = fh.read()
    h.update(head.split(b"// ---- kernel launchers")[0])
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str):
    """HBM bytes per collide-stream launch from the committed rocprofv3
    counter summary, or None if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "collide_stream_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload_key)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def run_gpu(case, precision, steps, warmup, graph=0, launch=None, tune=True, want_fields=False):
    import torch
    import paper_2609_02298_amd as ib

    if launch is None and tune:
        # the shipped table (written by the autotuner on an MI355X) when it
        # has this lattice, else tune now
        from paper_2609_02298_amd import autotune
        launch = autotune.tune_step(case, precision)
    sim = ib.Sim(case, precision=precision)
    if launch:
        sim.set_launch(**launch)
    if graph:
        sim.set_graph(graph)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    # the device-wide synchronize covers the sim's stream (and, for pipelined
    # steps, the two streams it joins into it)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # MDF passes applied in each timed step (history column 12)
    passes = sim.history(0, warmup + 1, steps)[:, 12] if steps else np.zeros(0)
    split, near = sim.overlap()
    fused = sim.fused()
    # IB pass duration from HIP events around each pass in a separate run of
    # unpipelined steps (the events add host and queue work to every step, so
    # the wall-clock run above has none)
    sim.set_overlap(False)
    sim.timing(True)
    sim.step(min(steps, 100))
    sim.sync()
    ibm_ms, n_ibm = sim.timing_read(1)
    sim.timing(False)
    sim.set_overlap(True)
    st = sim.forces(0, check=False)
    vel = sim.fields()[1:] if want_fields else None
    # boundary-fidelity diagnostics of the body (Sec. 2.8) on the final
    # state: host wall clock of the whole call (launch, wait, copy back)
    dts = []
    for _ in range(5):
        td = time.perf_counter()
        diag, _ = sim.diagnostics(0, 2, case.get("u_ref", 0.1))
        dts.append(time.perf_counter() - td)
    # collide-stream kernel duration: HIP events around 200 back-to-back
    # launches on a second sim of the same workload (two steps in, so that
    # the force box is set), on the stream they are launched on
    tsim = ib.Sim(case, precision=precision)
    if launch:
        tsim.set_launch(**launch)
    tsim.step(2)
    lbm_us, inner = tsim.time_collide_stream(200)
    tsim.close()
    lbm_ms, n_lbm = lbm_us * 1e-3, 1
    out = dict(seconds=t1 - t0, lbm_ms=lbm_ms, n_lbm=n_lbm, ibm_ms=ibm_ms, n_ibm=n_ibm,
               inner_nodes=inner,
               split=split, near_nodes=near, fused=fused,
               fx=st["fx"], status=st["status"], steps_done=sim.steps_done,
               diag=diag, diag_ms=float(np.median(dts)) * 1e3,
               passes_mean=float(passes.mean()) if len(passes) else 0.0,
               passes_min=int(passes.min()) if len(passes) else 0,
               passes_max=int(passes.max()) if len(passes) else 0,
               launch=sim.get_launch(), vel=vel, steps_total=sim.steps_done)
    sim.close()
    return out


def cpu_baseline(case, target_seconds=12.0, max_threads=16):
    """The FP64 oracle as it stands, one independent copy of the workload
    per host core: each thread steps its own oracle sim (ctypes releases the
    interpreter lock during the C call, so the copies run in parallel), and
    the aggregate node updates over the wall time of the parallel region
    give the rate.  Threads: the host's cores, at most max_threads (a GPU
    box gives one GPU's job 16 cores, whatever the OS count shows)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    ncores = os.cpu_count() or 1
    nthreads = max(1, min(ncores, max_threads))
    refs = []
    for _ in range(nthreads):
        r = oracle.OracleSim(case)
        for b in case["bodies"]:
            r.add_body(b)
        refs.append(r)
    t0 = time.perf_counter()
    refs[0].step(1)
    one = time.perf_counter() - t0
    # the copies share the memory bus; size the sample from one solo step
    n = max(1, min(200, int(target_seconds / max(one, 1e-3) / 2)))
    with ThreadPoolExecutor(nthreads) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda r: r.step(n), refs))
        dt = time.perf_counter() - t0
    for r in refs:
        r.close()
    nodes = case["nx"] * case["ny"]
    return dict(value=nthreads * nodes * n / dt / 1e6, unit="MLUPS", cores=nthreads, kind="oracle",
                host_cpus=ncores,
                per_core=nodes * n / dt / 1e6,
                sample=f"{nthreads} independent copies of {case['name']} (one per core, "
                       f"{ncores} host CPUs), {n} steps each after 1 untimed, single-threaded "
                       f"FP64 C oracle per copy, {dt:.1f} s wall")


def serving_leg(precision, launch, n_cases: int, step_scale: int, budget_gb: float,
                quantum: int, seed: int = 0):
    """Parameter-sweep serving: the seeded sweep cases (grid widths
    log-uniform in [128, 2048], aspect 2-4, all 18 scheme/kernel/collision
    combinations) with step counts divided by `step_scale`, served (a) all
    arriving at once and (b) by a Poisson process at 1.25x the measured
    sequential service rate, next to sequential plain solves of the same
    cases on the same GPU and precision."""
    import numpy as np
    import ib_cases
    from paper_2609_02298_amd import serving

    cases = ib_cases.sweep_cases(n_cases, seed=seed)
    steps = [max(1, c["steps"] // step_scale) for c in cases]
    log = sys.stderr
    seq = serving.sequential(cases, precision, steps=steps, launch=launch, progress=log)
    rate = 1.25 * len(cases) / seq["wall"]
    # arrival gaps from their own stream so that the cases are the same in
    # every mode
    gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, len(cases))
    arrivals = np.cumsum(gaps) - gaps[0]
    budget = int(budget_gb * 2**30)
    timeout = 600.0 + 20.0 * seq["wall"]
    burst = serving.serve(cases, precision, steps=steps, hbm_budget=budget, quantum=quantum,
                          launch=launch, timeout=timeout, progress=log)
    # the same burst with each round's batch steps replayed from captured
    # HIP graphs of graph_steps steps
    graph_steps = 32
    burst_graph = serving.serve(cases, precision, steps=steps, hbm_budget=budget, quantum=quantum,
                                graph_steps=graph_steps, launch=launch, timeout=timeout,
                                progress=log)
    pois = serving.serve(cases, precision, steps=steps, arrivals=arrivals, hbm_budget=budget,
                         quantum=quantum, launch=launch, timeout=timeout, progress=log)
    nodes = [c["nx"] * c["ny"] for c in cases]
    return {
        "workload": f"sweep seed {seed}: {len(cases)} cases, {min(nodes)}-{max(nodes)} nodes, "
                    f"steps U{{2000..20000}}/{step_scale}",
        "precision": "fp32-shifted" if precision == 1 else "fp64",
        "hbm_budget_gb": budget_gb, "quantum": quantum,
        "node_updates": int(sum(n * k for n, k in zip(nodes, steps))),
        "burst": serving.summary(cases, burst, seq),
        "burst_graph": dict(serving.summary(cases, burst_graph, seq), graph_steps=graph_steps),
        "poisson": dict(serving.summary(cases, pois, seq, arrivals=list(arrivals)),
                        rate_per_s=round(rate, 3)),
    }


def largest_leg(steps32: int = 60, steps64: int = 30):
    """The largest lattice of the seeded sweep (7175 x 2014, 14.45M nodes,
    1.04 GB of FP32 populations: well beyond the 256 MB Infinity Cache), with
    its body, in both precisions: whole-step MLUPS and the collide-stream
    roofline."""
    import ib_cases
    import paper_2609_02298_amd as ib

    cases = ib_cases.sweep_cases(256, seed=0)
    c = max(cases, key=lambda k: k["nx"] * k["ny"])
    b = c["bodies"][0]
    out = {"workload": c["name"], "nx": c["nx"], "ny": c["ny"], "diameter": c["diameter"],
           "scheme": ["DF", "MDF", "DFC"][b["scheme"]], "kernel": ["hat", "P4"][b["kernel"]],
           "collision": ["BGK", "TRT", "CMMRT"][c["collision"]]}
    nodes = c["nx"] * c["ny"]
    lbm_nodes = (c["nx"] - 3) * (c["ny"] - 2)
    for pname, p, bpn, steps in (("fp32", ib.FP32_SHIFTED, 72, steps32), ("fp64", ib.FP64, 144, steps64)):
        r = run_gpu(c, p, steps, 5)
        avg = r["lbm_ms"] / max(r["n_lbm"], 1) * 1e-3
        a = bpn * lbm_nodes / avg / 1e9
        out[pname] = {"value": round(nodes * steps / r["seconds"] / 1e6, 1), "unit": "MLUPS",
                      "roofline_achieved_GBs": round(a, 1), "roofline_frac": round(a / HBM_PEAK_GBS, 4),
                      "traffic": measured_traffic(f"{c['name']}-{pname}-{out['collision']}"),
                      "avg_launch_us": round(avg * 1e6, 2),
                      "ib_pass_avg_us": round(r["ibm_ms"] / max(r["n_ibm"], 1) * 1e3, 2),
                      "population_bytes": 2 * 9 * nodes * bpn // 18, "launch": r["launch"]}
    # the plain read + write stream of the same bytes (one FP32 lattice each
    # way) with the library's reference copy: what a streaming kernel reaches
    # on this part, beside the 8 TB/s of the roofline's peak
    ceil = stream_ceiling(9 * lbm_nodes * 4)
    out["stream_copy"] = ceil
    for pname in ("fp32", "fp64"):
        out[pname]["frac_of_stream_copy"] = round(out[pname]["roofline_achieved_GBs"] / ceil["achieved_GBs"], 4)
    return out


def stream_ceiling(nbytes: int, reps: int = 20):
    """Best rate over a few workgroup counts of ib_lbm_stream_copy moving
    nbytes (read nbytes, write nbytes), HIP events on the launch stream."""
    import torch
    import paper_2609_02298_amd as ib

    n = (nbytes + 15) // 16 * 4
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = None
    for wg in (256, 512, 1024):
        for _ in range(3):
            ib.stream_copy(a, b, wg)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ib.stream_copy(a, b, wg)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = 2 * 4 * n / us / 1e3
        if best is None or gbs > best["achieved_GBs"]:
            best = {"bytes_each_way": 4 * n, "workgroups": wg, "avg_us": round(us, 2),
                    "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del a, b
    torch.cuda.empty_cache()
    return best


def copy_calibration(mb: float):
    """One device copy of `mb` MB (read mb, write mb): the reference kernel
    against which the collide-stream's FETCH_SIZE / WRITE_SIZE counters are
    scaled."""
    import torch
    n = int(mb * 1e6) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    return n * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--scheme", default="MDF")
    ap.add_argument("--kernel", default="P4")
    ap.add_argument("--collision", default="TRT")
    ap.add_argument("--re", type=float, default=100.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="use the library's default launch shape")
    ap.add_argument("--extra", action="store_true", help="also time every scheme/kernel/collision")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep")
    ap.add_argument("--serve-cases", type=int, default=256)
    ap.add_argument("--serve-step-scale", type=int, default=40)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-quantum", type=int, default=128)
    ap.add_argument("--no-largest", action="store_true", help="skip the largest-lattice leg")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive-MDF leg (N in [5, 20], tolerance 1e-4)")
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU runs are not part of it", file=sys.stderr)
        sys.exit(2)

    import torch
    import ib_cases
    import paper_2609_02298_amd as ib

    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    ib.load_library()
    case = ib_cases.unsteady_cylinder(scheme=args.scheme, kernel=args.kernel,
                                      collision=args.collision, re=args.re)
    nodes = case["nx"] * case["ny"]
    prec = ib.FP32_SHIFTED if args.precision == "fp32" else ib.FP64
    bpn = 72 if prec == ib.FP32_SHIFTED else 144

    r = run_gpu(case, prec, args.steps, args.warmup, graph=args.graph, tune=not args.no_tune,
                want_fields=not args.no_fp64)
    mlups = nodes * args.steps / r["seconds"] / 1e6
    lbm_avg_s = r["lbm_ms"] / max(r["n_lbm"], 1) * 1e-3
    # the timed collide-stream launch updates the inner nodes; the face nodes
    # (rows 0 and ny-1, columns 0, nx-2, nx-1) go through a small second
    # launch with the face closures
    lbm_nodes = r["inner_nodes"]
    achieved = bpn * lbm_nodes / lbm_avg_s / 1e9
    key = f"{case['name']}-{args.precision}-{args.collision}"
    traffic = measured_traffic(key)

    line = {
        "metric": "MLUPS (IB-LBM step, FP32-shifted) + HBM roofline %",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["seconds"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == ib.FP32_SHIFTED else "f64",
        "data": "synthetic (parametric flow case, no dataset)",
        "config": {"workload": case["name"], "nx": case["nx"], "ny": case["ny"],
                   "diameter": case["diameter"], "markers": 251, "re": args.re,
                   "scheme": args.scheme, "kernel": args.kernel, "collision": args.collision,
                   "precision": "fp32-shifted" if prec == ib.FP32_SHIFTED else "fp64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "collide_stream_lean_kernel (all tiles)",
                     "bytes_per_node": bpn, "nodes_per_launch": lbm_nodes,
                     "avg_launch_us": round(lbm_avg_s * 1e6, 3),
                     "launch": r["launch"]},
        # fused: one launch per step (the IB pass beside every tile); else
        # pipelined: two streams, the tiles next to the body after the pass
        "pipelined_steps": {"in_use": r["split"], "fused": r["fused"],
                            "nodes_waiting_for_ib": 0 if r["fused"] else r["near_nodes"]},
        "ib_pass_avg_us": round(r["ibm_ms"] / max(r["n_ibm"], 1) * 1e3, 3),
        "hbm_fraction_of_step": round(bpn * nodes * args.steps / r["seconds"] / 1e9 / HBM_PEAK_GBS, 4),
        "lattice_bytes": 2 * 9 * nodes * (bpn // 18),
        "mall_resident_note": "2 lattices of this size fit in the 256 MB Infinity Cache",
        "diagnostics": {"call_ms": round(r["diag_ms"], 3), "kappa": 2,
                        **{k: round(v, 6) for k, v in r["diag"].items()}},
    }
    if not args.no_fp64 and prec == ib.FP32_SHIFTED:
        # the same workload and step sequence in FP64: its throughput, and
        # the FP32-shifted result's error against it after the same steps
        r64 = run_gpu(case, ib.FP64, args.steps, args.warmup, graph=args.graph,
                      tune=not args.no_tune, want_fields=True)
        s64 = args.steps
        a64 = 144 * lbm_nodes / (r64["lbm_ms"] / max(r64["n_lbm"], 1) * 1e-3) / 1e9
        ux32, uy32 = r["vel"]
        ux64, uy64 = r64["vel"]
        scale = max(np.abs(ux64).max(), np.abs(uy64).max())
        line["fp32_vs_fp64"] = {
            "steps": r["steps_total"],
            "drag_rel": abs(r["fx"] - r64["fx"]) / abs(r64["fx"]),
            "velocity_max_rel": float(max(np.abs(ux32 - ux64).max(), np.abs(uy32 - uy64).max()) / scale),
            "tolerance": {"drag": 1e-4, "velocity": 1e-5}}
        line["fp64"] = {"value": round(nodes * s64 / r64["seconds"] / 1e6, 2), "unit": "MLUPS",
                        "roofline_achieved_GBs": round(a64, 1),
                        "roofline_frac": round(a64 / HBM_PEAK_GBS, 4),
                        "avg_launch_us": round(r64["lbm_ms"] / max(r64["n_lbm"], 1) * 1e3, 3),
                        "ib_pass_avg_us": round(r64["ibm_ms"] / max(r64["n_ibm"], 1) * 1e3, 3)}
    if not args.no_adaptive and prec == ib.FP32_SHIFTED:
        # the paper's adaptive MDF on the same lattice and body: between 5
        # and 20 passes per step, as the slip residual decides
        ca = ib_cases.unsteady_cylinder(scheme="MDF", kernel=args.kernel,
                                        collision=args.collision, re=args.re)
        ca["bodies"][0].update(ib_cases.ADAPTIVE_MDF)
        sa = max(args.steps // 2, 50)
        ra = run_gpu(ca, prec, sa, args.warmup // 2, tune=not args.no_tune)
        line["adaptive_mdf"] = {
            "value": round(nodes * sa / ra["seconds"] / 1e6, 2), "unit": "MLUPS",
            "steps": sa, "bounds": [ib_cases.ADAPTIVE_MDF["mdf_nmin"], ib_cases.ADAPTIVE_MDF["mdf_iters"]],
            "tolerance": ib_cases.ADAPTIVE_MDF["mdf_tol"],
            "passes_mean": round(ra["passes_mean"], 2),
            "passes_min": ra["passes_min"], "passes_max": ra["passes_max"],
            "ib_pass_avg_us": round(ra["ibm_ms"] / max(ra["n_ibm"], 1) * 1e3, 3)}
        line["mdf_passes_per_step"] = r["passes_mean"]
    if args.extra:
        combos = {}
        for sch in ("DF", "MDF", "DFC"):
            for ker in ("hat", "P4"):
                for col in ("BGK", "TRT", "CMMRT"):
                    c = ib_cases.unsteady_cylinder(scheme=sch, kernel=ker, collision=col, re=args.re)
                    for pname, p in (("fp32", ib.FP32_SHIFTED), ("fp64", ib.FP64)):
                        rr = run_gpu(c, p, 100, 10, tune=not args.no_tune)
                        combos[f"{sch}/{ker}/{col}/{pname}"] = round(nodes * 100 / rr["seconds"] / 1e6, 1)
        line["combos_mlups"] = combos
    if not args.no_largest:
        line["largest_lattice"] = largest_leg()
    if not args.no_serving:
        line["serving"] = serving_leg(prec, r["launch"], args.serve_cases, args.serve_step_scale,
                                      args.serve_budget_gb, args.serve_quantum)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case)
    if args.copy_calibration_mb > 0:
        line["copy_calibration_bytes"] = copy_calibration(args.copy_calibration_mb)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
