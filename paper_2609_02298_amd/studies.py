"""The paper's prescribed-body setups at full scale, run on the GPU path.

``python -m paper_2609_02298_amd.studies inline-oscillation [--scheme ...]
[--kernel ...]`` runs the in-line oscillating cylinder of Sec. 2.9.2 (KC = 5,
Re = 100, 2401 x 1601, open faces) and reports the peak drag coefficient of
Table B.8 (largest |C_d| of each period after the first two, averaged), of
the body's whole IB force and of the outer fluid's force alone (the IB
force less the inertia of the fluid inside the cylinder).

``python -m paper_2609_02298_amd.studies settling [--density-ratio 1.5 1.1 1.01]``
runs the single-particle sedimentation of Sec. 2.9.3 (1281 x 3841, Zou-He
walls) and reports the largest settling speed over u_g (Table IV).

``python -m paper_2609_02298_amd.studies wake-interaction [--integrator verlet
euler] [--internal-mass feng none]`` runs the two-particle channel of Sec.
2.9.4 and reports each particle's peak Re_f = |v| D / nu (Table V), the
minimum gap and the overtaking step.

``python -m paper_2609_02298_amd.studies fixed-cylinder [--re 20 40 100 200]
[--scheme DF MDF DFC] [--kernel hat P4] [--precision fp64|fp32]`` runs the
fixed cylinder of Sec. 2.9.1 / Table I (2001 x 1601, D = 40 for Re <= 100;
3001 x 2401, D = 60 for Re = 200) for the paper's step counts and prints one
JSON line per case: the time-averaged drag coefficient over the paper's
averaging window (the quantity of Table II), the rms and amplitude of the
lift coefficient, the Strouhal number from the FFT peak and from the mean
period between zero crossings of the lift, the kernel-interpolated slip of
the last step normalised by u_inf (Table III), the boundary diagnostics of
Sec. 2.8 on the final field, the mean MDF pass count and the run's MLUPS.

``python -m paper_2609_02298_amd.studies taylor-green [--D 10 20 40 80]
[--mode pure DF MDF DFC] [--kernel P4 hat]`` runs the Taylor-Green check of
App. D.1 (Eq. D1, u0 = 0.04, Re = 10, t = L/u0) in pure LBM and in the
IB-LBM mode whose marker ring carries the analytic velocity, and prints the
L2 relative velocity errors with the pairwise and fitted convergence orders
(Tables D.1 / D.2).

Coefficients: C_d = 2 F_x / (rho0 u_inf^2 D), C_l = 2 F_y / (rho0 u_inf^2 D),
St = f D / u_inf (the normalisation is not printed in the paper; this is the
usual one).  Above Re = 50 the symmetric start state gets a small
transverse momentum kick behind the cylinder (``perturb_wake``) so that the
wake sheds.
Everything here is set-up and post-processing of the body history that the
library returns; the flow is computed by the HIP kernels.
"""
from __future__ import annotations

import argparse
import math
import json
import sys
import time

import numpy as np


def flow_statistics(fx: np.ndarray, fy: np.ndarray, u_ref: float, diameter: float,
                    rho0: float = 1.0) -> dict:
    """Drag / lift statistics of a force history sampled every step over the
    averaging window.  St is reported twice: from the peak of the lift
    spectrum (resolution 1/len of the window) and from the mean spacing of
    upward zero crossings of C_l - mean(C_l); both are None when the lift
    does not oscillate (amplitude below 1e-6)."""
    q = 0.5 * rho0 * u_ref * u_ref * diameter
    cd = np.asarray(fx, dtype=float) / q
    cl = np.asarray(fy, dtype=float) / q
    out = {"cd_mean": float(cd.mean()), "cl_mean": float(cl.mean()),
           "cl_rms": float(cl.std()), "cl_amp": float(0.5 * (cl.max() - cl.min())),
           "st_fft": None, "st_zero": None}
    if out["cl_amp"] < 1e-6 or len(cl) < 8:
        return out
    x = cl - cl.mean()
    spec = np.abs(np.fft.rfft(x))
    k = int(np.argmax(spec[1:])) + 1
    out["st_fft"] = float(k / len(x) * diameter / u_ref)
    up = np.nonzero((x[:-1] < 0) & (x[1:] >= 0))[0]
    if len(up) >= 2:
        # crossing instants by linear interpolation between the two samples
        t = up + x[up] / (x[up] - x[up + 1])
        out["st_zero"] = float(diameter / u_ref / np.diff(t).mean())
    return out


def perturb_wake(sim, case, du_over_u: float = 0.1):
    """Break the mirror symmetry of the start state: the setup (on-node
    cylinder, uniform inflow, markers symmetric about y = y_c) is exactly
    symmetric, so the wake would shed only once round-off grew.  At t = 0 a
    transverse momentum du_over_u * u_inf is added in a D x R patch behind
    the upper half of the cylinder by moving mass from population 4 (e_y =
    -1) to population 2 (e_y = +1), which leaves the density unchanged.  The
    paper does not say how its wakes were started; this is the reading."""
    b = case["bodies"][0]
    r = 0.5 * b["diameter"]
    x0, y0 = int(b["xc"] + r + 2), int(b["yc"] + 1)
    x1, y1 = x0 + int(b["diameter"]), int(b["yc"] + r)
    f = sim.populations()
    eps = 0.5 * du_over_u * case["u_ref"] * case["rho0"]
    f[2, y0:y1, x0:x1] += eps
    f[4, y0:y1, x0:x1] -= eps
    sim.set_populations(f)


def run_fixed_cylinder(re: float, scheme: str, kernel: str, collision: str = "BGK",
                       precision: str = "fp64", steps: int | None = None,
                       log=sys.stderr) -> dict:
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.paper_fixed_cylinder(re, scheme=scheme, kernel=kernel, collision=collision)
    nsteps = steps or case["steps"]
    avg0 = case["average_from"] if steps is None else int(0.7 * nsteps) + 1
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    sim = ib.Sim(case, precision=prec, history_capacity=nsteps)
    if re > 50.0:
        # the wake sheds above Re ~ 47; below it the flow is steady and a
        # kick would only add a slowly decaying transient
        perturb_wake(sim, case)
    chunk = 20000
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        n = min(chunk, nsteps - done)
        sim.step(n)
        sim.sync()
        done += n
        print(f"  {case['name']} {scheme}/{kernel}/{collision} {precision}: {done}/{nsteps} steps, "
              f"{time.perf_counter() - t0:.1f} s", file=log, flush=True)
    wall = time.perf_counter() - t0
    st = sim.forces(0, check=False)
    h = sim.history(0, avg0, nsteps - avg0 + 1)
    stats = flow_statistics(h[:, 1], h[:, 2], case["u_ref"], case["diameter"], case["rho0"])
    diag, _ = sim.diagnostics(0, 2, case["u_ref"])
    out = {"case": case["name"], "re": re, "scheme": scheme, "kernel": kernel,
           "collision": collision, "precision": precision, "steps": nsteps,
           "average_window": [avg0, nsteps], "status": st["status"],
           **{k: (round(v, 6) if isinstance(v, float) else v) for k, v in stats.items()},
           "slip_mean_over_uinf": st["slip_mean"] / case["u_ref"],
           "phi_leak": diag["phi_leak"], "u_inside_mean": diag["u_inside_mean"],
           "mdf_passes_mean": float(h[:, 12].mean()),
           "mlups": case["nx"] * case["ny"] * nsteps / wall / 1e6, "seconds": wall}
    sim.close()
    return out


def peak_drag(fx: np.ndarray, u_ref: float, diameter: float, period: int, rho0: float = 1.0):
    """Peak drag coefficient of an oscillating body: the largest |C_d| of
    each full period of the window, averaged over the periods, and the
    largest over the whole window."""
    cd = np.abs(np.asarray(fx, dtype=float)) / (0.5 * rho0 * u_ref * u_ref * diameter)
    n = len(cd) // period
    per = [float(cd[i * period:(i + 1) * period].max()) for i in range(n)]
    return {"cd_peak": float(np.mean(per)) if per else None, "cd_max": float(cd.max()),
            "periods": n}


def run_inline_oscillation(scheme: str, kernel: str, collision: str = "BGK",
                           precision: str = "fp64", log=sys.stderr) -> dict:
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.paper_inline_oscillation(scheme=scheme, kernel=kernel, collision=collision)
    nsteps, avg0 = case["steps"], case["average_from"]
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    sim = ib.Sim(case, precision=prec, history_capacity=nsteps)
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        n = min(10000, nsteps - done)
        sim.step(n)
        sim.sync()
        done += n
        print(f"  {case['name']} {scheme}/{kernel}/{collision} {precision}: {done}/{nsteps} steps, "
              f"{time.perf_counter() - t0:.1f} s", file=log, flush=True)
    wall = time.perf_counter() - t0
    st = sim.forces(0, check=False)
    h = sim.history(0, avg0, nsteps - avg0 + 1)
    pk = peak_drag(h[:, 1], case["u_ref"], case["diameter"], case["period"], case["rho0"])
    # the force of the outer fluid alone: the IB force also accelerates the
    # fictitious fluid inside the cylinder (mass m_f = rho0 pi r^2, moving
    # with the body), so F_out = F_hydro + m_f a_c with a_c the prescribed
    # acceleration at the step's time
    b = case["bodies"][0]
    w = 2.0 * np.pi * b["freq"]
    t = h[:, 0]
    acc = -b["amp"][0] * w * w * np.sin(w * t + b["phase"])
    mf = case["rho0"] * np.pi * (0.5 * case["diameter"]) ** 2
    pko = peak_drag(h[:, 1] + mf * acc, case["u_ref"], case["diameter"], case["period"],
                    case["rho0"])
    out = {"case": case["name"], "scheme": scheme, "kernel": kernel, "collision": collision,
           "precision": precision, "steps": nsteps, "window": [avg0, nsteps],
           "status": st["status"], **pk,
           "cd_peak_outer": pko["cd_peak"], "cd_max_outer": pko["cd_max"],
           "slip_mean_over_umax": float(h[:, 9].mean()) / case["u_ref"],
           "mdf_passes_mean": float(h[:, 12].mean()),
           "mlups": case["nx"] * case["ny"] * nsteps / wall / 1e6, "seconds": wall}
    sim.close()
    return out


def stop_reason(status: int) -> str:
    """What ended a free-body run: the step budget, a support reaching a wall
    or another body's support (range status), or a non-finite force."""
    if status == 0:
        return "step budget"
    if status == -5:
        return "wall or contact"
    if status == -4:
        return "diverged"
    return f"status {status}"


def run_settling(density_ratio: float, scheme: str, kernel: str, collision: str = "BGK",
                 precision: str = "fp64", height_d: float = 24.0, internal_mass: str = "feng",
                 diameter: float = 160.0, log=sys.stderr) -> dict:
    """One particle settling in the closed channel (Sec. 2.9.3; height_d = 60
    for the extended channel of App. C.2) until its support reaches the
    bottom wall or the step budget is spent.  Reports the largest settling
    speed over u_g (the quantity of Table IV) and its step, and the peak
    Re_f = |v_y| D / nu (Table C.1) over the whole fall and over the first
    15.5 D of it (the standard channel's contact-safe horizon)."""
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.paper_settling(density_ratio, scheme=scheme, kernel=kernel, collision=collision,
                                   height_d=height_d, diameter=diameter,
                                   internal_mass=ib.IM_FENG if internal_mass == "feng" else ib.IM_NONE)
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    nsteps = case["steps"]
    y0 = case["bodies"][0]["yc"]
    sim = ib.Sim(case, precision=prec, history_capacity=nsteps)
    t0 = time.perf_counter()
    done, status = 0, 0
    while done < nsteps:
        sim.step(min(10000, nsteps - done))
        sim.sync()
        done = sim.steps_done
        st = sim.forces(0, check=False)
        status = st["status"]
        print(f"  {case['name']} {scheme}/{kernel}/{collision} {precision}: {done} steps, "
              f"y = {st['yc']:.1f}, v/u_g = {st['vy'] / case['u_g']:.4f}, "
              f"{time.perf_counter() - t0:.1f} s", file=log, flush=True)
        if status:
            break
    wall = time.perf_counter() - t0
    n = sim.steps_done
    if n == 0:
        out = {"case": case["name"], "density_ratio": density_ratio, "scheme": scheme,
               "kernel": kernel, "collision": collision, "precision": precision,
               "internal_mass": internal_mass, "steps": 0, "stopped_by": stop_reason(status),
               "flags": int(st["flags"])}
        sim.close()
        return out
    h = sim.history(0, 1, n)
    v = -h[:, 7] / case["u_g"]
    fall = (y0 - h[:, 5]) / case["diameter"]
    win = fall <= 15.5
    to_re = case["u_g"] * case["diameter"] / case["nu"]
    out = {"case": case["name"], "density_ratio": density_ratio, "scheme": scheme,
           "kernel": kernel, "collision": collision, "precision": precision,
           "internal_mass": internal_mass, "steps": int(n), "stopped_by": stop_reason(status),
           "v_star_max": float(v.max()), "v_star_max_step": int(v.argmax()) + 1,
           "v_star_max_fall_15_5": float(v[win].max()),
           "re_f_max": float(v.max() * to_re), "re_f_max_fall_15_5": float(v[win].max() * to_re),
           "fall_final_d": float(fall[-1]),
           "y_final": float(h[-1, 5]), "mlups": case["nx"] * case["ny"] * n / wall / 1e6,
           "seconds": wall}
    sim.close()
    return out


def acceleration_proxy(vx, vy, u_g: float, D: float, cadence: int) -> np.ndarray:
    """Particle-bound acceleration proxy of Sec. 2.8, |a*| = |dv*/dt*| with
    v* = v / u_g and t* = t u_g / D, from velocity records stored every
    `cadence` steps.  Central differences inside the record, one-sided ones
    at its ends (reading: the paper defines the quantity, not the
    difference formula)."""
    v = np.stack([np.asarray(vx, float), np.asarray(vy, float)]) / u_g
    d = np.gradient(v, cadence * u_g / D, axis=1)
    return np.hypot(d[0], d[1])


def phase_peaks(a_heavy, a_light, t_star, t_closest: float, t_exchange: float) -> dict:
    """Largest |a*| of each particle before the closest approach and after
    the role exchange (the phases of Sec. 5.2.3 / Table C.4), and the
    light-over-heavy ratios of those peaks with their post/pre contrast."""
    t_star = np.asarray(t_star, float)
    pre, post = t_star < t_closest, t_star > t_exchange
    out = {"pre_heavy": float(np.max(a_heavy[pre])), "pre_light": float(np.max(a_light[pre])),
           "post_heavy": float(np.max(a_heavy[post])), "post_light": float(np.max(a_light[post]))}
    out["ratio_pre"] = out["pre_light"] / out["pre_heavy"]
    out["ratio_post"] = out["post_light"] / out["post_heavy"]
    out["contrast"] = out["ratio_post"] / out["ratio_pre"]
    return out


def run_wake_interaction(scheme="DF", kernel="P4", collision="BGK", integrator="verlet",
                         internal_mass="feng", precision="fp64", length_d: float = 50.0,
                         log=sys.stderr) -> dict:
    """Two particles settling along +x (Sec. 2.9.4) until a support reaches
    the end wall or the step budget is spent: the peak Reynolds number of
    each on the fluid-density basis Re_f = |v| D / nu (the quantity of
    Table V), the minimum surface gap over D and its step, and the step at
    which the heavy particle passes the light one."""
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.paper_wake_interaction(
        scheme=scheme, kernel=kernel, collision=collision,
        integrator=ib.EULER_A1 if integrator == "euler" else ib.VERLET,
        internal_mass=ib.IM_FENG if internal_mass == "feng" else ib.IM_NONE, length_d=length_d)
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    nsteps = case["steps"]
    sim = ib.Sim(case, precision=prec, history_capacity=nsteps)
    t0 = time.perf_counter()
    done, status = 0, 0
    while done < nsteps:
        sim.step(min(5000, nsteps - done))
        sim.sync()
        done = sim.steps_done
        st = [sim.forces(b, check=False) for b in range(2)]
        status = next((x["status"] for x in st if x["status"]), 0)
        print(f"  {case['name']} {scheme}/{kernel}/{collision}/{integrator}/{internal_mass} "
              f"{precision}: {done} steps, x = {st[0]['xc']:.1f} / {st[1]['xc']:.1f}, "
              f"{time.perf_counter() - t0:.1f} s", file=log, flush=True)
        if status:
            break
    wall = time.perf_counter() - t0
    n = sim.steps_done
    hh, hl = sim.history(0, 1, n), sim.history(1, 1, n)
    D, nu = case["diameter"], case["nu"]
    re_h = np.hypot(hh[:, 6], hh[:, 7]) * D / nu
    re_l = np.hypot(hl[:, 6], hl[:, 7]) * D / nu
    gap = np.hypot(hh[:, 4] - hl[:, 4], hh[:, 5] - hl[:, 5]) / D - 1.0
    passed = np.nonzero(hh[:, 4] > hl[:, 4])[0]
    out = {"case": case["name"], "scheme": scheme, "kernel": kernel, "collision": collision,
           "integrator": integrator, "internal_mass": internal_mass, "precision": precision,
           "steps": int(n), "stopped_by": stop_reason(status),
           "re_f_max_heavy": float(re_h.max()), "re_f_max_light": float(re_l.max()),
           "min_gap_over_d": float(gap.min()), "min_gap_step": int(gap.argmin()) + 1,
           "overtake_step": int(passed[0]) + 1 if len(passed) else None,
           "mlups": case["nx"] * case["ny"] * n / wall / 1e6, "seconds": wall}
    if len(passed):
        # acceleration proxy on records stored every 500 and 100 steps (the
        # first at the cadence itself), each particle on its own u_g; t* on
        # the heavy particle's, as are the phase boundaries
        g = float(np.hypot(*case["gravity"]))
        ug_h = math.sqrt((case["bodies"][0]["density_ratio"] - 1.0) * g * D)
        ug_l = math.sqrt((case["bodies"][1]["density_ratio"] - 1.0) * g * D)
        t_close = (int(gap.argmin()) + 1) * ug_h / D
        t_exch = (int(passed[0]) + 1) * ug_h / D
        out["t_star_closest"], out["t_star_exchange"] = t_close, t_exch
        for cad in (500, 100):
            idx = np.arange(cad - 1, n, cad)
            ah = acceleration_proxy(hh[idx, 6], hh[idx, 7], ug_h, D, cad)
            al = acceleration_proxy(hl[idx, 6], hl[idx, 7], ug_l, D, cad)
            out[f"a_star_{cad}"] = phase_peaks(ah, al, (idx + 1) * ug_h / D, t_close, t_exch)
    sim.close()
    return out


# ---- the benchmark configurations at their stated lengths, FP32 vs FP64
def _launch_for(case, prec):
    from . import autotune
    return autotune.lookup(case["nx"], case["ny"], case["collision"], prec)


def _run_steps(sim, nsteps, label, log, chunk=20000):
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        n = min(chunk, nsteps - done)
        sim.step(n)
        sim.sync()
        done += n
        print(f"  {label}: {done}/{nsteps} steps, {time.perf_counter() - t0:.1f} s", file=log,
              flush=True)
        if sim.forces(0, check=False)["status"] != 0:
            break
    return time.perf_counter() - t0


def run_unsteady_cylinder(re: float, scheme: str, kernel: str, collision: str, precision: str,
                          steps: int = 100000, log=sys.stderr) -> dict:
    """Configuration 2: the 2000 x 800 fixed cylinder (D = 80, 251 markers,
    u_inf = 0.1) for `steps` steps; mean C_d, rms C_l and St over the last
    30 % of the steps (wake started as in perturb_wake)."""
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.unsteady_cylinder(scheme=scheme, kernel=kernel, collision=collision, re=re,
                                      steps=steps)
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    sim = ib.Sim(case, precision=prec, history_capacity=steps)
    launch = _launch_for(case, prec)
    if launch:
        sim.set_launch(**launch)
    perturb_wake(sim, case)
    wall = _run_steps(sim, steps, f"{case['name']} {scheme}/{kernel}/{collision} {precision}", log)
    st = sim.forces(0, check=False)
    done = sim.steps_done
    avg0 = int(0.7 * done) + 1
    h = sim.history(0, avg0, done - avg0 + 1)
    stats = flow_statistics(h[:, 1], h[:, 2], case["u_ref"], case["diameter"], case["rho0"])
    sim.close()
    return {"config": 2, "re": re, "scheme": scheme, "kernel": kernel, "collision": collision,
            "precision": precision, "steps": done, "status": st["status"],
            "average_window": [avg0, done], **stats,
            "slip_mean_over_uinf": float(h[:, 9].mean() / case["u_ref"]),
            "mlups": case["nx"] * case["ny"] * done / wall / 1e6}


def run_oscillating_cylinder(precision: str, st0: float | None, steps: int = 60000,
                             log=sys.stderr) -> dict:
    """Configuration 3: the 1200 x 600 cylinder (D = 40, Re = 100, MDF / P4 /
    TRT).  st0 None: the stationary cylinder of the same setup, whose
    shedding Strouhal number (zero crossings of the lift over the last 30 %)
    sets the frequency; else the transverse oscillation y = 0.2 D sin(2 pi f
    t) with f = 0.8 st0 u_inf / D, reporting the marker slip and the drag and
    lift over the last 30 % and their histories' extremes."""
    import ib_cases
    from . import ib_lbm as ib

    fixed = st0 is None
    case = ib_cases.oscillating_cylinder(steps=steps, st0=st0 or ib_cases.ST0_RE100, fixed=fixed)
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    sim = ib.Sim(case, precision=prec, history_capacity=steps)
    launch = _launch_for(case, prec)
    if launch:
        sim.set_launch(**launch)
    perturb_wake(sim, case)
    label = f"oscillating cylinder {'stationary' if fixed else 'moving'} {precision}"
    wall = _run_steps(sim, steps, label, log)
    st = sim.forces(0, check=False)
    done = sim.steps_done
    avg0 = int(0.7 * done) + 1
    h = sim.history(0, avg0, done - avg0 + 1)
    stats = flow_statistics(h[:, 1], h[:, 2], case["u_ref"], case["diameter"], case["rho0"])
    q = 0.5 * case["rho0"] * case["u_ref"] ** 2 * case["diameter"]
    out = {"config": 3, "motion": "fixed" if fixed else "transverse", "precision": precision,
           "steps": done, "status": st["status"], "average_window": [avg0, done], **stats,
           "cd_max": float(h[:, 1].max() / q), "cl_max": float(np.abs(h[:, 2]).max() / q),
           "slip_mean_over_uinf": float(h[:, 9].mean() / case["u_ref"]),
           "slip_max_over_uinf": float(h[:, 10].max() / case["u_ref"]),
           "mlups": case["nx"] * case["ny"] * done / wall / 1e6}
    if not fixed:
        out["st0"] = st0
        out["frequency"] = case["bodies"][0]["freq"]
    sim.close()
    return out


def run_sedimentation(pair: bool, precision: str, steps: int = 200000, log=sys.stderr) -> dict:
    """Configuration 4: sedimentation in the 400 x 2000 Zou-He box (D = 20,
    Ar ~ 1000, DFC / P4 / CM-MRT, Feng correction, FP64 body update) for up
    to `steps` steps, stopping when a support reaches a wall (no contact
    model).  Reports each body's largest settling speed |v_y| (and over u_g
    = (0.5 g D)^(1/2)) and its speed at the last step."""
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.sedimentation(pair=pair, steps=steps)
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    sim = ib.Sim(case, precision=prec, history_capacity=steps)
    wall = _run_steps(sim, steps, f"sedimentation {'pair' if pair else 'single'} {precision}", log)
    done = sim.steps_done
    bodies = []
    for b in range(len(case["bodies"])):
        st = sim.forces(b, check=False)
        h = sim.history(b, 1, done)
        vy = h[:, 7]
        k = int(np.argmax(np.abs(vy)))
        bodies.append({"density_ratio": case["bodies"][b]["density_ratio"],
                       "v_settle_max": float(abs(vy[k])), "step_of_max": int(h[k, 0]),
                       "v_settle_max_over_ug": float(abs(vy[k]) / case["u_ref"]),
                       "v_final": float(vy[-1]), "y_final": float(h[-1, 5]),
                       "status": st["status"]})
    sim.close()
    return {"config": 4, "pair": pair, "precision": precision, "steps": done,
            "stop": "support reached a wall" if done < steps else "step budget", "bodies": bodies,
            "mlups": case["nx"] * case["ny"] * done / wall / 1e6}


def run_taylor_green(D: int, scheme: str | None, kernel: str, precision: str = "fp64",
                     collision: str = "BGK") -> dict:
    """App. D.1: the Taylor-Green check at resolution D (pure LBM when
    scheme is None, else the IB-LBM mode of ``ib_cases.taylor_green_ib``),
    started from the equilibrium of Eq. D1 with the vortex's pressure, and
    its L2 relative velocity error at t = L/u0."""
    import ib_cases
    from . import ib_lbm as ib

    case = ib_cases.taylor_green_ib(D, scheme, kernel, collision=ib_cases.COLLISIONS[collision])
    prec = ib.FP64 if precision == "fp64" else ib.FP32_SHIFTED
    sim = ib.Sim(case, precision=prec)
    n, u0, nu, steps = case["nx"], case["tg_u0"], case["tg_nu"], case["steps"]
    ux, uy = ib_cases.taylor_green_velocity(n, n, u0)
    sim.set_equilibrium(ux, uy, ib_cases.taylor_green_pressure_density(n, n, u0))
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    wall = time.perf_counter() - t0
    _, vx, vy = sim.fields()
    sim.close()
    ax, ay = ib_cases.taylor_green_velocity(n, n, u0, steps, nu)
    l2 = float(np.sqrt(((vx - ax) ** 2 + (vy - ay) ** 2).sum() / (ax ** 2 + ay ** 2).sum()))
    return {"study": "taylor-green", "D": D, "mode": scheme or "pure", "kernel": kernel,
            "collision": collision, "precision": precision, "steps": steps, "l2": l2,
            "seconds": wall}


def rel_diff(a, b):
    if a is None or b is None:
        return None
    return abs(a - b) / abs(b) if b != 0 else abs(a - b)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="study", required=True)
    fc = sub.add_parser("fixed-cylinder", help="Sec. 2.9.1 fixed cylinder at paper scale")
    fc.add_argument("--re", type=float, nargs="+", default=[20.0, 40.0, 100.0, 200.0])
    fc.add_argument("--scheme", nargs="+", default=["DF", "MDF", "DFC"])
    fc.add_argument("--kernel", nargs="+", default=["hat", "P4"])
    fc.add_argument("--collision", default="BGK")
    fc.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    fc.add_argument("--steps", type=int, default=None,
                    help="override the paper's step count (averaging over the last 30%%)")
    oc = sub.add_parser("inline-oscillation", help="Sec. 2.9.2 in-line oscillation, KC = 5")
    oc.add_argument("--scheme", nargs="+", default=["DF", "MDF", "DFC"])
    oc.add_argument("--kernel", nargs="+", default=["hat", "P4"])
    oc.add_argument("--collision", default="BGK")
    oc.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    se = sub.add_parser("settling", help="Sec. 2.9.3 single-particle sedimentation")
    se.add_argument("--density-ratio", type=float, nargs="+", default=[1.5, 1.1, 1.01])
    se.add_argument("--scheme", nargs="+", default=["DF", "MDF", "DFC"])
    se.add_argument("--kernel", nargs="+", default=["P4", "hat"])
    se.add_argument("--collision", default="BGK")
    se.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    se.add_argument("--height-d", type=float, default=24.0,
                    help="channel height in diameters: 24 (Sec. 2.9.3) or 60 (App. C.2)")
    se.add_argument("--internal-mass", nargs="+", default=["feng"], choices=["feng", "none"])
    se.add_argument("--diameter", type=float, default=160.0,
                    help="particle diameter in nodes: 160 (Sec. 2.9.3) or 240 (App. C.5)")
    wi = sub.add_parser("wake-interaction", help="Sec. 2.9.4 two-particle wake interaction")
    wi.add_argument("--scheme", nargs="+", default=["DF"])
    wi.add_argument("--kernel", default="P4")
    wi.add_argument("--collision", default="BGK")
    wi.add_argument("--integrator", nargs="+", default=["verlet"], choices=["verlet", "euler"])
    wi.add_argument("--internal-mass", nargs="+", default=["feng", "none"], choices=["feng", "none"])
    wi.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    wi.add_argument("--length-d", type=float, default=50.0,
                    help="channel length in diameters: 50 (Sec. 2.9.4) or 60 (Table C.3)")
    tg = sub.add_parser("taylor-green", help="App. D.1 Taylor-Green convergence, pure LBM and "
                                              "the IB-LBM mode (Tables D.1 / D.2)")
    tg.add_argument("--D", type=int, nargs="+", default=[10, 20, 40, 80])
    tg.add_argument("--mode", nargs="+", default=["pure", "DF", "MDF", "DFC"])
    tg.add_argument("--kernel", nargs="+", default=["P4", "hat"])
    tg.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    cf = sub.add_parser("configs", help="benchmark configurations 2-4 at their stated lengths, "
                                           "FP32 shifted against FP64")
    cf.add_argument("which", choices=["unsteady-cylinder", "oscillating-cylinder", "sedimentation"])
    cf.add_argument("--re", type=float, nargs="+", default=[100.0, 200.0])
    cf.add_argument("--scheme", nargs="+", default=["DF", "MDF", "DFC"])
    cf.add_argument("--kernel", nargs="+", default=["hat", "P4"])
    cf.add_argument("--collision", nargs="+", default=["BGK", "TRT", "CMMRT"])
    cf.add_argument("--steps", type=int, default=None)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("studies: no HIP device", file=sys.stderr)
        return 1
    if args.study == "taylor-green":
        for kernel in args.kernel:
            for mode in args.mode:
                if mode == "pure" and kernel != args.kernel[0]:
                    continue
                rows = [run_taylor_green(D, None if mode == "pure" else mode, kernel, args.precision)
                        for D in args.D]
                for r in rows:
                    print(json.dumps(r), flush=True)
                e = [r["l2"] for r in rows]
                orders = [float(np.log2(a / b)) for a, b in zip(e, e[1:])]
                fit = float(-np.polyfit(np.log(args.D), np.log(e), 1)[0]) if len(e) > 1 else None
                print(json.dumps({"summary": mode, "kernel": kernel, "D": args.D, "l2": e,
                                  "pairwise_orders": orders, "fitted_order": fit}), flush=True)
        return 0
    if args.study == "configs":
        if args.which == "unsteady-cylinder":
            for re in args.re:
                for col in args.collision:
                    for kernel in args.kernel:
                        for scheme in args.scheme:
                            r = {p: run_unsteady_cylinder(re, scheme, kernel, col, p,
                                                          args.steps or 100000)
                                 for p in ("fp64", "fp32")}
                            r["fp32_vs_fp64"] = {k: rel_diff(r["fp32"][k], r["fp64"][k])
                                                 for k in ("cd_mean", "cl_rms", "st_fft", "st_zero")}
                            print(json.dumps(r), flush=True)
        elif args.which == "oscillating-cylinder":
            n = args.steps or 60000
            st = run_oscillating_cylinder("fp64", None, n)
            print(json.dumps(st), flush=True)
            st0 = st["st_zero"]
            r = {p: run_oscillating_cylinder(p, st0, n) for p in ("fp64", "fp32")}
            r["fp32_vs_fp64"] = {k: rel_diff(r["fp32"][k], r["fp64"][k])
                                 for k in ("cd_mean", "cl_rms", "slip_mean_over_uinf", "cd_max",
                                           "cl_max")}
            print(json.dumps(r), flush=True)
        else:
            for pair in (False, True):
                r = {p: run_sedimentation(pair, p, args.steps or 200000) for p in ("fp64", "fp32")}
                r["fp32_vs_fp64"] = [rel_diff(a["v_settle_max"], b["v_settle_max"])
                                     for a, b in zip(r["fp32"]["bodies"], r["fp64"]["bodies"])]
                print(json.dumps(r), flush=True)
        return 0
    if args.study == "settling":
        for rr in args.density_ratio:
            for kernel in args.kernel:
                for scheme in args.scheme:
                    for im in args.internal_mass:
                        r = run_settling(rr, scheme, kernel, args.collision, args.precision,
                                         args.height_d, im, args.diameter)
                        print(json.dumps(r), flush=True)
        return 0
    if args.study == "wake-interaction":
        for scheme in args.scheme:
            for integ in args.integrator:
                for im in args.internal_mass:
                    r = run_wake_interaction(scheme, args.kernel, args.collision, integ, im,
                                             args.precision, args.length_d)
                    print(json.dumps(r), flush=True)
        return 0
    if args.study == "inline-oscillation":
        for kernel in args.kernel:
            for scheme in args.scheme:
                r = run_inline_oscillation(scheme, kernel, args.collision, args.precision)
                print(json.dumps(r), flush=True)
        return 0
    for re in args.re:
        for kernel in args.kernel:
            for scheme in args.scheme:
                r = run_fixed_cylinder(re, scheme, kernel, args.collision, args.precision,
                                       args.steps)
                print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
