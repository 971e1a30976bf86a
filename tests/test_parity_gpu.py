"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 path velocity / populations max-abs relative 1e-12, drag
1e-10 relative; FP32 shifted path velocity 1e-5 relative, drag 1e-4
relative.  "Relative" for a field is max|a - b| / max|b| over the nodes.
"""
import math
import sys

import numpy as np
import pytest

import ib_cases
import oracle
import paper_2609_02298_amd as ib

pytestmark = pytest.mark.gpu

F64_FIELD, F64_DRAG = 1e-12, 1e-10
F32_FIELD, F32_DRAG = 1e-5, 1e-4


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ib.load_library()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def make_pair(case, precision=ib.FP64, pops=None):
    sim = ib.Sim(case, precision=precision)
    ref = oracle.OracleSim(case)
    for b in case.get("bodies", []):
        ref.add_body(b)
    if pops is not None:
        sim.set_populations(pops)
        ref.set_populations(pops)
    return sim, ref


def compare_fields(sim, ref, tol):
    _, ux, uy = sim.fields()
    _, rx, ry = ref.fields()
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    e = max(np.abs(ux - rx).max(), np.abs(uy - ry).max()) / scale
    return e


# ------------------------------------------------------------------ lattice
@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("col", [ib.BGK, ib.TRT, ib.CMMRT])
def test_periodic_box(col, prec):
    say(f"periodic box col={col} prec={prec}")
    case = dict(nx=67, ny=29, collision=col, tau=0.73, bc=(ib.PERIODIC,) * 4,
                fluid_force=(3e-6, -2e-6))
    pops = ib_cases.random_populations(67, 29, 1, amp=0.02, u=(0.03, 0.01))
    sim, ref = make_pair(case, prec, pops)
    sim.step(40)
    ref.step(40)
    if prec == ib.FP64:
        assert rel(sim.populations(), ref.populations()) < F64_FIELD
    assert compare_fields(sim, ref, None) < (F64_FIELD if prec == ib.FP64 else F32_FIELD)
    assert sim.steps_done == 40


FACE_SETS = {
    "periodic": ((ib.PERIODIC,) * 4, 0.0),
    "channel": ((ib.VEL_PARABOLIC, ib.ZERO_GRADIENT, ib.BOUNCE_BACK, ib.BOUNCE_BACK), 0.05),
    "farfield": ((ib.VEL_UNIFORM, ib.ZERO_GRADIENT, ib.VEL_UNIFORM, ib.VEL_UNIFORM), 0.08),
    "box": ((ib.BOUNCE_BACK,) * 4, 0.0),
    # zero-gradient on every face (the open boundaries of the in-line
    # oscillating cylinder, Sec. 2.9.2), and mixed with a wall and a
    # velocity face so that every kind of corner meets one
    "open": ((ib.ZERO_GRADIENT,) * 4, 0.0),
    "open-mixed": ((ib.ZERO_GRADIENT, ib.ZERO_GRADIENT, ib.BOUNCE_BACK, ib.VEL_UNIFORM), 0.04),
    "inflow-open": ((ib.VEL_UNIFORM, ib.ZERO_GRADIENT, ib.ZERO_GRADIENT, ib.ZERO_GRADIENT), 0.06),
    # on-node Zou-He walls: a closed box (all four corners) and a channel
    "zh-box": ((ib.ZOU_HE,) * 4, 0.0),
    "zh-channel": ((ib.PERIODIC, ib.PERIODIC, ib.ZOU_HE, ib.ZOU_HE), 0.0),
}


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("col", [ib.BGK, ib.TRT, ib.CMMRT])
@pytest.mark.parametrize("faces", ["channel", "farfield", "box", "open", "open-mixed", "inflow-open",
                                   "zh-box", "zh-channel"])
def test_faces(col, prec, faces):
    """Every face closure on a ragged lattice (not a multiple of the tile)."""
    say(f"faces {faces} col={col} prec={prec}")
    bc, u = FACE_SETS[faces]
    case = dict(nx=77, ny=41, collision=col, tau=0.66, bc=bc, u_bc=u)
    u0 = (u * 0.5, 0.0) if u > 0 else (0.05, 0.03)  # closed box: sloshing start
    pops = ib_cases.random_populations(77, 41, 2, amp=0.01, u=u0)
    sim, ref = make_pair(case, prec, pops)
    sim.step(60)
    ref.step(60)
    if prec == ib.FP64:
        assert rel(sim.populations(), ref.populations()) < F64_FIELD
    assert compare_fields(sim, ref, None) < (F64_FIELD if prec == ib.FP64 else F32_FIELD)


@pytest.mark.parametrize("col", [ib.BGK, ib.TRT, ib.CMMRT])
@pytest.mark.parametrize("faces", ["periodic", "channel", "farfield", "box", "open", "open-mixed",
                                   "zh-box", "zh-channel"])
def test_faces_even_width_fp32(col, faces):
    """FP32 on a wider lattice (several tiles in x and y, inner nodes and
    face nodes in separate launches), every face closure."""
    say(f"even width fp32 {faces} col={col}")
    bc, u = FACE_SETS[faces]
    nx, ny = 390, 46
    case = dict(nx=nx, ny=ny, collision=col, tau=0.66, bc=bc, u_bc=u,
                fluid_force=(2e-6, -1e-6) if faces in ("periodic", "zh-channel") else (0.0, 0.0))
    u0 = (u * 0.5, 0.0) if u > 0 else (0.05, 0.03)
    pops = ib_cases.random_populations(nx, ny, 5, amp=0.01, u=u0)
    sim, ref = make_pair(case, ib.FP32_SHIFTED, pops)
    sim.set_launch(64, 2, 1, 1)
    sim.step(60)
    ref.step(60)
    assert compare_fields(sim, ref, None) < F32_FIELD


def test_set_get_populations_roundtrip():
    case = dict(nx=33, ny=17, tau=0.8, bc=(ib.PERIODIC,) * 4)
    pops = ib_cases.random_populations(33, 17, 3)
    sim = ib.Sim(case, precision=ib.FP64)
    sim.set_populations(pops)
    np.testing.assert_array_equal(sim.populations(), pops)
    s32 = ib.Sim(case, precision=ib.FP32_SHIFTED)
    s32.set_populations(pops)
    assert np.abs(s32.populations() - pops).max() < 1e-8


def test_initial_state_matches_oracle():
    for case in (ib_cases.fixed_cylinder_channel(), ib_cases.unsteady_cylinder(nx=120, ny=60, diameter=12)):
        case = dict(case, bodies=[])
        sim, ref = make_pair(case)
        assert rel(sim.populations(), ref.populations()) < 1e-15


# ------------------------------------------------------------------ bodies
COMBOS = [(s, k, c) for s in (ib.DF, ib.MDF, ib.DFC) for k in (ib.HAT, ib.PESKIN4)
          for c in (ib.BGK, ib.TRT, ib.CMMRT)]


def body_case(scheme, kernel, col, nx=96, ny=64, D=16.0, **bkw):
    body = dict(xc=nx / 3 + 0.37, yc=ny / 2 - 0.21, diameter=D, scheme=scheme, kernel=kernel,
                mdf_iters=5)
    body.update(bkw)
    return dict(nx=nx, ny=ny, collision=col, tau=0.7, trt_magic=0.25, cm_s_q=1.2, cm_s_eps=1.4,
                bc=(ib.VEL_UNIFORM, ib.ZERO_GRADIENT, ib.VEL_UNIFORM, ib.VEL_UNIFORM), u_bc=0.06,
                bodies=[body])


@pytest.mark.parametrize("scheme,kernel,col", COMBOS)
def test_fixed_body_fp64(scheme, kernel, col):
    say(f"fixed body scheme={scheme} kernel={kernel} col={col}")
    case = body_case(scheme, kernel, col)
    sim, ref = make_pair(case)
    for _ in range(3):
        sim.step(8)
        ref.step(8)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < F64_DRAG
        assert abs(fs["fy"] - fr["fy"]) < F64_DRAG * abs(fr["fx"])
        assert abs(fs["torque"] - fr["torque"]) < 1e-9 * abs(fr["fx"]) * 8
        assert abs(fs["slip_mean"] - fr["slip_mean"]) < 1e-10 * max(fr["slip_mean"], 1e-12)
        if scheme == ib.MDF:
            assert abs(fs["mdf_residual"] - fr["mdf_residual"]) < 1e-10 * fr["mdf_residual"]
            assert abs(fs["mdf_omega"] - ref.mdf_omega(0)) < 1e-13 * ref.mdf_omega(0)
    assert rel(sim.populations(), ref.populations()) < F64_FIELD
    if scheme != ib.DFC:
        gx, gy = sim.force()
        rx, ry = ref.force()
        assert rel(np.stack([gx, gy]), np.stack([rx, ry])) < F64_FIELD
    ms, mr = sim.markers(0), ref.markers(0)
    np.testing.assert_allclose(ms[:, :4], mr[:, :4], rtol=0, atol=1e-12)
    assert rel(ms[:, 4:6], mr[:, 4:6]) < 1e-11
    if scheme == ib.DFC:
        assert rel(ms[:, 6], mr[:, 6]) < 1e-13


@pytest.mark.parametrize("scheme,kernel,col", [(ib.DF, ib.HAT, ib.BGK), (ib.MDF, ib.PESKIN4, ib.TRT),
                                               (ib.DFC, ib.PESKIN4, ib.CMMRT),
                                               (ib.DFC, ib.HAT, ib.BGK)])
def test_fixed_body_fp32(scheme, kernel, col):
    say(f"fixed body fp32 scheme={scheme} kernel={kernel} col={col}")
    case = body_case(scheme, kernel, col)
    sim, ref = make_pair(case, ib.FP32_SHIFTED)
    sim.step(150)
    ref.step(150)
    assert compare_fields(sim, ref, None) < F32_FIELD
    fs, fr = sim.forces(0), ref.body_state(0)
    assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < F32_DRAG


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_prescribed_oscillation(prec):
    say(f"prescribed oscillation prec={prec}")
    case = body_case(ib.MDF, ib.PESKIN4, ib.TRT, nx=120, ny=80, D=16.0,
                     motion=ib.PRESCRIBED_SIN, amp=(0.0, 3.2), freq=0.004, phase=0.0)
    sim, ref = make_pair(case, prec)
    for _ in range(4):
        sim.step(25)
        ref.step(25)
        fs, fr = sim.forces(0), ref.body_state(0)
        tol = F64_DRAG if prec == ib.FP64 else F32_DRAG
        assert abs(fs["yc"] - fr["yc"]) < 1e-12
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < tol
        assert abs(fs["fy"] - fr["fy"]) < tol * abs(fr["fx"]) * 5
    assert compare_fields(sim, ref, None) < (F64_FIELD if prec == ib.FP64 else F32_FIELD)


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("pair", [False, True])
@pytest.mark.parametrize("im", [ib.IM_NONE, ib.IM_FENG])
@pytest.mark.parametrize("integ", [ib.VERLET, ib.EULER_A1])
def test_free_bodies(prec, pair, im, integ):
    """Free disks settling in a closed box (Eq. 21-23, A3), with the
    Velocity-Verlet or the Euler-explicit (Eq. A1) update, every body and
    every checked step at the stated tolerances (drag and settling velocity
    1e-10 in FP64, 1e-4 in FP32).  The light disk of the pair (density ratio
    1.1) is the sensitive one; the oracle itself, perturbed every step by
    the rounding of either store, moves its velocity and force by ~1e-12
    (FP64) and ~1e-7 (FP32) relative over these 80 steps, well inside the
    tolerances."""
    say(f"free bodies pair={pair} im={im} integrator={integ} prec={prec}")
    case = ib_cases.sedimentation(pair=pair, nx=80, ny=200, diameter=12.0, internal_mass=im)
    for b in case["bodies"]:
        b["integrator"] = integ
    case["gravity"] = (0.0, -1e-4)
    if pair:
        case["bodies"][0].update(xc=39.0, yc=140.0)
        case["bodies"][1].update(xc=41.0, yc=170.0)
    else:
        case["bodies"][0].update(xc=40.0, yc=160.0)
    sim, ref = make_pair(case, prec)
    y0 = [b["yc"] for b in case["bodies"]]
    tol = 1e-10 if prec == ib.FP64 else F32_DRAG
    for t in (12, 40, 80):
        n = t - sim.steps_done
        sim.step(n)
        ref.step(n)
        for b in range(len(case["bodies"])):
            fs, fr = sim.forces(b), ref.body_state(b)
            assert abs(fs["vy"] - fr["vy"]) < tol * abs(fr["vy"]), (b, t, fs["vy"], fr["vy"])
            assert abs(fs["yc"] - fr["yc"]) < tol * abs(fr["yc"] - y0[b]) + 1e-13, (b, t)
            assert abs(fs["fy"] - fr["fy"]) < tol * abs(fr["fy"]) + 1e-15, (b, t, fs["fy"], fr["fy"])
    assert fr["vy"] < 0


@pytest.mark.parametrize("scheme,kernel,prec", [
    ("DF", "P4", ib.FP64), ("MDF", "P4", ib.FP64), ("DFC", "P4", ib.FP64),
    ("DF", "hat", ib.FP64), ("MDF", "hat", ib.FP64), ("DFC", "hat", ib.FP64),
    ("MDF", "P4", ib.FP32_SHIFTED), ("DFC", "P4", ib.FP32_SHIFTED)])
def test_settling_in_zou_he_box(scheme, kernel, prec):
    """The single-particle sedimentation of Sec. 2.9.3 on a reduced lattice:
    Zou-He walls on all four sides, BGK, Velocity-Verlet with the Feng
    correction, marker spacing 2/3, the adaptive MDF of Sec. 2.5.2; a
    density-ratio-1.5 disk of D = 20 released at rest, 60 steps.  The
    fluid field is compared too, since the walls act on it."""
    say(f"settling zou-he box {scheme}/{kernel} prec={prec}")
    D = 20.0
    body = dict(xc=48.0, yc=110.0, diameter=D, n_markers=int(round(math.pi * D / (2.0 / 3.0))),
                scheme=ib_cases.SCHEMES[scheme], kernel=ib_cases.KERNELS[kernel], mdf_iters=5,
                motion=ib.FREE, density_ratio=1.5, internal_mass=ib.IM_FENG, integrator=ib.VERLET)
    if scheme == "MDF":
        body.update(ib_cases.ADAPTIVE_MDF)
    case = dict(nx=97, ny=161, collision=ib.BGK, tau=0.6, bc=(ib.ZOU_HE,) * 4, u_bc=0.0,
                gravity=(0.0, -1e-4), bodies=[body])
    sim, ref = make_pair(case, prec)
    tol = F64_DRAG if prec == ib.FP64 else F32_DRAG
    for t in (15, 60):
        n = t - sim.steps_done
        sim.step(n)
        ref.step(n)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert abs(fs["vy"] - fr["vy"]) < tol * abs(fr["vy"]), (t, fs["vy"], fr["vy"])
        assert abs(fs["fy"] - fr["fy"]) < tol * abs(fr["fy"]), (t, fs["fy"], fr["fy"])
        assert abs(fs["yc"] - fr["yc"]) < tol * abs(fr["yc"] - 110.0) + 1e-13, t
        if scheme == "MDF":
            assert fs["mdf_iters"] == fr["mdf_iters"], t
    assert compare_fields(sim, ref, None) < (F64_FIELD if prec == ib.FP64 else F32_FIELD)
    assert fr["vy"] < 0


# --------------------------------- IB-LBM Taylor-Green mode (App. D.1, Eq. D1)
def _tg_pops(case):
    n, u0 = case["nx"], case["tg_u0"]
    ux, uy = ib_cases.taylor_green_velocity(n, n, u0)
    rho = ib_cases.taylor_green_pressure_density(n, n, u0)
    f = np.zeros((9, n, n))
    for j in range(n):
        for i in range(n):
            f[:, j, i] = oracle.equilibrium(rho[j, i], ux[j, i], uy[j, i])
    return f


def _tg_l2(case, ux, uy, steps):
    n = case["nx"]
    ax, ay = ib_cases.taylor_green_velocity(n, n, case["tg_u0"], steps, case["tg_nu"])
    return math.sqrt(((ux - ax) ** 2 + (uy - ay) ** 2).sum() / (ax ** 2 + ay ** 2).sum())


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("scheme,kernel", [(ib.DF, ib.PESKIN4), (ib.MDF, ib.PESKIN4),
                                           (ib.DFC, ib.PESKIN4), (ib.DF, ib.HAT), (ib.DFC, ib.HAT)])
def test_taylor_green_ib_mode(scheme, kernel, prec):
    """The ring of markers driven to Eq. D1 (D = 20, 40 x 40 periodic box,
    500 steps = one convective time), started from the device's equilibrium
    of the vortex: fields and marker forces against the
    oracle after 100 steps, the desired velocities the oracle assigns, and
    the L2 error of the check at t = L/u0 to the oracle's."""
    say(f"taylor-green IB mode scheme={scheme} kernel={kernel} prec={prec}")
    case = ib_cases.taylor_green_ib(20, scheme, kernel)
    f0 = _tg_pops(case)
    sim, ref = make_pair(case, prec)
    ref.set_populations(f0)
    n = case["nx"]
    ux, uy = ib_cases.taylor_green_velocity(n, n, case["tg_u0"])
    sim.set_equilibrium(ux, uy, ib_cases.taylor_green_pressure_density(n, n, case["tg_u0"]))
    f64 = prec == ib.FP64
    # the device's equilibrium of Eq. 2 against the oracle's
    assert rel(sim.populations(), f0) < (1e-15 if f64 else 1e-7)
    sim.step(100)
    ref.step(100)
    assert compare_fields(sim, ref, None) < (F64_FIELD if f64 else F32_FIELD)
    ms, mr = sim.markers(0), ref.markers(0)
    np.testing.assert_allclose(ms[:, 2:4], mr[:, 2:4], rtol=0, atol=1e-15)
    fscale = np.abs(mr[:, 4:6]).max()
    assert np.abs(ms[:, 4:6] - mr[:, 4:6]).max() < (F64_DRAG if f64 else F32_DRAG) * fscale
    sim.step(400)
    ref.step(400)
    _, ux, uy = sim.fields()
    _, rx, ry = ref.fields()
    es, er = _tg_l2(case, ux, uy, 500), _tg_l2(case, rx, ry, 500)
    assert abs(es - er) < (1e-10 if f64 else 1e-4) * er, (es, er)


def test_taylor_green_body_has_no_rigid_diagnostics():
    case = ib_cases.taylor_green_ib(20, ib.DF, ib.PESKIN4)
    sim = ib.Sim(case)
    sim.step(1)
    with pytest.raises(ib.IbLbmError):
        sim.diagnostics(0, 2, 0.04)
    bad = dict(case["bodies"][0], motion=ib.PRESCRIBED_SIN, amp=(1.0, 0.0), freq=1e-3)
    sim2 = ib.Sim(dict(case, bodies=[]))
    with pytest.raises(ib.IbLbmError):
        sim2.add_body(bad)
    sim.close()
    sim2.close()


# ---------------------------------------------------------- full workloads
@pytest.fixture(scope="module")
def cylinder_channel_ref():
    case = ib_cases.fixed_cylinder_channel(steps=5000)
    ref = oracle.OracleSim(case)
    for b in case["bodies"]:
        ref.add_body(b)
    ref.step(case["steps"])
    return case, ref


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_cylinder_channel_full_run(cylinder_channel_ref, prec):
    """200x80 channel, D = 20 cylinder, DF + hat, BGK, Re = 20: 5000 steps."""
    say(f"cylinder channel 5000 steps prec={prec}")
    case, ref = cylinder_channel_ref
    sim = ib.Sim(case, precision=prec)
    sim.step(case["steps"])
    e = compare_fields(sim, ref, None)
    fs, fr = sim.forces(0), ref.body_state(0)
    cd_s = 2 * fs["fx"] / (case["u_ref"] ** 2 * case["diameter"])
    cd_r = 2 * fr["fx"] / (case["u_ref"] ** 2 * case["diameter"])
    say(f"  velocity err {e:.3e}  Cd gpu {cd_s:.12f} oracle {cd_r:.12f}")
    if prec == ib.FP64:
        assert e < F64_FIELD and abs(cd_s - cd_r) / abs(cd_r) < F64_DRAG
    else:
        assert e < F32_FIELD and abs(cd_s - cd_r) / abs(cd_r) < F32_DRAG


WINDOW_CHECKS = (25, 50, 75, 100)


def _window_reference(scheme, kernel, col):
    """The oracle over the first 100 steps of the 2000 x 800 benchmark
    lattice (D = 80, 251 markers, Re = 100): body state at every check step,
    populations and fields at the last."""
    case = ib_cases.unsteady_cylinder(scheme=scheme, kernel=kernel, collision=col, re=100.0)
    ref = oracle.OracleSim(case)
    ref.add_body(case["bodies"][0])
    states = {}
    for t in WINDOW_CHECKS:
        ref.step(t - ref.steps_done)
        states[t] = ref.body_state(0)
    out = dict(case=case, states=states, pops=ref.populations(), fields=ref.fields())
    ref.close()
    return out


@pytest.fixture(scope="module")
def headline_window():
    say("oracle: 100 steps of 2000x800 MDF/P4/TRT")
    return _window_reference("MDF", "P4", "TRT")


@pytest.fixture(scope="module")
def dfc_cmmrt_window():
    say("oracle: 100 steps of 2000x800 DFC/P4/CM-MRT")
    return _window_reference("DFC", "P4", "CMMRT")


def _check_window(ref, prec, launch=None, pipelined=True, fused=None):
    case = ref["case"]
    sim = ib.Sim(case, precision=prec)
    if launch:
        sim.set_launch(**launch)
    if fused is not None:
        sim.set_fused(fused)
    f64 = prec == ib.FP64
    for t in WINDOW_CHECKS:
        sim.step(t - sim.steps_done)
        fs, fr = sim.forces(0), ref["states"][t]
        say(f"  step {t}: drag gpu {fs['fx']:.15e} oracle {fr['fx']:.15e}")
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < (F64_DRAG if f64 else F32_DRAG), t
        if f64:
            assert abs(fs["slip_mean"] - fr["slip_mean"]) < 1e-9 * fr["slip_mean"], t
    assert sim.overlap()[0] == pipelined
    if fused is not None:
        assert sim.fused() == fused
    _, ux, uy = sim.fields()
    _, rx, ry = ref["fields"]
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    e = max(np.abs(ux - rx).max(), np.abs(uy - ry).max()) / scale
    say(f"  velocity field max-rel error after 100 steps: {e:.3e}")
    assert e < (F64_FIELD if f64 else F32_FIELD)
    if f64:
        assert rel(sim.populations(), ref["pops"]) < F64_FIELD
    sim.close()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("prec", [ib.FP32_SHIFTED, ib.FP64])
def test_headline_window_pipelined(headline_window, prec, fused):
    """The benchmark's own configuration, element by element against the
    oracle for 100 steps: 2000 x 800, MDF (k = 5) / Peskin 4-point / TRT,
    the launch shape of the shipped tuning table, FP32 shifted (the
    headline) and FP64; as fused steps (one launch per step, the default
    here) and as two-stream pipelined steps."""
    from paper_2609_02298_amd import autotune
    say(f"2000x800 MDF/P4/TRT 100-step window prec={prec} fused={fused}")
    launch = autotune.lookup(2000, 800, ib.TRT, prec)
    _check_window(headline_window, prec, launch, fused=fused)


@pytest.mark.parametrize("prec", [ib.FP32_SHIFTED, ib.FP64])
def test_dfc_cmmrt_full_size_window(dfc_cmmrt_window, prec):
    """2000 x 800, DFC / Peskin 4-point / CM-MRT for 100 steps (in FP64 the
    body's workspace exceeds the LDS budget and runs from device memory)."""
    say(f"2000x800 DFC/P4/CM-MRT 100-step window prec={prec}")
    _check_window(dfc_cmmrt_window, prec)


def test_df_hat_bgk_full_size_window():
    say("2000x800 DF/hat/BGK 100-step window FP64")
    _check_window(_window_reference("DF", "hat", "BGK"), ib.FP64)


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_inline_oscillation_open_faces(prec):
    """A body oscillating in x in a quiescent fluid with zero-gradient faces on
    all four sides (the in-line case of Sec. 2.9.2, reduced): fields, drag
    and position against the oracle."""
    say(f"in-line oscillation, open faces, prec={prec}")
    case = dict(nx=150, ny=100, collision=ib.BGK, tau=0.74, bc=(ib.ZERO_GRADIENT,) * 4,
                bodies=[dict(xc=74.6, yc=49.7, diameter=16.0, scheme=ib.MDF, kernel=ib.PESKIN4,
                             mdf_iters=5, motion=ib.PRESCRIBED_SIN,
                             amp=(-5 * 16 / (2 * math.pi), 0.0), freq=0.1 / 80.0)])
    sim, ref = make_pair(case, prec)
    for _ in range(4):
        sim.step(30)
        ref.step(30)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert abs(fs["xc"] - fr["xc"]) < 1e-12
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < (F64_DRAG if prec == ib.FP64 else F32_DRAG)
    assert compare_fields(sim, ref, None) < (F64_FIELD if prec == ib.FP64 else F32_FIELD)


def test_oscillating_cylinder_full_size_window():
    """1200 x 600, D = 40, transverse oscillation, MDF / P4 / TRT: 100 steps."""
    say("1200x600 oscillating cylinder 100-step window FP64")
    case = ib_cases.oscillating_cylinder()
    sim, ref = make_pair(case)
    for _ in range(4):
        sim.step(25)
        ref.step(25)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < F64_DRAG
        assert abs(fs["fy"] - fr["fy"]) < F64_DRAG * abs(fr["fx"])
        assert abs(fs["yc"] - fr["yc"]) < 1e-12
        assert abs(fs["slip_mean"] - fr["slip_mean"]) < 1e-9 * fr["slip_mean"]
    assert rel(sim.populations(), ref.populations()) < F64_FIELD


@pytest.mark.parametrize("pair", [False, True])
def test_sedimentation_full_size_window(pair):
    """400 x 2000 Zou-He box, DFC / P4 / CM-MRT, free bodies: 100 steps."""
    say(f"400x2000 sedimentation 100-step window FP64 pair={pair}")
    case = ib_cases.sedimentation(pair=pair)
    sim, ref = make_pair(case)
    for _ in range(4):
        sim.step(25)
        ref.step(25)
        for b in range(len(case["bodies"])):
            fs, fr = sim.forces(b), ref.body_state(b)
            assert abs(fs["vy"] - fr["vy"]) < 1e-10 * abs(fr["vy"]), (b, fs["vy"], fr["vy"])
            assert abs(fs["fy"] - fr["fy"]) < 1e-10 * abs(fr["fy"]) + 1e-15, b
    assert rel(sim.populations(), ref.populations()) < F64_FIELD


# ------------------------------------------ adaptive MDF (Sec. 2.5.2, App. A.2)
def decision_margin(rs, nmin, tol):
    """Smallest relative distance of the oracle's residuals r_n from the
    thresholds that its stop decisions compared them with (the tolerance
    after nmin passes, 1.5 r_(n-1) from the second interpolation on)."""
    m = math.inf
    for n in range(1, len(rs) + 1):
        if n > nmin:
            m = min(m, abs(rs[n - 1] - tol) / tol)
        if n > 1:
            m = min(m, abs(rs[n - 1] - 1.5 * rs[n - 2]) / (1.5 * rs[n - 2]))
    return m


ADAPTIVE_GPU = [(ib.HAT, 1e-3, ib.PRESCRIBED_SIN, ib.SPREAD_GATHER),
                (ib.PESKIN4, 1e-4, ib.PRESCRIBED_SIN, ib.SPREAD_GATHER),
                (ib.PESKIN4, 1e-4, ib.FIXED, ib.SPREAD_GATHER),
                (ib.PESKIN4, 1e-4, ib.PRESCRIBED_SIN, ib.SPREAD_ATOMIC)]


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("kernel,tol,motion,spread", ADAPTIVE_GPU)
def test_adaptive_mdf(kernel, tol, motion, spread, prec):
    """Adaptive MDF (N in [5, 20]) step by step against the oracle: the pass
    count of every step, its last residual, the forces and the fields.  The
    stop decisions are taken in FP64 on both sides; these seeded cases keep
    each of the oracle's residuals at least 1e-4 (relative) away from the
    threshold it was compared with (asserted), ten times further than the
    FP32 store moves them (the residuals agree to 1e-5), so the counts must
    agree exactly."""
    say(f"adaptive MDF kernel={kernel} tol={tol} motion={motion} spread={spread} prec={prec}")
    case = body_case(ib.MDF, kernel, ib.TRT, mdf_iters=20, mdf_nmin=5, mdf_tol=tol,
                     motion=motion, amp=(0.0, 3.2), freq=0.004)
    sim, ref = make_pair(case, prec)
    sim.set_spread(spread)
    f64 = prec == ib.FP64
    counts, rerr = [], 0.0
    for _ in range(40):
        sim.step(1)
        ref.step(1)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert decision_margin(ref.mdf_residuals(0), 5, tol) > (1e-9 if f64 else 1e-4)
        assert fs["mdf_iters"] == fr["mdf_iters"]
        counts.append(fs["mdf_iters"])
        rerr = max(rerr, abs(fs["mdf_residual"] - fr["mdf_residual"]) / fr["mdf_residual"])
        assert rerr < (1e-10 if f64 else 1e-5)
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < (F64_DRAG if f64 else F32_DRAG)
    say(f"  pass counts {counts}; residual max rel err {rerr:.2e}")
    assert len(set(counts)) > 1 or counts[0] == 20
    if f64:
        assert rel(sim.populations(), ref.populations()) < F64_FIELD
        gx, gy = sim.force()
        rx, ry = ref.force()
        assert rel(np.stack([gx, gy]), np.stack([rx, ry])) < F64_FIELD
    else:
        assert compare_fields(sim, ref, None) < F32_FIELD
    h = sim.history(0, 1, 40)
    np.testing.assert_array_equal(h[:, 12], counts)


def test_adaptive_mdf_single_marker_closed_form_gpu():
    """The closed form of the single-marker iteration (r_n = |u0| |factor|^(n-1))
    on the GPU: pass counts, residual and F_total for the tolerance stop,
    the N_min floor, the N_max cap and the divergence guard."""
    u0, ds = 0.05, 0.35
    a = (3 / 8) ** 2 * ds
    feq = oracle.equilibrium(1.0, u0, 0.0)
    cases = [((0.5, 5, 20, 1e-4), (9, 0.05 / 2 ** 9)), ((0.5, 5, 20, 0.1), (5, 0.05 / 2 ** 5)),
             ((0.5, 5, 7, 1e-4), (7, 0.05 / 2 ** 6)), ((-1.0, 5, 12, 1e-4), (12, 0.05)),
             ((-2.0, 5, 20, 1e-4), (1, 0.1)), ((-1.4, 5, 6, 1e-4), (6, 0.05 * 1.4 ** 5))]
    for (factor, nmin, nmax, tol), (npass, res) in cases:
        say(f"single marker factor={factor} nmin={nmin} nmax={nmax} tol={tol}")
        om = (1 - factor) / a
        D = ds / math.pi
        case = dict(nx=24, ny=22, collision=ib.BGK, tau=0.8, bc=(ib.PERIODIC,) * 4,
                    bodies=[dict(xc=10.3 - D / 2, yc=9.71, diameter=D, n_markers=1, scheme=ib.MDF,
                                 kernel=ib.PESKIN4, mdf_iters=nmax, mdf_nmin=nmin, mdf_tol=tol,
                                 mdf_omega=om)])
        sim = ib.Sim(case)
        f = np.zeros((9, 22, 24))
        f[:] = feq[:, None, None]
        sim.set_populations(f)
        sim.step(1)
        st, m = sim.forces(0), sim.markers(0)[0]
        assert st["mdf_iters"] == npass
        assert abs(st["mdf_residual"] - res) < 1e-12 * res
        ftot = -2.0 * om * u0 * sum(factor ** n for n in range(npass))
        assert abs(m[4] - ftot) < 1e-12 * 2.0 * om * u0
        assert abs(st["slip_mean"] - u0 * abs(factor) ** npass) < 1e-12 * u0


# --------------------------- coupled multi-body MDF (Sec. 2.5.2, two-particle path)
def _coupled_markers_case(ds_list, omega, nmin=5, nmax=20, tol=1e-4):
    nx, ny = 40 * len(ds_list) + 40, 40
    bodies = []
    for i, ds in enumerate(ds_list):
        D = ds / math.pi
        bodies.append(dict(xc=30.0 + 40 * i + 0.3 - D / 2, yc=20.4, diameter=D, n_markers=1,
                           scheme=ib.MDF, kernel=ib.PESKIN4, mdf_iters=nmax, mdf_nmin=nmin,
                           mdf_tol=tol, mdf_omega=omega, mdf_coupled=1))
    return dict(nx=nx, ny=ny, collision=ib.BGK, tau=0.8, bc=(ib.PERIODIC,) * 4, bodies=bodies)


@pytest.mark.parametrize("spread", [ib.SPREAD_GATHER, ib.SPREAD_ATOMIC])
def test_coupled_mdf_single_marker_closed_forms_gpu(spread):
    """The closed forms of the coupled path on the GPU (both IB kernel
    instances; the bodies' workgroups exchange their residuals): the 0.8 cap
    with the joint residual, rejection with halving, and the stop at 1/8 of
    the initial relaxation, against the oracle and the formulas."""
    u0 = 0.05
    feq = oracle.equilibrium(1.0, u0, 0.0)
    for ds_list, omega, npass, res in (
            ((0.35, 0.9), 0.0, 20, u0 * (1 - 0.8 * 0.35 * (3 / 8) ** 2) ** 20),
            ((20.0, 20.0), 1.0, 5, u0 * 0.125 ** 5),
            ((80.0,), 1.0, 0, u0)):
        say(f"coupled single markers ds={ds_list} omega={omega} spread={spread}")
        case = _coupled_markers_case(ds_list, omega)
        sim, ref = make_pair(case)
        sim.set_spread(spread)
        f = np.zeros((9, case["ny"], case["nx"]))
        f[:] = feq[:, None, None]
        sim.set_populations(f)
        ref.set_populations(f)
        sim.step(1)
        ref.step(1)
        for b in range(len(ds_list)):
            st, fr = sim.forces(b), ref.body_state(b)
            assert st["mdf_iters"] == npass == fr["mdf_iters"], b
            assert abs(st["mdf_residual"] - res) < 1e-12 * u0, b
            mg, mo = sim.markers(b)[0], ref.markers(b)[0]
            assert abs(mg[4] - mo[4]) < 1e-13 * u0 and abs(mg[5] - mo[5]) < 1e-15, b
        assert rel(sim.populations(), ref.populations()) < F64_FIELD


def _coupled_decision_margin(rs, nmin, tol):
    """Smallest relative distance of the oracle's coupled-path residuals from
    the thresholds its decisions compared them with (1.2 R for each trial,
    the tolerance for each kept residual once nmin passes are kept)."""
    m = math.inf
    R, kept = rs[0], 0
    if kept >= nmin:
        m = min(m, abs(R - tol) / tol)
    for rt in rs[1:]:
        m = min(m, abs(rt - 1.2 * R) / (1.2 * R))
        if not rt > 1.2 * R:
            R, kept = rt, kept + 1
            if kept >= nmin:
                m = min(m, abs(R - tol) / tol)
    return m


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("free", [False, True])
def test_coupled_mdf_pair_step_by_step(prec, free):
    """Two MDF / P4 bodies on the coupled path, the paper's bounds N in
    [5, 20] and tolerance 1e-4: fixed bodies in a channel, or a settling
    pair (density ratios 1.5 and 1.25, Velocity-Verlet with the Feng
    correction).  Every step's kept-pass count equals the oracle's; the
    oracle's residuals stay at least 1e-4 (relative) from the thresholds of
    its decisions; forces and fields at the stated tolerances."""
    say(f"coupled MDF pair free={free} prec={prec}")
    if free:
        case = ib_cases.sedimentation(pair=True, nx=90, ny=200, diameter=12.0)
        case["gravity"] = (0.0, -1e-4)
        for b, (x, y, rr) in zip(case["bodies"], ((44.0, 140.0, 1.5), (46.5, 168.0, 1.25))):
            b.update(xc=x, yc=y, density_ratio=rr, scheme=ib.MDF, kernel=ib.PESKIN4,
                     mdf_coupled=1, **ib_cases.ADAPTIVE_MDF)
    else:
        case = body_case(ib.MDF, ib.PESKIN4, ib.TRT, nx=160, ny=70, D=12.0)
        case["bodies"][0].update(xc=40.3, yc=24.6, mdf_coupled=1, **ib_cases.ADAPTIVE_MDF)
        case["bodies"].append(dict(case["bodies"][0], xc=70.7, yc=45.2))
    sim, ref = make_pair(case, prec)
    f64 = prec == ib.FP64
    counts = []
    for t in range(1, 41):
        sim.step(1)
        ref.step(1)
        rs = ref.mdf_residuals(0)
        assert _coupled_decision_margin(rs, 5, 1e-4) > 1e-4, (t, rs)
        for b in range(2):
            fs, fr = sim.forces(b), ref.body_state(b)
            assert fs["mdf_iters"] == fr["mdf_iters"], (t, b, fs["mdf_iters"], fr["mdf_iters"])
            tl = F64_DRAG if f64 else F32_DRAG
            assert abs(fs["fy"] - fr["fy"]) < tl * max(abs(fr["fy"]), abs(fr["fx"])) + 1e-15, (t, b)
            assert abs(fs["mdf_residual"] - fr["mdf_residual"]) <= (1e-9 if f64 else 1e-3) * fr["mdf_residual"] + 1e-16
        counts.append(int(fr["mdf_iters"]))
    say(f"  kept passes per step: {counts}")
    ftol = F64_FIELD if f64 else F32_FIELD
    if free and f64:
        # The settling pair moves at 8e-4 after 40 steps, a thousandth of the
        # populations' scale: the oracle itself, its populations perturbed
        # once by 1e-16 (relative), ends 2e-12 away in this measure, and
        # 3e-12 when perturbed every step.
        ftol = 1e-11
    assert compare_fields(sim, ref, None) < ftol


def test_coupled_mdf_is_rejected_where_it_cannot_run():
    case = body_case(ib.MDF, ib.PESKIN4, ib.TRT, nx=160, ny=70, D=12.0)
    case["bodies"][0].update(xc=40.3, yc=24.6, mdf_coupled=1, **ib_cases.ADAPTIVE_MDF)
    other = dict(case["bodies"][0], xc=70.7, yc=45.2)
    sim = ib.Sim(dict(case, bodies=[case["bodies"][0]]))
    with pytest.raises(ib.IbLbmError):
        sim.add_body(dict(other, mdf_coupled=0))
    with pytest.raises(ib.IbLbmError):
        sim.add_body(dict(other, mdf_tol=1e-3))
    sim.close()
    b = ib.Batch(precision=ib.FP64)
    s2 = ib.Sim(case)
    with pytest.raises(ib.IbLbmError):
        b.attach(s2)


def test_adaptive_mdf_full_size_window():
    """2000x800, D = 80, MDF P4 TRT with the paper's adaptive bounds, FP64,
    through the split (pipelined) step of this lattice."""
    say("2000x800 adaptive MDF window")
    case = ib_cases.unsteady_cylinder(scheme="MDF", kernel="P4", collision="TRT", re=100.0)
    case["bodies"][0].update(ib_cases.ADAPTIVE_MDF)
    sim, ref = make_pair(case)
    for _ in range(4):
        sim.step(1)
        ref.step(1)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert decision_margin(ref.mdf_residuals(0), 5, 1e-4) > 1e-6
        assert fs["mdf_iters"] == fr["mdf_iters"]
        assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < F64_DRAG
    assert rel(sim.populations(), ref.populations()) < F64_FIELD


def test_adaptive_mdf_bounds_are_checked():
    for bad in (dict(mdf_nmin=0, mdf_iters=5, mdf_tol=1e-4), dict(mdf_nmin=6, mdf_iters=5, mdf_tol=1e-4)):
        case = body_case(ib.MDF, ib.PESKIN4, ib.TRT, **bad)
        with pytest.raises(ib.IbLbmError):
            ib.Sim(case)


# --------------------------------- boundary diagnostics (Sec. 2.8, Sec. 4.2)
DIAG_GPU = [(ib.DF, ib.HAT, ib.FIXED), (ib.MDF, ib.PESKIN4, ib.PRESCRIBED_SIN),
            (ib.DFC, ib.PESKIN4, ib.FIXED), (ib.DFC, ib.HAT, ib.FREE)]


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("scheme,kernel,motion", DIAG_GPU)
def test_diagnostics_match_oracle(scheme, kernel, motion, prec):
    """Slip, leakage flux, internal residual (kappa 0 and 2) and the marker
    profiles on the device against the oracle after 30 steps.  Velocity
    quantities are divided by u_ref, so they are held to the field tolerance
    times max|u|/u_ref; the pressure deviation in FP32 to 1e-7, above the
    density error of the FP32 store (nine populations of at most 0.1 rounded
    to 2^-24 relative: 5e-8 in rho, 2e-8 in rho/3)."""
    say(f"diagnostics scheme={scheme} kernel={kernel} motion={motion} prec={prec}")
    case = body_case(scheme, kernel, ib.TRT, motion=motion, amp=(0.0, 3.2), freq=0.004,
                     density_ratio=3.0)
    sim, ref = make_pair(case, prec)
    sim.step(30)
    ref.step(30)
    uref = 0.06
    _, rx, ry = ref.fields()
    umax = float(np.hypot(rx, ry).max())
    f64 = prec == ib.FP64
    tv = (F64_FIELD if f64 else F32_FIELD) * umax / uref
    tdp = 1e-15 if f64 else 1e-7
    for kappa in (0, 2):
        gs, gp = sim.diagnostics(0, kappa, uref)
        rs, rp = ref.diagnostics(0, kappa, uref)
        say(f"  kappa={kappa} slip {gs['slip_mean']:.4e} leak {gs['phi_leak']:.3e} "
            f"inside {gs['u_inside_mean']:.4e} n {gs['n_inside']:.0f}")
        assert gs["n_inside"] == rs["n_inside"] and gs["n_inside"] > 0
        for k in ("slip_mean", "slip_max", "phi_leak", "u_inside_mean", "u_inside_max"):
            assert abs(gs[k] - rs[k]) < tv, k
        assert abs(gs["dp_mean"] - rs["dp_mean"]) < tdp
        assert abs(gs["force_mean"] - rs["force_mean"]) < (1e-11 if f64 else F32_DRAG) * rs["force_mean"]
        np.testing.assert_allclose(gp[:, [0, 4, 5]], rp[:, [0, 4, 5]], rtol=0, atol=tv)
        np.testing.assert_allclose(gp[:, 1], rp[:, 1], rtol=0, atol=tdp)
        np.testing.assert_allclose(gp[:, 3], rp[:, 3], rtol=0, atol=3 * tdp)
        np.testing.assert_allclose(gp[:, 2], rp[:, 2], rtol=1e-11 if f64 else F32_DRAG,
                                   atol=1e-11 * rp[:, 2].max())


def test_diagnostics_state_and_arguments():
    case = body_case(ib.DF, ib.HAT, ib.BGK)
    sim = ib.Sim(case)
    with pytest.raises(ib.IbLbmError):
        sim.diagnostics(0, 2, 0.06)  # no step completed yet
    sim.step(1)
    for kappa, uref in ((-1, 0.06), (2, 0.0)):
        with pytest.raises(ib.IbLbmError):
            sim.diagnostics(0, kappa, uref)
    # a buffer wider than the radius leaves no interior node
    sm, _ = sim.diagnostics(0, 9, 0.06)
    assert sm["n_inside"] == 0 and sm["u_inside_mean"] == 0.0


# ------------------------------------------------------------- properties
@pytest.mark.parametrize("col", [ib.BGK, ib.TRT, ib.CMMRT])
def test_fp32_collision_returns_the_momentum(col):
    """A periodic box without force conserves total momentum exactly; in
    FP32 the collision may only add rounding that does not accumulate.  A
    momentum-carrying constant rounded to FP32 (3w = 1/3 in binary is 3e-8
    off) would add that fraction of s_o j at every node and step: 2e-4 of
    the momentum over 8000 steps here, against a bound of 2e-6."""
    say(f"fp32 momentum drift col={col}")
    n, u0 = 64, 0.05
    case = dict(nx=n, ny=n, collision=col, tau=0.62, bc=(ib.PERIODIC,) * 4, bodies=[])
    rng = np.random.default_rng(0)
    ux = u0 + 0.01 * rng.standard_normal((n, n))
    uy = 0.01 * rng.standard_normal((n, n))
    f0 = np.zeros((9, n, n))
    for j in range(n):
        for i in range(n):
            f0[:, j, i] = oracle.equilibrium(1.0, ux[j, i], uy[j, i])
    sim = ib.Sim(case, precision=ib.FP32_SHIFTED)
    sim.set_populations(f0)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])[:, None, None]
    j0 = (sim.populations() * ex).sum()
    sim.step(8000)
    j1 = (sim.populations() * ex).sum()
    sim.close()
    assert abs(j1 / j0 - 1) < 2e-6, (j0, j1)


def test_run_to_run_bitwise_and_gather_vs_atomic():
    case = body_case(ib.MDF, ib.PESKIN4, ib.CMMRT)
    a = ib.Sim(case); b = ib.Sim(case); c = ib.Sim(case)
    c.set_spread(ib.SPREAD_ATOMIC)
    for s in (a, b, c):
        s.step(30)
    np.testing.assert_array_equal(a.populations(), b.populations())
    assert rel(c.populations(), a.populations()) < 1e-13
    assert abs(c.forces(0)["fx"] - a.forces(0)["fx"]) < 1e-12 * abs(a.forces(0)["fx"])
    dcase = body_case(ib.DFC, ib.HAT, ib.TRT)
    d = ib.Sim(dcase); e = ib.Sim(dcase)
    e.set_spread(ib.SPREAD_ATOMIC)
    d.step(20); e.step(20)
    assert rel(e.populations(), d.populations()) < 1e-13


@pytest.mark.parametrize("scheme,kernel", [(ib.MDF, ib.PESKIN4), (ib.DF, ib.HAT), (ib.DFC, ib.PESKIN4)])
def test_ib_workgroup_size_changes_rounding_only(scheme, kernel):
    """The IB pass at 256, 512 and 1024 threads per body: the same result up
    to the order of the force sums, and the oracle's within tolerance."""
    say(f"IB workgroup sizes scheme={scheme} kernel={kernel}")
    case = body_case(scheme, kernel, ib.TRT)
    ref = oracle.OracleSim(case)
    ref.add_body(case["bodies"][0])
    ref.step(20)
    _, rx, ry = ref.fields()
    out = []
    for t in (256, 512, 1024):
        s = ib.Sim(case)
        s.set_launch(64, 2, 1, 1, ib_threads=t)
        assert s.get_launch()["ib_threads"] == t
        s.step(20)
        out.append((s.populations(), s.forces(0)["fx"]))
        assert compare_fields(s, ref, None) < F64_FIELD
        s.close()
    for f, fx in out[1:]:
        assert rel(f, out[0][0]) < 1e-13
        assert abs(fx - out[0][1]) < 1e-12 * abs(out[0][1])


def test_graph_replay_matches_direct_launches():
    case = body_case(ib.DFC, ib.PESKIN4, ib.TRT)
    a = ib.Sim(case); g = ib.Sim(case)
    g.set_graph(5)
    for rep in range(3):
        a.step(10)
        g.step(10)
        # eager work between replays
        _ = g.forces(0)
        np.testing.assert_array_equal(a.populations(), g.populations())
    assert g.steps_done == 30


def test_batch_matches_alone():
    import torch
    cases = [body_case(ib.DF, ib.HAT, ib.BGK, nx=96, ny=48, D=12.0),
             body_case(ib.MDF, ib.PESKIN4, ib.TRT, nx=150, ny=70, D=14.0),
             body_case(ib.DFC, ib.PESKIN4, ib.CMMRT, nx=81, ny=63, D=10.0),
             dict(nx=40, ny=30, tau=0.8, bc=(ib.PERIODIC,) * 4, bodies=[]),
             # open faces in the TRT group: the group takes the general face
             # instance, which must give the east-outflow case above the same
             # bits as its own instance does alone
             dict(body_case(ib.MDF, ib.PESKIN4, ib.TRT, nx=90, ny=60, D=12.0),
                  bc=(ib.ZERO_GRADIENT,) * 4)]
    targets = [25, 40, 33, 17, 29]
    alone = []
    for c, t in zip(cases, targets):
        s = ib.Sim(c, precision=ib.FP32_SHIFTED)
        s.step(t)
        alone.append(s.populations())
    stream = torch.cuda.current_stream().cuda_stream
    batch = ib.Batch(ib.FP32_SHIFTED, stream=stream)
    sims = [ib.Sim(c, precision=ib.FP32_SHIFTED, stream=stream) for c in cases]
    for s, t in zip(sims, targets):
        batch.attach(s, target=t)
    batch.set_graph(4)
    batch.step(50)
    batch.sync()
    for s, t, ref in zip(sims, targets, alone):
        assert s.steps_done == t
        np.testing.assert_array_equal(s.populations(), ref)


def test_history_matches_forces():
    case = body_case(ib.MDF, ib.HAT, ib.BGK)
    s = ib.Sim(case, history_capacity=64)
    rows = []
    for _ in range(5):
        s.step(1)
        rows.append(s.forces(0))
    h = s.history(0, 1, 5)
    for i, r in enumerate(rows):
        assert h[i, 0] == i + 1
        assert h[i, 1] == r["fx"] and h[i, 2] == r["fy"] and h[i, 3] == r["torque"]

    # a ring of 7 rows read across its wrap (rows 9..15 sit at 1..6 and 0)
    w = ib.Sim(case, history_capacity=7)
    rows = []
    for _ in range(15):
        w.step(1)
        rows.append(w.forces(0))
    h = w.history(0, 9, 7)
    for i in range(7):
        assert h[i, 0] == 9 + i and h[i, 1] == rows[8 + i]["fx"]
    h = w.history(0, 13, 2)
    assert list(h[:, 0]) == [13, 14]
    with pytest.raises(ib.IbLbmError):
        w.history(0, 8, 2)  # row 8 has been overwritten


# ------------------------------------------------------------- edge cases
@pytest.mark.parametrize("motion", [ib.FIXED, ib.FREE])
@pytest.mark.parametrize("scheme", [ib.MDF, ib.DFC])
def test_large_body_support_tables(motion, scheme):
    """A body of diameter 220 (radius well above the 98 at which the
    support tables were once sized too small): the capacity flag stays
    clear and forces and fields match the oracle over a few steps, for a
    fixed and a free (moving) body."""
    say(f"large body D=220 motion={motion} scheme={scheme}")
    case = dict(nx=300, ny=290, collision=ib.TRT, tau=0.62, trt_magic=0.25,
                bc=(ib.BOUNCE_BACK,) * 4, gravity=(0.0, -2e-5),
                bodies=[dict(xc=150.37, yc=146.21, diameter=220.0, scheme=scheme,
                             kernel=ib.PESKIN4, mdf_iters=5, motion=motion, density_ratio=1.4,
                             internal_mass=ib.IM_FENG)])
    sim, ref = make_pair(case)
    for _ in range(3):
        sim.step(4)
        ref.step(4)
        fs, fr = sim.forces(0), ref.body_state(0)
        assert fs["flags"] == 0
        assert abs(fs["fy"] - fr["fy"]) < F64_DRAG * max(abs(fr["fy"]), 1e-12)
    assert rel(sim.populations(), ref.populations()) < F64_FIELD


def test_invalid_configurations_are_rejected():
    base = dict(nx=40, ny=30, tau=0.8, bc=(ib.PERIODIC,) * 4)
    for bad in (dict(base, tau=0.5), dict(base, bc=(ib.PERIODIC, ib.BOUNCE_BACK, 0, 0)),
                dict(base, bc=(ib.PERIODIC, ib.PERIODIC, ib.VEL_PARABOLIC, 1)),
                dict(base, bc=(ib.ZERO_GRADIENT, 7, 1, 1)), dict(base, nx=2)):
        with pytest.raises(ib.IbLbmError):
            ib.Sim(bad)


def test_body_outside_lattice_is_rejected():
    case = dict(nx=40, ny=30, tau=0.8, bc=(ib.PERIODIC,) * 4)
    s = ib.Sim(case)
    with pytest.raises(ib.IbLbmError) as e:
        s.add_body(dict(xc=4.0, yc=15.0, diameter=8.0, kernel=ib.PESKIN4))
    assert e.value.status == -5
    with pytest.raises(ib.IbLbmError):
        s.add_body(dict(xc=20.0, yc=15.0, diameter=8.0, scheme=ib.MDF, mdf_iters=0))


def test_body_reaching_wall_halts_like_the_oracle():
    case = dict(nx=40, ny=60, collision=ib.BGK, tau=0.8, bc=(ib.BOUNCE_BACK,) * 4,
                gravity=(0.0, -2e-3),
                bodies=[dict(xc=20.0, yc=22.0, diameter=10.0, scheme=ib.DFC, kernel=ib.PESKIN4,
                             motion=ib.FREE, density_ratio=3.0)])
    sim, ref = make_pair(case)
    r = 0
    for _ in range(400):
        r = ref.step(1)
        if r != 0:
            break
    assert r == -5
    n_ok = ref.steps_done
    sim.step(400)
    st = sim.forces(0, check=False)
    assert st["status"] == -5 and st["flags"] & ib.ib_lbm.FLAG_RANGE
    assert sim.steps_done == n_ok


def test_empty_lattice_and_zero_steps():
    case = dict(nx=5, ny=4, tau=0.9, bc=(ib.PERIODIC,) * 4)
    sim, ref = make_pair(case, pops=ib_cases.random_populations(5, 4, 9))
    sim.step(0)
    assert sim.steps_done == 0
    sim.step(7)
    ref.step(7)
    assert rel(sim.populations(), ref.populations()) < F64_FIELD


# ------------------------------------------------------------- split step
def _split_case(scheme, kernel, col, motion=ib.FIXED):
    body = dict(xc=101.37, yc=79.8, diameter=24.0, scheme=scheme, kernel=kernel, mdf_iters=5,
                motion=motion)
    if motion == ib.PRESCRIBED_SIN:
        body.update(amp=(0.0, 4.0), freq=0.01, phase=0.3)
    return dict(nx=400, ny=160, collision=col, tau=0.62, trt_magic=0.25, cm_s_q=1.2,
                cm_s_eps=1.4, bc=(ib.VEL_UNIFORM, ib.ZERO_GRADIENT, ib.VEL_UNIFORM, ib.VEL_UNIFORM),
                u_bc=0.08, bodies=[body])


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("scheme,kernel,col,motion", [
    (ib.DF, ib.HAT, ib.BGK, ib.FIXED), (ib.MDF, ib.PESKIN4, ib.TRT, ib.FIXED),
    (ib.DFC, ib.PESKIN4, ib.CMMRT, ib.FIXED), (ib.MDF, ib.PESKIN4, ib.TRT, ib.PRESCRIBED_SIN),
    (ib.DFC, ib.HAT, ib.TRT, ib.PRESCRIBED_SIN)])
def test_split_step_is_bitwise_the_plain_step(scheme, kernel, col, motion, prec):
    """Pipelined steps (the collide-stream of step n+1 overlapping the IB
    pass of step n, with only the tiles next to the body waiting for it)
    and fused steps (one launch per step, the IB pass colliding its support
    itself; fixed DF/MDF bodies with BGK or TRT) change no bit of the
    result, with direct launches and mixed with graph replays, over several
    calls."""
    say(f"split step scheme={scheme} kernel={kernel} col={col} motion={motion} prec={prec}")
    case = _split_case(scheme, kernel, col, motion)
    fusable = motion == ib.FIXED and scheme != ib.DFC and col != ib.CMMRT
    runs = []
    for overlap, fused, graph in ((False, False, 0), (True, False, 0), (True, False, 7),
                                  (True, True, 0), (True, True, 7)):
        sim = ib.Sim(case, precision=prec)
        sim.set_launch(64, 1, 1, 1)
        sim.set_overlap(overlap)
        sim.set_fused(fused)
        if graph:
            sim.set_graph(graph)
        for n in (1, 20, 29):
            sim.step(n)
        sim.sync()
        used, near = sim.overlap()
        assert used == overlap
        assert sim.fused() == (fused and fusable)
        if overlap:
            assert 0 < near < case["nx"] * case["ny"] // 4
        runs.append((sim.populations(), sim.forces(0), sim.force()))
        sim.close()
    base = runs[0]
    for pops, st, (fx, fy) in runs[1:]:
        assert np.array_equal(pops, base[0])
        for k in ("fx", "fy", "torque", "slip_mean", "xc", "yc"):
            assert st[k] == base[1][k], k
        assert np.array_equal(fx, base[2][0]) and np.array_equal(fy, base[2][1])


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_split_step_with_zou_he_walls(prec):
    """A body in a force-driven channel between Zou-He walls: the wall pass
    runs after the face nodes in both the plain and the pipelined step; the
    two are bitwise equal and match the oracle."""
    say(f"split step, Zou-He channel, prec={prec}")
    case = _split_case(ib.MDF, ib.PESKIN4, ib.TRT)
    case.update(bc=(ib.PERIODIC, ib.PERIODIC, ib.ZOU_HE, ib.ZOU_HE), u_bc=0.0,
                fluid_force=(4e-6, 0.0))
    runs = []
    for overlap in (False, True):
        sim = ib.Sim(case, precision=prec)
        sim.set_launch(64, 1, 1, 1)
        sim.set_overlap(overlap)
        sim.step(1)
        sim.step(24)
        assert sim.overlap()[0] == overlap
        runs.append((sim.populations(), sim.forces(0)))
    assert np.array_equal(runs[0][0], runs[1][0])
    ref = oracle.OracleSim(case)
    ref.add_body(case["bodies"][0])
    ref.step(25)
    fs, fr = runs[1][1], ref.body_state(0)
    f64 = prec == ib.FP64
    assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < (F64_DRAG if f64 else F32_DRAG)
    if f64:
        assert rel(runs[1][0], ref.populations()) < F64_FIELD


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_split_step_body_one_tile_from_zou_he_wall(prec):
    """A fixed body as close to a Zou-He wall as the pipelined step allows:
    rounded to tiles of 4 rows the hold rectangle covers row 1, whose pushes
    the wall pass of the same step rebuilds the wall from.  Plain and
    pipelined steps are bitwise equal and match the oracle."""
    say(f"split step, body one tile from a Zou-He wall, prec={prec}")
    r = 12.0
    case = _split_case(ib.MDF, ib.PESKIN4, ib.TRT)
    case.update(bc=(ib.PERIODIC, ib.PERIODIC, ib.ZOU_HE, ib.ZOU_HE), u_bc=0.0,
                fluid_force=(4e-6, 0.0))
    case["bodies"][0].update(yc=r + 5.25, xc=90.6)
    runs = []
    for overlap in (False, True):
        sim = ib.Sim(case, precision=prec)
        sim.set_launch(64, 2, 2, 1)
        sim.set_overlap(overlap)
        sim.step(1)
        sim.step(19)
        sim.sync()
        used, near = sim.overlap()
        assert used == overlap
        runs.append((sim.populations(), sim.forces(0)))
        sim.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for k in ("fx", "fy", "torque"):
        assert runs[0][1][k] == runs[1][1][k], k
    ref = oracle.OracleSim(case)
    ref.add_body(case["bodies"][0])
    ref.step(20)
    fs, fr = runs[1][1], ref.body_state(0)
    f64 = prec == ib.FP64
    assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < (F64_DRAG if f64 else F32_DRAG)
    assert rel(runs[1][0], ref.populations()) < (F64_FIELD if f64 else 1e-5)


def test_zou_he_sims_stay_out_of_batches():
    case = dict(nx=40, ny=30, tau=0.8, bc=(ib.ZOU_HE,) * 4)
    b = ib.Batch(precision=ib.FP64)
    s = ib.Sim(case)
    with pytest.raises(ib.IbLbmError):
        b.attach(s)
    for bad in ((ib.ZOU_HE, ib.ZOU_HE, ib.BOUNCE_BACK, ib.ZOU_HE), (ib.ZOU_HE, 6, 5, 5)):
        with pytest.raises(ib.IbLbmError):
            ib.Sim(dict(case, bc=bad))


def test_split_step_matches_oracle_and_is_off_for_free_bodies():
    case = _split_case(ib.MDF, ib.PESKIN4, ib.CMMRT, ib.PRESCRIBED_SIN)
    sim, ref = make_pair(case)
    sim.set_launch(64, 2, 1, 1)
    sim.step(30)
    ref.step(30)
    assert sim.overlap()[0]
    assert rel(sim.populations(), ref.populations()) < F64_FIELD
    fs, fr = sim.forces(0), ref.body_state(0)
    assert abs(fs["fx"] - fr["fx"]) / abs(fr["fx"]) < F64_DRAG
    free = ib_cases.sedimentation(pair=False, nx=80, ny=200, diameter=12.0)
    free["bodies"][0].update(xc=40.0, yc=160.0)
    s2 = ib.Sim(free, precision=ib.FP64)
    s2.step(2)
    assert s2.overlap() == (False, 0)
    near_face = _split_case(ib.DF, ib.HAT, ib.BGK)
    near_face["bodies"][0].update(xc=14.0)
    s3 = ib.Sim(near_face, precision=ib.FP64)
    s3.step(2)
    assert s3.overlap() == (False, 0)


def test_benchmark_lattice_uses_split_step():
    case = ib_cases.unsteady_cylinder(scheme="MDF", kernel="P4", collision="TRT", re=100.0)
    sim = ib.Sim(case, precision=ib.FP32_SHIFTED)
    sim.step(3)
    used, near = sim.overlap()
    assert used and near < case["nx"] * case["ny"] // 25
    assert sim.fused()


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 1 << 22])
def test_stream_copy_copies_every_byte(nbytes):
    """The reference read + write stream (the benchmark's streaming ceiling)
    copies exactly, for sizes below, at and beyond one grid-stride round."""
    import torch
    say(f"stream copy {nbytes} bytes")
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    a = torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, generator=g).cuda()
    b = torch.zeros_like(a)
    for wg in (0, 1, 7):
        b.zero_()
        ib.stream_copy(a, b, wg)
        torch.cuda.synchronize()
        assert torch.equal(a, b), wg


def test_time_collide_stream_counts_inner_nodes():
    """The measurement entry point times back-to-back launches of the inner
    collide-stream and reports the inner node count (columns 1..nx-3, rows
    1..ny-2) that the roofline divides by."""
    case = dict(nx=130, ny=40, collision=ib.TRT, tau=0.8, bc=(ib.PERIODIC,) * 4)
    say("time_collide_stream 130x40")
    sim = ib.Sim(case, precision=ib.FP32_SHIFTED)
    try:
        us, n = sim.time_collide_stream(8)
    finally:
        sim.close()
    assert n == 127 * 38
    assert 0.0 < us < 1e5


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
@pytest.mark.parametrize("walls", [False, True])
def test_pipelined_graph_replay_is_bitwise_the_direct_steps(prec, walls):
    """Pipelined steps replayed from the explicitly built graph (4 steps per
    graph, both starting lattices) are bitwise the directly launched
    pipelined steps and the plain steps, over calls that mix replays and
    direct remainders, with eager work between the calls; with and without
    Zou-He walls (the wall pass is a node of its own)."""
    say(f"pipelined graph replay prec={prec} walls={walls}")
    case = _split_case(ib.MDF, ib.PESKIN4, ib.TRT)
    if walls:
        case.update(bc=(ib.PERIODIC, ib.PERIODIC, ib.ZOU_HE, ib.ZOU_HE), u_bc=0.0,
                    fluid_force=(4e-6, 0.0))
    sims = []
    configs = ((False, False, 0), (True, False, 0), (True, False, 4), (True, True, 4))
    for overlap, fused, graph in configs:
        sim = ib.Sim(case, precision=prec)
        sim.set_launch(64, 1, 1, 1)
        sim.set_overlap(overlap)
        sim.set_fused(fused)
        sim.set_graph(graph)
        sims.append(sim)
    for n in (5, 10, 3, 8):
        for sim in sims:
            sim.step(n)
        fx = [sim.forces(0)["fx"] for sim in sims]
        pops = [sim.populations() for sim in sims]
        assert [sim.overlap()[0] for sim in sims] == [False, True, True, True]
        # fused steps (captured as plain launches) only without the walls
        assert [sim.fused() for sim in sims] == [False, False, False, not walls]
        for k in range(1, len(sims)):
            assert fx[k] == fx[0], k
            assert np.array_equal(pops[k], pops[0]), k
    assert sims[2].steps_done == 26 and sims[3].steps_done == 26
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_fused_step_with_general_zero_gradient_faces(prec):
    """Fused steps on a channel whose south and north faces are zero-gradient
    as well (the face code's general copy rules, a kernel instance of its
    own) are bitwise the plain steps."""
    say(f"fused step, zero-gradient S/N faces, prec={prec}")
    case = _split_case(ib.MDF, ib.PESKIN4, ib.TRT)
    case.update(bc=(ib.VEL_UNIFORM, ib.ZERO_GRADIENT, ib.ZERO_GRADIENT, ib.ZERO_GRADIENT))
    runs = []
    for overlap in (False, True):
        sim = ib.Sim(case, precision=prec)
        sim.set_launch(64, 1, 1, 1)
        sim.set_overlap(overlap)
        sim.step(17)
        sim.step(6)
        assert sim.fused() == overlap
        runs.append((sim.populations(), sim.forces(0)))
        sim.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for k in ("fx", "fy", "torque", "slip_mean"):
        assert runs[0][1][k] == runs[1][1][k], k


def test_fused_step_after_collide_stream_timing_is_the_plain_step():
    """The collide-stream timing launches consume the IB force without an IB
    pass; fused steps afterwards (which keep their own copy of that force)
    still match plain steps bit for bit."""
    say("fused step after time_collide_stream")
    case = _split_case(ib.DF, ib.HAT, ib.BGK)
    runs = []
    for overlap in (False, True):
        sim = ib.Sim(case, precision=ib.FP32_SHIFTED)
        sim.set_launch(64, 1, 1, 1)
        sim.set_overlap(overlap)
        sim.step(9)
        sim.time_collide_stream(3)
        sim.step(11)
        assert sim.fused() == overlap
        runs.append((sim.populations(), sim.forces(0)))
        sim.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1]["fx"] == runs[1][1]["fx"]


def test_split_step_over_many_calls_is_the_plain_step():
    """Pipelined steps issued over many small calls (each IB launch of a
    pipelined step is replicated once per XCD and the first copy to start
    runs it, through a ticket advanced once per launch) give the plain
    steps' result bit for bit."""
    say("split step over 40 calls")
    case = _split_case(ib.MDF, ib.PESKIN4, ib.TRT)
    runs = []
    for overlap, fused in ((False, False), (True, False), (True, True)):
        sim = ib.Sim(case, precision=ib.FP32_SHIFTED)
        sim.set_launch(64, 1, 1, 1)
        sim.set_overlap(overlap)
        sim.set_fused(fused)
        for n in [1, 2, 3] * 13 + [1]:
            sim.step(n)
        sim.sync()
        assert sim.steps_done == 79
        assert sim.overlap()[0] == overlap
        assert sim.fused() == fused
        runs.append((sim.populations(), sim.forces(0)))
        sim.close()
    for r in runs[1:]:
        assert np.array_equal(runs[0][0], r[0])
        for k in ("fx", "fy", "torque", "slip_mean"):
            assert runs[0][1][k] == r[1][k], k
