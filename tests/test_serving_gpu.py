"""GPU tests of the serving loop: a request served in a mix of other
requests, admitted under a device-memory budget and stepped in shared batch
launches, gives the same result as the same case stepped alone.

The bar is bitwise equality (every node update and every IB reduction reads
only its own case and has a fixed order), which is stricter than the FP32
shifted tolerance (velocity 1e-5, drag 1e-4 relative).  One FP64 request is
also checked against the FP64 oracle (velocity 1e-12, drag 1e-10).
"""
import sys
import time

import numpy as np
import pytest

import ib_cases
import paper_2609_02298_amd as ib
from paper_2609_02298_amd import serving

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ib.load_library()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


COMBOS = [(ib.DF, ib.HAT, ib.BGK), (ib.MDF, ib.PESKIN4, ib.TRT), (ib.DFC, ib.PESKIN4, ib.CMMRT),
          (ib.DFC, ib.HAT, ib.TRT), (ib.MDF, ib.HAT, ib.CMMRT), (ib.DF, ib.PESKIN4, ib.BGK),
          (ib.MDF, ib.PESKIN4, ib.BGK), (ib.DFC, ib.PESKIN4, ib.TRT)]
SIZES = [(96, 40), (128, 48), (160, 64), (112, 56), (144, 48), (120, 60), (200, 80), (104, 52)]
STEPS = [40, 75, 60, 23, 90, 51, 33, 64]


def mix_cases():
    return [ib_cases.channel_case(nx, ny, s, k, c, re=40.0 + 10 * i, steps=n, name=f"mix-{i}")
            for i, ((nx, ny), (s, k, c), n) in enumerate(zip(SIZES, COMBOS, STEPS))]


def alone(case, precision):
    sim = ib.Sim(case, precision=precision)
    sim.step(case["steps"])
    sim.sync()
    st = sim.forces(0, check=False)
    rho, ux, uy = sim.fields()
    n = sim.steps_done
    sim.close()
    return st, (rho, ux, uy), n


@pytest.mark.parametrize("precision", [ib.FP32_SHIFTED, ib.FP64], ids=["fp32", "fp64"])
def test_served_in_a_mix_equals_alone(precision):
    cases = mix_cases()
    fps = [ib.footprint(c, precision) for c in cases]
    # room for about three of them at once, so later ones queue and are
    # admitted as earlier ones retire
    budget = sum(sorted(fps)[-3:])
    say(f"serving {len(cases)} cases, budget {budget} B, precision {precision}")
    arrivals = [0.0, 0.0, 0.0, 0.002, 0.004, 0.02, 0.03, 0.05]
    out = serving.serve(cases, precision, arrivals=arrivals, hbm_budget=budget, max_resident=3,
                        quantum=16, fields=True, timeout=120.0)
    st = out["stats"]
    say(f"stats {st}")
    assert st["completed"] == len(cases) and st["failed"] == 0
    assert st["peak_resident"] <= 3
    assert st["peak_resident_bytes"] <= budget
    assert st["rounds"] >= 4
    for c, r in zip(cases, out["results"]):
        say(f"case {c['name']}: status {r['status']} steps {r['steps_done']} "
            f"wait {r['t_admit'] - r['t_submit']:.4f}s latency {r['latency']:.4f}s")
        assert r["status"] == 0
        assert r["steps_done"] == c["steps"]
        st_a, (rho, ux, uy), n = alone(c, precision)
        assert n == c["steps"]
        b = r["bodies"][0]
        for key in ("fx", "fy", "torque", "slip_mean", "slip_max", "mdf_residual"):
            assert b[key] == st_a[key], (c["name"], key, b[key], st_a[key])
        assert np.array_equal(r["rho"], rho), c["name"]
        assert np.array_equal(r["ux"], ux), c["name"]
        assert np.array_equal(r["uy"], uy), c["name"]


def test_served_fp64_matches_oracle():
    import oracle
    case = ib_cases.channel_case(120, 48, ib.DFC, ib.PESKIN4, ib.CMMRT, re=30.0, steps=40)
    out = serving.serve([case], ib.FP64, quantum=7, fields=True, timeout=60.0)
    r = out["results"][0]
    assert r["status"] == 0 and r["steps_done"] == 40
    ref = oracle.OracleSim(case)
    for b in case["bodies"]:
        ref.add_body(b)
    ref.step(40)
    rho, ux, uy = ref.fields()
    bs = ref.body_state(0)
    ref.close()
    scale = max(np.abs(ux).max(), np.abs(uy).max())
    assert np.abs(r["ux"] - ux).max() / scale <= 1e-12
    assert np.abs(r["uy"] - uy).max() / scale <= 1e-12
    fx = r["bodies"][0]["fx"]
    assert abs(fx - bs["fx"]) <= 1e-10 * abs(bs["fx"])


def test_server_rejections_and_pending():
    precision = ib.FP32_SHIFTED
    small = ib_cases.channel_case(96, 40, steps=20, name="small")
    big = ib_cases.channel_case(400, 200, steps=5, name="big")
    bad = dict(small, tau=0.4, name="bad-tau")
    outside = ib_cases.channel_case(96, 40, steps=5, name="outside")
    outside["bodies"] = [dict(outside["bodies"][0], xc=1.0)]
    budget = ib.footprint(small, precision) * 2
    srv = ib.Server(precision=precision, hbm_budget=budget, quantum=8)
    try:
        ids = [srv.submit(c, c["steps"]) for c in (small, big, bad, outside, small)]
        res = [srv.wait(i, 60.0) for i in ids]
        assert all(r is not None for r in res)
        codes = [r["status"] for r in res]
        say(f"statuses {codes}")
        assert codes == [0, -2, -1, -5, 0]
        assert res[0]["steps_done"] == 20 and res[4]["steps_done"] == 20
        with pytest.raises(ib.IbLbmError):
            srv.wait(10**9, 0.0)  # unknown id
        st = srv.stats()
        assert st["completed"] == 5 and st["failed"] == 3
        assert st["peak_resident_bytes"] <= budget
        # a long request is still running when waited on with a short limit
        rid = srv.submit(dict(small, steps=6000, name="long"), 6000)
        t0 = time.perf_counter()
        assert srv.wait(rid, 0.001) is None
        assert time.perf_counter() - t0 < 5.0
        r = srv.wait(rid, 120.0)
        assert r is not None and r["status"] == 0 and r["steps_done"] == 6000
    finally:
        srv.close()
