"""Host-side logic of the serving drivers (no device): FIFO latencies of
the sequential baseline and the latency percentiles."""
import numpy as np

from paper_2609_02298_amd import serving


def test_fifo_latencies_single_server_queue():
    # arrivals 0, 1, 1.5 with service 2, 0.5, 1: finishes 2, 2.5, 3.5
    assert serving.fifo_latencies([0.0, 1.0, 1.5], [2.0, 0.5, 1.0]) == [2.0, 1.5, 2.0]
    # an idle gap resets the queue
    assert serving.fifo_latencies([0.0, 10.0], [1.0, 1.0]) == [1.0, 1.0]
    # burst arrival: latencies are the running sums of service times
    lat = serving.fifo_latencies([0.0] * 4, [1.0, 2.0, 3.0, 4.0])
    assert lat == [1.0, 3.0, 6.0, 10.0]


def test_percentiles_match_numpy():
    rng = np.random.default_rng(0)
    v = rng.exponential(1.0, 1000)
    assert serving.percentile(v, 50) == np.percentile(v, 50)
    assert serving.percentile(v, 99) == np.percentile(v, 99)
    assert np.isnan(serving.percentile([], 50))


def test_summary_counts_and_spans():
    cases = [dict(nx=10, ny=10), dict(nx=20, ny=10)]
    served = dict(results=[dict(status=0, steps_done=100, t_submit=1.0, t_finish=2.0),
                           dict(status=0, steps_done=50, t_submit=1.5, t_finish=3.0)],
                  stats=dict(peak_resident=2, peak_resident_bytes=2**30, rounds=7))
    seq = dict(results=[dict(service=1.0), dict(service=1.0)], node_updates=100 * 100 + 200 * 50)
    s = serving.summary(cases, served, seq, arrivals=[0.0, 0.5])
    assert s["cases"] == 2 and s["failed"] == 0
    assert s["makespan_s"] == 2.0
    assert s["aggregate_mlups"] == round((100 * 100 + 200 * 50) / 2.0 / 1e6, 1)
    assert s["p50_latency_s"] == 1.25
    # sequential: finishes 1.0 and 2.0 -> latencies 1.0, 1.5; span 2.0
    assert s["sequential"]["makespan_s"] == 2.0
    assert s["sequential"]["p99_latency_s"] == round(np.percentile([1.0, 1.5], 99), 4)
    assert s["peak_resident_gb"] == 1.0


def test_sweep_keeps_cmmrt_cases_below_the_stability_limit():
    """No CM-MRT sweep case gets a relaxation time above the limit of the
    central-moment operator with s_q = 1.2, s_eps = 1.4; the capped cases
    say so, and the cap changes no other case."""
    import ib_cases
    capped = ib_cases.sweep_cases(256, seed=0)
    free = ib_cases.sweep_cases(256, seed=0, tau_max_cmmrt=1e9)
    for c, f in zip(capped, free):
        assert (c["nx"], c["ny"], c["collision"], c["steps"]) == (f["nx"], f["ny"], f["collision"],
                                                                f["steps"])
        if c["collision"] == ib_cases.CMMRT:
            assert c["tau"] <= ib_cases.CMMRT_TAU_MAX + 1e-12
        if c["cap"] == "cmmrt_tau_max":
            assert c["re_capped"] and f["tau"] > ib_cases.CMMRT_TAU_MAX
            assert abs(c["tau"] - ib_cases.CMMRT_TAU_MAX) < 1e-12
        else:
            assert c["tau"] == f["tau"]
    assert sum(c["cap"] == "cmmrt_tau_max" for c in capped) == 2


def test_sweep_keeps_trt_cases_above_the_floor():
    """No TRT sweep case gets a relaxation time below TRT_TAU_MIN; the
    lifted cases say so, and the floor changes no other case."""
    import ib_cases
    lifted = ib_cases.sweep_cases(256, seed=0)
    free = ib_cases.sweep_cases(256, seed=0, tau_min_trt=0.0)
    n = 0
    for c, f in zip(lifted, free):
        assert (c["nx"], c["ny"], c["collision"], c["steps"]) == (f["nx"], f["ny"], f["collision"],
                                                                f["steps"])
        if c["collision"] == ib_cases.TRT:
            assert c["tau"] >= ib_cases.TRT_TAU_MIN - 1e-12
        if c["cap"] == "trt_tau_min":
            n += 1
            assert f["tau"] < ib_cases.TRT_TAU_MIN and abs(c["tau"] - ib_cases.TRT_TAU_MIN) < 1e-12
        else:
            assert c["tau"] == f["tau"]
    assert n >= 3
