"""Host-side statistics of the paper-scale studies (no GPU): drag / lift
coefficients and Strouhal numbers of force histories with known answers."""
import math

import numpy as np
import pytest

import ib_cases
from paper_2609_02298_amd.studies import (acceleration_proxy, flow_statistics, phase_peaks,
                                          stop_reason)


def test_statistics_of_a_pure_shedding_signal():
    """F_x constant, F_y a sinusoid of an integer number of periods: mean
    C_d, rms lift A/sqrt(2), amplitude A, and both Strouhal estimates equal
    f D / u (the FFT exactly, as f N is an integer)."""
    u, D, n = 0.1, 40.0, 20000
    f = 0.005  # 100 periods in the window
    t = np.arange(n)
    q = 0.5 * u * u * D
    fx = np.full(n, 1.35 * q)
    fy = 0.33 * q * np.sin(2 * math.pi * f * t + 0.3)
    s = flow_statistics(fx, fy, u, D)
    assert abs(s["cd_mean"] - 1.35) < 1e-12
    assert abs(s["cl_rms"] - 0.33 / math.sqrt(2)) < 1e-9
    # sampled 200 times a period, the extremes miss the peak by at most
    # 1 - cos(pi / 200) = 1.2e-4 relative
    assert abs(s["cl_amp"] - 0.33) < 1.3e-4 * 0.33
    assert abs(s["st_fft"] - f * D / u) < 1e-12
    assert abs(s["st_zero"] - f * D / u) < 1e-6 * f * D / u


def test_statistics_of_a_steady_wake():
    u, D = 0.1, 40.0
    q = 0.5 * u * u * D
    s = flow_statistics(np.full(500, 2.08 * q), np.zeros(500), u, D)
    assert abs(s["cd_mean"] - 2.08) < 1e-12
    assert s["st_fft"] is None and s["st_zero"] is None and s["cl_rms"] == 0.0


@pytest.mark.parametrize("re,nx,ny,D,nb,tau", [(20, 2001, 1601, 40.0, 188, 1.1),
                                                (100, 2001, 1601, 40.0, 188, 0.62),
                                                (200, 3001, 2401, 60.0, 283, 0.59)])
def test_paper_fixed_cylinder_parameters(re, nx, ny, D, nb, tau):
    """Table I: grid, diameter, marker count at spacing 2/3, tau = 1/2 + 3 nu
    (0.59 at Re = 200, as printed), cylinder at (0.4 L_x, 0.5 L_y)."""
    c = ib_cases.paper_fixed_cylinder(re)
    b = c["bodies"][0]
    assert (c["nx"], c["ny"], c["diameter"], b["n_markers"]) == (nx, ny, D, nb)
    assert abs(c["tau"] - tau) < 1e-12
    assert b["xc"] == 0.4 * (nx - 1) and b["yc"] == 0.5 * (ny - 1)
    assert b["mdf_tol"] == 1e-4 and (b["mdf_nmin"], b["mdf_iters"]) == (5, 20)


def test_peak_drag_of_a_periodic_force():
    """|C_d| peaks of a known periodic force: each period's maximum, their
    mean, and the window maximum."""
    from paper_2609_02298_amd.studies import peak_drag
    u, D, T = 0.1, 80.0, 4000
    t = np.arange(4 * T)
    q = 0.5 * u * u * D
    amp = np.repeat([2.0, 2.1, 2.05, 2.15], T)
    fx = q * amp * np.sin(2 * math.pi * t / T)
    p = peak_drag(fx, u, D, T)
    assert p["periods"] == 4
    assert abs(p["cd_peak"] - 2.075) < 1e-9 and abs(p["cd_max"] - 2.15) < 1e-9


def test_paper_inline_oscillation_parameters():
    """Sec. 2.9.2 / Table I: KC = 5, Re = 100, T = 4000, tau = 0.74, 2401 x
    1601, D = 80, open faces, A = KC D / (2 pi)."""
    c = ib_cases.paper_inline_oscillation()
    b = c["bodies"][0]
    assert (c["nx"], c["ny"], c["diameter"], c["period"]) == (2401, 1601, 80.0, 4000)
    assert abs(c["tau"] - 0.74) < 1e-12 and c["bc"] == (ib_cases.ZERO_GRADIENT,) * 4
    assert abs(b["amp"][0] + 5 * 80 / (2 * math.pi)) < 1e-12 and b["freq"] == 1 / 4000
    # velocity amplitude 2 pi f0 A = U_max
    assert abs(2 * math.pi * b["freq"] * abs(b["amp"][0]) - 0.1) < 1e-15


def test_paper_wake_interaction_parameters():
    """Sec. 2.9.4: 4001 x 801 over [0, 10] x [-1, 1] (spacing 0.0025), D = 80,
    heavy 1.5 at (0.8, -0.13), light 1.25 at (1.2, 0.13), gravity +x,
    tau = 0.59, Zou-He walls."""
    c = ib_cases.paper_wake_interaction()
    h, l = c["bodies"]
    assert (c["nx"], c["ny"], c["diameter"], c["tau"]) == (4001, 801, 80.0, 0.59)
    np.testing.assert_allclose([h["xc"], h["yc"], l["xc"], l["yc"]], [320, 348, 480, 452],
                               rtol=0, atol=1e-9)
    assert (h["density_ratio"], l["density_ratio"]) == (1.5, 1.25)
    assert c["gravity"] == (2.156e-4, 0.0) and c["bc"] == (ib_cases.ZOU_HE,) * 4
    assert abs(c["nu"] - 0.03) < 1e-15


@pytest.mark.parametrize("ratio,tau_printed", [(1.5, 0.56), (1.1, 0.64), (1.01, 0.95), (1.25, 1.41)])
def test_paper_settling_parameters(ratio, tau_printed):
    """Sec. 2.9.3 on 1281 x 3841 (D = 160): the Mach rule of Appendix A.1 at
    Ma = 0.064 gives each printed relaxation time to its two digits; the
    gravity velocity scale u_g is Ma c_s for every density ratio."""
    c = ib_cases.paper_settling(ratio)
    assert (c["nx"], c["ny"]) == (1281, 3841)
    assert round(c["tau"], 2) == tau_printed
    assert math.isclose(c["u_g"] * math.sqrt(3.0), 0.064, rel_tol=1e-12)
    b = c["bodies"][0]
    assert (b["xc"], b["yc"], b["diameter"], b["n_markers"]) == (640.0, 2560.0, 160.0, 754)
    assert c["bc"] == (ib_cases.ZOU_HE,) * 4 and c["gravity"][0] == 0.0 and c["gravity"][1] < 0


def test_stop_reasons():
    assert stop_reason(0) == "step budget"
    assert stop_reason(-5) == "wall or contact"
    assert stop_reason(-4) == "diverged"


def test_paper_settling_extended_channel():
    """App. C.2: the 60 D channel keeps the width, spacing and relaxation
    time and releases the particle 8 D below the top wall, so that its
    contact-safe fall is 51.5 D."""
    std, tall = ib_cases.paper_settling(1.5), ib_cases.paper_settling(1.5, height_d=60.0)
    assert (tall["nx"], tall["ny"]) == (1281, 9601)
    assert tall["tau"] == std["tau"] and tall["u_g"] == std["u_g"] and tall["nu"] == std["nu"]
    assert tall["bodies"][0]["yc"] == 8320.0 and std["bodies"][0]["yc"] == 2560.0
    assert (tall["ny"] - 1 - tall["bodies"][0]["yc"]) / 160.0 == 8.0
    assert tall["steps"] == 375000 and std["steps"] == 150000


def test_paper_settling_internal_mass_arm():
    """Table B.5: the scheme-(A) arm differs from the baseline only in the
    internal-mass treatment of the body."""
    a = ib_cases.paper_settling(1.5, internal_mass=ib_cases.IM_NONE)
    b = ib_cases.paper_settling(1.5)
    assert a["bodies"][0]["internal_mass"] == ib_cases.IM_NONE
    assert b["bodies"][0]["internal_mass"] == ib_cases.IM_FENG
    a["bodies"][0]["internal_mass"] = ib_cases.IM_FENG
    assert a == b


def test_acceleration_proxy_of_a_uniform_acceleration():
    """v = a t along a fixed direction: |dv*/dt*| = |a| D / u_g^2 at every
    record, ends included (Sec. 2.8)."""
    a, u_g, D, cad = (3e-7, -4e-7), 0.09, 80.0, 500
    t = cad * np.arange(1, 60)
    out = acceleration_proxy(a[0] * t, a[1] * t, u_g, D, cad)
    np.testing.assert_allclose(out, math.hypot(*a) * D / u_g ** 2, rtol=1e-12)


def test_acceleration_proxy_of_a_circular_motion():
    """v = V (cos w t, sin w t): |dv/dt| = V w, up to the central difference's
    sin(w h)/(w h) inside the record."""
    V, w, u_g, D, cad = 0.05, 2e-4, 0.1, 40.0, 100
    t = cad * np.arange(1, 200)
    out = acceleration_proxy(V * np.cos(w * t), V * np.sin(w * t), u_g, D, cad)
    h = w * cad
    np.testing.assert_allclose(out[1:-1], V * w * D / u_g ** 2 * math.sin(h) / h, rtol=1e-10)


def test_phase_peaks():
    t = np.arange(10.0)
    ah = np.array([1, 2, 1, 1, 9, 9, 1, 4, 1, 1.0])
    al = np.array([3, 1, 1, 1, 9, 9, 1, 1, 8, 1.0])
    p = phase_peaks(ah, al, t, t_closest=3.5, t_exchange=5.5)
    assert (p["pre_heavy"], p["pre_light"], p["post_heavy"], p["post_light"]) == (2, 3, 4, 8)
    assert p["ratio_pre"] == 1.5 and p["ratio_post"] == 2.0 and math.isclose(p["contrast"], 4 / 3)


def test_paper_wake_interaction_extended_channel():
    """Table C.3: the 60 D channel lengthens the domain at the same spacing,
    with the particles at the same starting nodes."""
    std, ext = ib_cases.paper_wake_interaction(), ib_cases.paper_wake_interaction(length_d=60.0)
    assert (std["nx"], std["ny"]) == (4001, 801) and (ext["nx"], ext["ny"]) == (4801, 801)
    assert [(b["xc"], b["yc"]) for b in ext["bodies"]] == [(b["xc"], b["yc"]) for b in std["bodies"]]
    assert ext["tau"] == std["tau"] and ext["gravity"] == std["gravity"]


def test_paper_settling_refined_grid():
    """App. C.5: D = 240 on 1921 x 5761 nodes, the release point and the
    gravity velocity scale unchanged in physical and Mach terms."""
    c = ib_cases.paper_settling(1.5, diameter=240.0)
    assert (c["nx"], c["ny"]) == (1921, 5761)
    b = c["bodies"][0]
    assert (b["xc"], b["yc"], b["n_markers"]) == (960.0, 3840.0, 1131)
    assert round(c["tau"], 3) == 0.596
    assert math.isclose(c["u_g"] * math.sqrt(3.0), 0.064, rel_tol=1e-12)
