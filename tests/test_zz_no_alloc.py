"""The allocation-free diagnostics entry point (ib_lbm_diagnostics_noalloc)
against ib_lbm_diagnostics, through the C ABI: two calls in a row, the second
on a body with fewer markers, and a body beyond the static staging."""
import sys

import numpy as np
import pytest

import paper_2609_02298_amd as ib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ib.load_library()


def _sim(nx, ny, D, nmarkers, prec):
    case = dict(nx=nx, ny=ny, collision=ib.TRT, tau=0.7, trt_magic=0.25,
                bc=(ib.VEL_UNIFORM, ib.ZERO_GRADIENT, ib.VEL_UNIFORM, ib.VEL_UNIFORM), u_bc=0.06,
                bodies=[dict(xc=nx / 3 + 0.37, yc=ny / 2 - 0.21, diameter=D, n_markers=nmarkers,
                             scheme=ib.MDF, kernel=ib.PESKIN4, mdf_iters=5)])
    return ib.Sim(case, precision=prec)


@pytest.mark.parametrize("prec", [ib.FP64, ib.FP32_SHIFTED])
def test_noalloc_diagnostics_match_the_allocating_call(prec):
    print(f"noalloc diagnostics prec={prec}", flush=True)
    sims = [_sim(160, 90, 30.0, 0, prec), _sim(96, 64, 14.0, 0, prec)]
    assert sims[0].nmarkers[0] > sims[1].nmarkers[0]
    for s in sims:
        s.step(12)
    for kappa in (2, 0):
        for s in sims:  # the second call stages fewer markers than the first
            a_sum, a_pm = s.diagnostics(0, kappa, 0.06)
            b_sum, b_pm = s.diagnostics_noalloc(0, kappa, 0.06)
            assert a_sum == b_sum
            assert np.array_equal(a_pm, b_pm)
    for s in sims:
        s.close()


def test_noalloc_diagnostics_rejects_a_body_beyond_the_staging():
    print("noalloc diagnostics, 9000 markers", flush=True)
    s = _sim(160, 90, 30.0, 9000, ib.FP64)
    # the marker count is checked before anything else (no step needed)
    with pytest.raises(ib.IbLbmError):
        s.diagnostics_noalloc(0, 2, 0.06)
    s.close()
