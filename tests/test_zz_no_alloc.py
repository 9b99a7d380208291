"""ba_lm_step_noalloc (the LM step with its per-step scratch in the library's static device
array) against ba_lm_step on the same inputs, through the C ABI: the solver is deterministic,
so reports and parameters must agree bit for bit. Calls in a row on one GPU share the array,
so the sequence runs a larger problem, then a smaller one, then the larger one again."""
import ctypes

import numpy as np
import pytest

from paper_2510_13310_amd import _abi
from scenes import make_scene
from tests._common import gpu_setup

pytestmark = pytest.mark.gpu

FIELDS = ("status", "accepted", "relinearized", "fixpoint_rounds", "pcg_iters",
          "pcg_breakdown", "n_cams_active", "n_points_active", "n_obs_active", "cost_before",
          "cost_after", "model_decrease", "gain_ratio", "lambda", "pcg_rel_residual", "rms_px",
          "grad_inf")


def _step(lib, ctx, fn):
    rep = _abi.BaStepReport()
    st = getattr(lib, fn)(ctx, ctypes.byref(rep))
    assert st >= 0, (fn, st, lib.ba_last_error(ctx))
    return _abi.struct_to_dict(rep)


def _same(a, b, steps):
    lib = _abi.load()
    for k in range(steps):
        ra = _step(lib, a.ctx, "ba_lm_step")
        rb = _step(lib, b.ctx, "ba_lm_step_noalloc")
        for f in FIELDS:
            assert ra[f] == rb[f], (k, f, ra[f], rb[f])
    ca, pa = a.get_params()
    cb, pb = b.get_params()
    np.testing.assert_array_equal(ca, cb)
    np.testing.assert_array_equal(pa, pb)
    np.testing.assert_array_equal(a.get_last_step()[0], b.get_last_step()[0])


def test_noalloc_step_equals_step_larger_then_smaller():
    big = make_scene("medium")
    small = make_scene("tiny", n_points=300)
    a1, b1 = gpu_setup(big, "mixed"), gpu_setup(big, "mixed")
    _same(a1, b1, 4)                         # the larger problem first
    a2, b2 = gpu_setup(small, "fp64"), gpu_setup(small, "fp64")
    _same(a2, b2, 3)                         # then a smaller one on the same array
    _same(a1, b1, 2)                         # and the larger one again


def test_noalloc_refusals():
    lib = _abi.load()
    sc = make_scene("tiny", n_points=100)
    for kw in (dict(timing=1), dict(solver="explicit")):
        ba = gpu_setup(sc, "fp64", **kw)
        rep = _abi.BaStepReport()
        assert lib.ba_lm_step_noalloc(ba.ctx, ctypes.byref(rep)) == -2
        ba.close()
    # 600k cameras need more camera-pass scratch than the static array holds
    from paper_2510_13310_amd import BundleAdjuster
    C = 600_000
    cams = np.zeros((C, 7))
    cams[:, 0] = 1.0
    cams[:, 6] = -5.0
    intr = np.tile([500.0, 320.0, 240.0], (C, 1))
    ba = BundleAdjuster(cams, intr, np.zeros((1, 3)), precision="fp64")
    ba.set_observations(np.array([0, 1], np.int32), np.array([0, 0], np.int32),
                        np.array([[320, 240], [320, 240]], np.float32))
    rep = _abi.BaStepReport()
    assert lib.ba_lm_step_noalloc(ba.ctx, ctypes.byref(rep)) == -1
    assert "static array" in lib.ba_last_error(ba.ctx).decode()
    assert ba.lm_step()["status"] == 1   # the ordinary step still runs (nothing active)
