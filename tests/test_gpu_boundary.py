"""C ABI behaviour on the device (needs an MI355X): input checks, the one-problem entry point,
per-dimension evaluation output and traces from plans.

* Lemma 1 needs sigma^2 > 0 (and finite inputs): an instance with a NaN or infinite entry in H or
  y, or sigma^2 = 0, is flagged DMALA_ERR_NONFINITE in the status output and skipped (symbols -1,
  NaN estimates), dmala_sync_status reports it, and the other instances of the batch are
  unaffected (bit for bit the outputs of a clean batch);
* dmala_detect_one gives exactly dmala_detect's result for one problem and returns
  DMALA_ERR_NONFINITE for a non-finite H.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.helpers import gpu_available, PREC_NP

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

OUTS = ("symbols", "marginals", "llrs", "best_energy", "final_state", "accept_count", "marginals_mc", "status")


def _run(b, precision, C=16, T=25, seed=4321):
    import torch
    import paper_2407_06042_amd as dm
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    det = dm.Detector(len(b.sigma2), b.nt, b.nr, b.M, C, T, seed, precision, outputs=OUTS)
    out = det(Hcm, y, s2)
    torch.cuda.synchronize()
    return det, {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_nonfinite_inputs_are_flagged_and_skipped(precision):
    import paper_2407_06042_amd as dm
    clean = W.make_batch(8, 8, 16, 14.0, 6, seed=31).as_precision(PREC_NP[precision])
    bad = W.Batch(clean.H.copy(), clean.y.copy(), clean.sigma2.copy(), clean.x_idx, clean.M)
    bad.H[1, 2, 3] = np.nan
    bad.sigma2[3] = 0.0
    bad.y[4, 5] = np.inf
    _, ref = _run(clean, precision)
    det, out = _run(bad, precision)
    flagged = [1, 3, 4]
    ok = [0, 2, 5]
    np.testing.assert_array_equal(out["status"], [0 if i in ok else -3 for i in range(6)])
    assert np.all(ref["status"] == 0)
    print("status", out["status"].tolist(), flush=True)
    for i in flagged:
        assert np.all(out["symbols"][i] == -1)
        for k in ("marginals", "llrs", "marginals_mc"):
            assert np.all(np.isnan(out[k][i])), k
        assert np.isnan(out["best_energy"][i])
        assert np.all(out["final_state"][i] == 0) and np.all(out["accept_count"][i] == 0)
    for k in OUTS:
        if k != "status":
            np.testing.assert_array_equal(out[k][ok], ref[k][ok])
    with pytest.raises(dm.DmalaError) as e:
        dm.sync_status(det.out["status"])
    assert e.value.status == -3 and "3 of 6" in str(e.value) and "instance 1" in str(e.value)
    dm.sync_status(_run(clean, precision)[0].out["status"])       # a clean batch passes


def test_detect_one_matches_detect_and_flags_nan_h():
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(12, 16, 64, 20.0, 1, seed=8).as_precision(np.float32)
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
    det = dm.Detector(1, 12, 16, 64, 24, 40, 99, "fp32", outputs=("symbols", "marginals"))
    ref = {k: v.cpu().numpy() for k, v in det(Hcm, y, s2).items()}
    sym, marg = dm.detect_one(Hcm[0].contiguous(), y[0].contiguous(), float(b.sigma2[0]), 64, 24, 40, 99,
                              constellation=W.qam_points(64))
    np.testing.assert_array_equal(sym.cpu().numpy(), ref["symbols"][0])
    np.testing.assert_array_equal(marg.cpu().numpy(), ref["marginals"][0])
    Hn = Hcm[0].clone()
    Hn[3, 5] = complex(float("nan"), 0.0)
    with pytest.raises(dm.DmalaError) as e:
        dm.detect_one(Hn, y[0].contiguous(), float(b.sigma2[0]), 64, 24, 40, 99)
    assert e.value.status == -3
    torch.cuda.synchronize()


def test_debug_eval_per_dimension_terms_sum_to_the_forward_log_q():
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(16, 16, 64, 22.0, 2, seed=19).as_precision(np.float32)
    rng = np.random.default_rng(0)
    xf = rng.integers(0, 8, size=(2, 64, 32))
    xt = np.where(rng.random(xf.shape) < 0.3, rng.integers(0, 8, size=xf.shape), xf)
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
    for prop in ("precond", "mhgd"):
        out, od = dm.debug_eval(Hcm, y, s2, 64, torch.from_numpy(xf).cuda(), torch.from_numpy(xt).cuda(),
                                proposal=prop, per_dim=True)
        out, od = out.cpu().numpy(), od.cpu().numpy()
        np.testing.assert_allclose(od.sum(-1), out[..., 0], rtol=1e-5, atol=1e-4)


def test_gradient_loop_runs_the_packed_contraction():
    """dmala_gx_loop (the G.X stage alone): deterministic, finite, and each loop depends on the last."""
    import torch
    import paper_2407_06042_amd as dm
    for nt, M in ((16, 16), (32, 64), (64, 64), (128, 256)):
        b = W.make_batch(nt, nt, M, 20.0, 5, seed=nt).as_precision(np.float32)
        Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
        for prec in ("bf16", "fp16"):
            g = dm.GxLoop(5, nt, nt, M, 48, prec)
            a = g(Hcm, y, s2, 7, run_setup=True).cpu().numpy().copy()
            a2 = g(Hcm, y, s2, 7).cpu().numpy().copy()
            c = g(Hcm, y, s2, 8).cpu().numpy().copy()
            torch.cuda.synchronize()
            assert np.all(np.isfinite(a)) and np.array_equal(a, a2), (nt, prec)
            assert not np.array_equal(a, c), (nt, prec)
