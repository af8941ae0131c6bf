"""dmala_detect_static (workspace in the library's fixed device array) against dmala_detect.

Two calls in a row through the C ABI, the second on a smaller batch of another
shape and precision: every output equals dmala_detect's bit for bit on the same
inputs (the same kernels run; only the workspace address differs).  A batch
beyond the array's size is refused on the host.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.helpers import gpu_available, PREC_NP

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

OUTS = ("symbols", "marginals", "llrs", "best_energy", "final_state", "accept_count", "marginals_mc")


def _pair(batch, C, T, seed, precision):
    import torch
    import paper_2407_06042_amd as dm
    b = batch.as_precision(PREC_NP[precision])
    n = len(b.sigma2)
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    kw = dict(outputs=OUTS, trace=True)
    ref = dm.Detector(n, b.nt, b.nr, b.M, C, T, seed, precision, **kw)
    sta = dm.Detector(n, b.nt, b.nr, b.M, C, T, seed, precision, **kw)
    assert ref.ws_bytes <= dm.STATIC_SCRATCH_BYTES
    r = {k: v.cpu().numpy() for k, v in ref(Hcm, y, s2).items()}
    for v in sta.out.values():
        v.fill_(-7)
    s = {k: v.cpu().numpy() for k, v in sta(Hcm, y, s2, static_scratch=True).items()}
    torch.cuda.synchronize()
    return r, s


def _check(r, s, tag):
    for k in r:
        assert np.array_equal(r[k], s[k], equal_nan=True), (tag, k)
    print(tag, "identical outputs:", sorted(r), flush=True)


def test_static_scratch_matches_caller_workspace_twice():
    # first call: 96 problems of 32x32 64-QAM, fp32; second: 7 problems of 8x12 16-QAM, bf16
    r, s = _pair(W.make_batch(32, 32, 64, 22.0, 96, seed=11, cfg_id=2), 32, 40, 0x5151, "fp32")
    _check(r, s, "call 1 (96 x 32x32 64-QAM fp32)")
    r, s = _pair(W.make_batch(8, 12, 16, 14.0, 7, seed=12), 20, 30, 0x5152, "bf16")
    _check(r, s, "call 2 (7 x 8x12 16-QAM bf16)")


def test_static_scratch_refuses_oversized_batches():
    import paper_2407_06042_amd as dm
    p = dm.make_params(32, 10, 1)
    need = dm.workspace_size(4096, 64, 64, 64, p)
    assert need > dm.STATIC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)
    o = dm.Outputs()
    st = dm.lib().dmala_detect_static(fake, fake, fake, 4096, 64, 64, 64, None, ctypes.byref(p), ctypes.byref(o), None)
    assert st == -4 and "static scratch" in dm.last_error()
