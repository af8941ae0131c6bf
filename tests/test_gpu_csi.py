"""Imperfect channel knowledge (Section IV-F setting, needs an MI355X): 16x16 16-QAM at 16.5 dB,
detection with H_hat = H + E over a sweep of the estimation NMSE.

The detector is unchanged (it sees H_hat); chains on H_hat still follow the oracle run on
H_hat, and the symbol error rate grows with the NMSE.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from tests.helpers import gpu_available, compare_chains

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_symbol_error_rate_against_channel_estimation_error():
    import torch
    import paper_2407_06042_amd as dm
    base = W.make_batch(16, 16, 16, 16.5, 512, seed=91)
    ser = {}
    for nmse in (None, -30.0, -20.0, -15.0, -10.0):
        b = (base if nmse is None else W.imperfect_csi(base, nmse, seed=1)).as_precision(np.float32)
        Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
        det = dm.Detector(512, 16, 16, 16, 32, 100, 17, outputs=("symbols", "final_state"), trace=True)
        out = det(Hcm, y, s2)
        sym = out["symbols"].cpu().numpy()
        ser[nmse] = float(np.mean(sym != b.x_idx))
        if nmse == -20.0:
            th = out["trace_hash"].cpu().numpy().view(np.uint32)
            for i in range(3):
                o = odm.detect(b.H[i], b.y[i], b.sigma2[i], 16, 32, 100, 17, instance=i, trace=True, estimators=False)
                ni, nf, bad = compare_chains(th[i], o, 2e-5, 2e-3)
                assert not bad, bad
    print("SER vs NMSE (dB):", ser, flush=True)
    sd = np.sqrt(0.25 / (512 * 16))
    assert ser[-10.0] > ser[-20.0] + 4 * sd > ser[None] + 4 * sd
    assert abs(ser[-30.0] - ser[None]) < 0.02
