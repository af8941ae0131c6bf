"""Rounding of the fp32 chain against the float64 oracle on real trajectories (needs an MI355X).

The fp32 chain follows the oracle's trajectory exactly unless a draw's oracle margin is smaller
than the fp32 error of the quantity it compares (the near-tie rule of the parity tests).  This
test measures those errors on state pairs (x, x') taken from oracle trajectories of the
32x32 64-QAM sweep (16, 22, 28 dB, both proposals) and the 128x128 256-QAM rho = 0.5 system at
30 dB, evaluated on the device with the sampler's own code (dmala_debug_eval):

* per dimension, |log q_n(x'_n | x)_fp32 - log q_n(x'_n | x)_fp64|: an error delta in every
  log-probability moves each CDF value of the inverse-CDF draw by at most about delta (relative),
  so a categorical draw is safe when its oracle margin exceeds it;
* |log A_fp32 - log A_fp64| for the MH test, against the scale (E + E') / (tau sigma^2) of the
  tempered energies whose difference it contains.

It asserts that the thresholds of tests/helpers.py (EPS32) stay at least SAFETY times above the
measured maxima, and prints the figures the thresholds are derived from.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from tests.helpers import gpu_available, EPS32, EPS32_SAFETY, eps32_mh

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASES = [
    ("32x32 64-QAM 16 dB", dict(nt=32, M=64, snr=16.0, rho=0.0), "precond", 32, 100),
    ("32x32 64-QAM 22 dB", dict(nt=32, M=64, snr=22.0, rho=0.0), "precond", 32, 100),
    ("32x32 64-QAM 28 dB", dict(nt=32, M=64, snr=28.0, rho=0.0), "precond", 32, 100),
    ("32x32 64-QAM 28 dB naive", dict(nt=32, M=64, snr=28.0, rho=0.0), "naive", 32, 100),
    ("128x128 256-QAM rho 0.5 30 dB", dict(nt=128, M=256, snr=30.0, rho=0.5), "precond", 32, 60),
]


@pytest.mark.parametrize("name,shape,proposal,C,T", CASES, ids=[c[0] for c in CASES])
def test_fp32_rounding_against_the_oracle_on_trajectories(name, shape, proposal, C, T):
    import torch
    import paper_2407_06042_amd as dm
    nt, M = shape["nt"], shape["M"]
    b = W.make_batch(nt, nt, M, shape["snr"], 2, seed=int(shape["snr"]) + nt, rho=shape["rho"], cfg_id=2)
    b = b.as_precision(np.float32)
    rng = np.random.default_rng(nt)
    P = 1024
    xf = np.zeros((2, P, 2 * nt), np.int8)
    xt = np.zeros((2, P, 2 * nt), np.int8)
    ref_dim, ref_lr, scale = [], [], []
    for i in range(2):
        prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], M, proposal)
        o = odm.dmala_sample(prob, 0x5EED + i, i, C, T, trace="states")
        tr = o["trace"]
        pick = rng.choice(T * C, size=P, replace=False)
        kf = tr["k_from"].reshape(T * C, -1)[pick].astype(np.int64)
        kp = tr["k_prop"].reshape(T * C, -1)[pick].astype(np.int64)
        xf[i], xt[i] = kf, kp
        logq = odm.log_softmax(prob.proposal_logits(prob.x_of(kf)))          # (P, N, Q)
        ref_dim.append(np.take_along_axis(logq, kp[..., None], -1)[..., 0])
        ref_lr.append(tr["log_ratio"].reshape(-1)[pick])
        scale.append((tr["E_from"].reshape(-1)[pick] + tr["E_prop"].reshape(-1)[pick]) / (prob.tau * prob.sigma2))
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
    out, od = dm.debug_eval(Hcm, y, s2, M, torch.from_numpy(xf).cuda(), torch.from_numpy(xt).cuda(), proposal=proposal,
                            per_dim=True)
    out, od = out.cpu().numpy(), od.cpu().numpy()
    d_dim = np.abs(od - np.stack(ref_dim))
    d_la = np.abs(out[..., 3] - np.stack(ref_lr))
    sc = np.stack(scale)
    rel = d_la / sc
    print("near-ties %s: max|dlog q_n| %.3g (p99 %.3g); max|dlog A| %.3g (p99 %.3g); "
          "max|dlog A|/((E+E')/(tau s2)) %.3g; scale range %.3g..%.3g"
          % (name, d_dim.max(), np.percentile(d_dim, 99), d_la.max(), np.percentile(d_la, 99), rel.max(),
             sc.min(), sc.max()), flush=True)
    assert SAFETY_OK(d_dim.max(), EPS32[0]), (name, d_dim.max())
    assert np.all(EPS32_SAFETY * d_la <= eps32_mh(sc)), (name, d_la.max(), rel.max())


def SAFETY_OK(err, eps):
    return EPS32_SAFETY * err <= eps
