"""The precision direction: error of every arithmetic form against the float64 oracle, per result
(needs an MI355X).

For the 32x32 64-QAM sweep (16, 22, 28 dB) and the 128x128 256-QAM rho = 0.5 system at 30 dB the
float64 oracle runs its own chains (same seed); the device runs fp32 (fp16-split contraction),
BF16 and FP16 gradients, and fp32 with another seed.  Reported per form: mean absolute error of
the symbol marginals and of the bit LLRs against the oracle's estimates, and the SER.  The fp32
chains are the oracle's (up to near-ties), so their error is rounding only; the BF16/FP16 chains
are different Markov chains on the same target (their gradient is quantised, the energy and the
MH test are exact), so their estimates differ from the oracle's by Monte Carlo error: the test
requires that error to be no larger than that of fp32 chains on an independent seed (plus a
small allowance for the finite number of problems).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from tests.helpers import gpu_available, run_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASES = [
    ("32x32 64-QAM 16 dB", lambda: W.make_batch(32, 32, 64, 16.0, 24, seed=216, cfg_id=2), 32, 100, None),
    ("32x32 64-QAM 22 dB", lambda: W.make_batch(32, 32, 64, 22.0, 24, seed=222, cfg_id=2), 32, 100, None),
    ("32x32 64-QAM 28 dB", lambda: W.make_batch(32, 32, 64, 28.0, 24, seed=228, cfg_id=2), 32, 100, None),
    ("128x128 256-QAM rho 0.5 30 dB", lambda: W.c4_correlated(n_inst=2, seed=404), 64, 200, [0, 31, 64, 97, 127]),
]


@pytest.mark.parametrize("name,make,C,T,ants", CASES, ids=[c[0] for c in CASES])
def test_error_against_the_fp64_oracle_per_form(name, make, C, T, ants):
    batch = make()
    seed = 0x5EC0 + C + T
    forms = [("fp32", seed), ("bf16", seed), ("fp16", seed), ("fp32 other seed", seed + 1)]
    outs = ("symbols", "marginals", "llrs")
    gpu = {}
    for f, sd in forms:
        b, g = run_gpu(batch, C, T, sd, f.split()[0], trace=False, outputs=outs)
        gpu[f] = g
    n = len(b.sigma2)
    ref_m, ref_l, ref_s = [], [], []
    for i in range(n):
        o = odm.detect(b.H[i], b.y[i], b.sigma2[i], b.M, C, T, seed, instance=i, estimators=False)
        prob = o["problem"]
        ref_m.append(odm.marginals_is(prob, o["k"], antennas=ants))
        ref_l.append(odm.llr_is(prob, o["k"], antennas=ants))
        ref_s.append(o["symbols"])
    rows = ants if ants is not None else slice(None)
    ref_m = np.stack(ref_m)[:, rows]
    ref_l = np.stack(ref_l)[:, rows]
    res = {}
    for f, _ in forms:
        g = gpu[f]
        res[f] = dict(marg_mae=float(np.abs(g["marginals"][:, rows] - ref_m).mean()),
                      llr_mae=float(np.abs(g["llrs"][:, rows] - ref_l).mean()),
                      ser=float(np.mean(g["symbols"] != b.x_idx)),
                      sym_vs_oracle=float(np.mean(g["symbols"] != np.stack(ref_s))))
    res["oracle"] = dict(ser=float(np.mean(np.stack(ref_s) != b.x_idx)))
    for f, r in res.items():
        print("precision %s %-16s %s" % (name, f, " ".join("%s=%.4g" % kv for kv in r.items())), flush=True)
    # fp32 follows the oracle's chains: rounding-level error
    assert res["fp32"]["marg_mae"] < 0.2 * res["fp32 other seed"]["marg_mae"] + 1e-4
    # BF16 / FP16: no worse than independent fp32 chains (Monte Carlo error), 15 % + 0.002 allowance
    ind = res["fp32 other seed"]
    for f in ("bf16", "fp16"):
        assert res[f]["marg_mae"] <= 1.15 * ind["marg_mae"] + 2e-3, (f, res[f], ind)
        assert res[f]["llr_mae"] <= 1.15 * ind["llr_mae"] + 2e-2, (f, res[f], ind)
