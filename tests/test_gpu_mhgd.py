"""The MHGD baseline on the device (proposal DMALA_MHGD) against its oracle (needs an MI355X).

* chain identity with oracle/mhgd.py on the shared random numbers (float64: every chain; fp32:
  up to the first near-tie -- a candidate within EPS_CAND level spacings of a cell boundary, or an
  MH draw within the fp32 threshold);
* the device's own kernel (dmala_debug_eval: log q of the nearest-point candidate law, log A
  without the proposal ratio) equals the oracle's exact MHGD kernel;
* Section III-B, fig. tv_theory: on 2x2 QPSK at 8 dB, about 10^5 device chains of DMALA and of
  MHGD follow the exact uniform-start laws P^t of their kernels; DMALA's total-variation distance
  to pi falls to the sampling-noise floor, MHGD's levels off at the bias of its stationary law.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from oracle import exact, mhgd
from tests.helpers import gpu_available, compare_chains, eps32_mh

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# candidate near-tie (level spacings): fp32 error of mu + sigma Phi^-1(u) in index units
EPS_CAND32 = 1e-4


def _gpu_mhgd(b, C, T, seed, precision, tau=2.0):
    import torch
    import paper_2407_06042_amd as dm
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    det = dm.Detector(len(b.sigma2), b.nt, b.nr, b.M, C, T, seed, precision, "mhgd", tau,
                      outputs=("symbols", "final_state", "accept_count"), trace=True)
    out = det(Hcm, y, s2)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["trace_hash"] = res["trace_hash"].view(np.uint32)
    return res


@pytest.mark.parametrize("precision,nt,M,snr,C,T", [("fp64", 4, 16, 10.0, 16, 50), ("fp32", 4, 16, 10.0, 16, 50),
                                                     ("fp32", 32, 64, 22.0, 32, 60), ("fp64", 32, 64, 22.0, 16, 30),
                                                     ("fp32", 64, 64, 24.0, 32, 40)])
def test_mhgd_chains_match_the_oracle(precision, nt, M, snr, C, T):
    batch = W.make_batch(nt, nt, M, snr, 3, seed=nt + M)
    b = batch.as_precision(np.float64 if precision == "fp64" else np.float32)
    seed = 0x3D6D + nt
    g = _gpu_mhgd(b, C, T, seed, precision)
    eps = (1e-9, 1e-9) if precision == "fp64" else (EPS_CAND32, eps32_mh)
    tot_id = 0
    for i in range(3):
        prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], M)
        o = mhgd.mhgd_sample(prob, seed, i, C, T, trace=True)
        o["problem"] = prob
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *eps)
        print("mhgd", precision, nt, M, "inst", i, "identical", n_id, "flagged", n_fd, "bad", bad[:3], flush=True)
        assert not bad
        same = [c for c in range(C) if np.array_equal(g["trace_hash"][i, c], o["trace"]["hash"][:, c])]
        np.testing.assert_array_equal(g["final_state"][i][same], o["k"][same])
        np.testing.assert_array_equal(g["accept_count"][i][same], o["n_acc"][same])
        tot_id += n_id
    assert tot_id >= (3 * C if precision == "fp64" and nt <= 4 else 3 * C // 2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_device_mhgd_kernel_equals_the_exact_kernel(precision):
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(2, 2, 4, 8.0, 1, seed=9).as_precision(np.float64 if precision == "fp64" else np.float32)
    prob = odm.Problem(b.H[0], b.y[0], b.sigma2[0], 4, tau=1.0)
    K = exact.all_states(prob.N, prob.Q)
    S = len(K)
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    out = dm.debug_eval(Hcm, y, s2, 4, torch.from_numpy(np.repeat(K, S, 0)[None]).cuda(),
                        torch.from_numpy(np.tile(K, (S, 1))[None]).cuda(), precision=precision, proposal="mhgd",
                        tau=1.0).cpu().numpy().reshape(S, S, 4)
    P = np.exp(out[..., 0] + np.minimum(0.0, out[..., 3]))
    np.fill_diagonal(P, 0.0)
    P[np.arange(S), np.arange(S)] = 1.0 - P.sum(1)
    Po, LQo = mhgd.transition_matrix(prob, K)
    tol = 1e-9 if precision == "fp64" else 2e-5
    assert np.abs(P - Po).max() < tol
    np.testing.assert_allclose(out[..., 0], LQo, atol=1e-8 if precision == "fp64" else 5e-4)


def test_tv_distance_mhgd_levels_off_dmala_converges():
    """2x2 QPSK, 8 dB, tau = 1, 98 x 1024 chains from the uniform start; the law after t transitions is
    read from the final states of runs with n_iters = t (the same seed continues the same chains)."""
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(2, 2, 4, 8.0, 1, seed=9).as_precision(np.float32)
    prob = odm.Problem(b.H[0], b.y[0], b.sigma2[0], 4, tau=1.0)
    K = exact.all_states(prob.N, prob.Q)
    S = len(K)
    pi = np.exp(exact.log_target(prob, K))
    kern = {"mhgd": mhgd.transition_matrix(prob, K)[0], "precond": exact.transition_matrix(prob, K)[0]}
    code = prob.Q ** np.arange(prob.N - 1, -1, -1)
    reps, C = 98, 1024
    times = [1, 2, 3, 5, 8, 12, 20, 30, 45, 60]
    Hcm, y, s2 = dm.device_inputs(np.repeat(b.H, reps, 0), np.repeat(b.y, reps, 0), np.repeat(b.sigma2, reps, 0))
    n = reps * C
    floor = 0.5 * np.sum(np.sqrt(pi * (1 - pi) / n))          # about the TV of n exact samples
    res = {}
    for prop in ("precond", "mhgd"):
        tv_pi, tv_law = [], []
        for t in times:
            det = dm.Detector(reps, 2, 2, 4, C, t, 0x7F + len(prop), "fp32", prop, 1.0, outputs=("final_state",))
            k = det(Hcm, y, s2)["final_state"].cpu().numpy().reshape(n, prob.N).astype(np.int64)
            torch.cuda.synchronize()
            emp = np.bincount(k @ code, minlength=S) / n
            pt = np.full(S, 1.0 / S) @ np.linalg.matrix_power(kern[prop], t)
            tv_law.append(exact.tv(emp, pt))
            tv_pi.append(exact.tv(emp, pi))
        res[prop] = (np.array(tv_pi), np.array(tv_law), exact.tv(mhgd.stationary(kern[prop]), pi))
        print("tv %s: TV(law, pi) at t=%s: %s; max TV(law, exact P^t) %.4f; stationary bias %.4f; noise floor %.4f"
              % (prop, times, np.round(res[prop][0], 4), res[prop][1].max(), res[prop][2], floor), flush=True)
        # the device chain follows its exact kernel at every t (multinomial noise)
        assert res[prop][1].max() < 4 * floor + 2e-3
    assert res["precond"][0][-1] < 4 * floor + 2e-3               # DMALA: at the noise floor
    assert res["mhgd"][2] > 0.1                                   # MHGD's stationary law is biased ...
    assert res["mhgd"][0][-1] > 0.5 * res["mhgd"][2]              # ... and its chains level off away from pi
