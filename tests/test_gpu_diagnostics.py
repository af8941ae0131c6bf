"""Convergence diagnostics from the device chain's exact transition matrices (needs an MI355X).

2x2 QPSK, 100 realisations (unit-variance channel, as in the convergence
experiment of Section III-B) at 4, 6, 8 and 10 dB: the second-largest
eigenvalue modulus of the device kernel equals the oracle's; for the naive
proposal it rises towards 1 with the SNR while the preconditioned proposal
keeps it flat (the comparison of Section III-B); the TV distance from the
uniform start obeys the spectral bound of a reversible chain.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from oracle import exact
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_second_eigenvalue_trend_naive_vs_preconditioned():
    from paper_2407_06042_amd import diagnostics as dg
    med = {}
    for snr in (4, 6, 8, 10):
        b = W.make_batch(2, 2, 4, snr, 100, seed=77, var_h=1.0)
        for prop in ("naive", "precond"):
            P, K, lpi = dg.device_kernels(b.H, b.y, b.sigma2, 4, precision="fp64", proposal=prop)
            lam = dg.second_eigenvalue(P)
            ref = []
            for i in range(0, 100, 10):
                prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], 4, variant=prop)
                Po, _, _ = exact.transition_matrix(prob, K)
                ref.append(exact.second_eigenvalue(Po))
                np.testing.assert_allclose(P[i], Po, atol=1e-10)
                np.testing.assert_allclose(lpi[i], exact.log_target(prob, K), atol=1e-9)
            np.testing.assert_allclose(lam[::10], ref, atol=1e-8)
            med[(snr, prop)] = float(np.median(lam))
            # spectral bound of a reversible chain: TV(t) <= 1/2 sqrt((1 - pi_min) / pi_min) lambda_2^t
            for i in range(0, 100, 25):
                tv = dg.tv_curve(P[i], lpi[i], 40)
                pmin = np.exp(lpi[i]).min()
                bound = 0.5 * np.sqrt((1 - pmin) / pmin) * lam[i] ** np.arange(41)
                assert np.all(tv <= bound * (1 + 1e-9) + 1e-12)
    print("median lambda_2:", {k: round(v, 3) for k, v in med.items()}, flush=True)
    naive = [med[(s, "naive")] for s in (4, 6, 8, 10)]
    pre = [med[(s, "precond")] for s in (4, 6, 8, 10)]
    assert all(a < b for a, b in zip(naive, naive[1:]))          # rises with the SNR
    assert naive[-1] > 0.93 and naive[-1] > pre[-1] + 0.1
    assert max(pre) - min(pre) < 0.05                           # flat for the preconditioned proposal


def test_learned_kernel_rate_is_a_kernel_property():
    """The mixture's components: the learned kernel's rate from the device matrices equals the oracle's."""
    import torch
    from paper_2407_06042_amd import diagnostics as dg
    from oracle import learned as ol
    P0 = ol.init_params(5)
    rng = np.random.default_rng(6)
    P0["W3"] = rng.standard_normal(P0["W3"].shape) * 0.5
    P0 = {k: v.astype(np.float32).astype(np.float64) for k, v in P0.items()}
    w = torch.from_numpy(ol.flatten(P0).astype(np.float32)).cuda()
    b = W.make_batch(2, 2, 4, 8.0, 8, seed=78, var_h=1.0).as_precision(np.float32)
    P, K, lpi = dg.device_kernels(b.H, b.y, b.sigma2, 4, precision="fp32", proposal="learned", mlp_weights=w)
    lam = dg.second_eigenvalue(P)
    for i in range(8):
        prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], 4)
        _, _, Pl, _ = ol.mixture_transition_matrix(prob, P0, 0.0, K)
        assert abs(lam[i] - exact.second_eigenvalue(Pl)) < 1e-3
