"""Pins of the MHGD baseline oracle (oracle/mhgd.py) against brute force and the exact kernel.

* the nearest-level mapping is the argmin over the levels; the cell probabilities of
  N(c, alpha beta) under the mapping match a large Monte Carlo sample of numpy normals;
* the candidate centre is the maximum of DMALA's preconditioned proposal (Remark after
  Algorithm 1): both methods start from the same Gaussian, discretised two ways;
* the sampler's chain law after t transitions equals uniform-start P^t, P its exact kernel;
* Section III-B, fig. tv_theory: without the mapping's probability in the MH test the
  kernel is not reversible and its stationary law differs from pi (the TV distance
  levels off above zero), while DMALA's stationary law is pi; restoring the proposal
  ratio makes the MHGD kernel reversible again.
"""
import numpy as np

import workloads as W
from oracle import dmala as odm
from oracle import exact, mhgd


def _prob(seed, M=4, snr=8.0, tau=1.0, nt=2):
    b = W.make_batch(nt, 2, M, snr, 1, seed=seed)
    return odm.Problem(b.H[0], b.y[0], b.sigma2[0], M, tau=tau)


def test_nearest_level_is_the_argmin():
    prob = _prob(1, M=16)
    rng = np.random.default_rng(0)
    xt = rng.normal(0.0, 1.5, size=(5000,))
    k, margin = mhgd.nearest_level(prob, xt)
    np.testing.assert_array_equal(k, np.argmin(np.abs(xt[:, None] - prob.levels[None, :]), axis=1))
    # margin: distance to the nearest of the Q-1 boundaries, in level spacings
    d = np.abs(xt[:, None] - 0.5 * (prob.levels[1:] + prob.levels[:-1])[None, :]).min(1) / (2 * prob.s)
    np.testing.assert_allclose(margin, d)


def test_cell_probabilities_match_monte_carlo():
    prob = _prob(2, M=16)
    rng = np.random.default_rng(1)
    c = np.array([-1.3, -0.2, 0.05, 0.9])                     # centres inside and outside the alphabet
    cp = mhgd.cell_probs(prob, c)
    np.testing.assert_allclose(cp.sum(-1), 1.0, atol=1e-12)
    n = 2_000_000
    sd = mhgd.noise_std(prob)
    for i, ci in enumerate(c):
        k, _ = mhgd.nearest_level(prob, ci + sd * rng.standard_normal(n))
        emp = np.bincount(k, minlength=prob.Q) / n
        se = np.sqrt(cp[i] * (1 - cp[i]) / n)
        assert np.all(np.abs(emp - cp[i]) <= 5 * se + 1e-7), (ci, emp, cp[i])


def test_candidate_centre_is_the_dmala_proposal_maximum():
    prob = _prob(3, M=64, snr=20.0, tau=2.0)
    rng = np.random.default_rng(2)
    k = rng.integers(0, prob.Q, size=(7, prob.N))
    x = prob.x_of(k)
    lg = prob.proposal_logits(x)                                # quadratic in the level value
    L = prob.levels
    # fit the parabola through three levels: its vertex is the continuous maximiser
    a = (lg[..., 2] - 2 * lg[..., 1] + lg[..., 0]) / (2 * (L[1] - L[0]) ** 2)
    b = (lg[..., 2] - lg[..., 0]) / (2 * (L[1] - L[0])) - 2 * a * L[1]
    np.testing.assert_allclose(-b / (2 * a), mhgd.candidate_centre(prob, x), rtol=1e-9, atol=1e-9)
    # and its curvature is that of N(., alpha beta)
    np.testing.assert_allclose(-1.0 / (2 * a), prob.alpha * prob.beta, rtol=1e-9)


def test_chain_law_matches_the_exact_kernel():
    prob = _prob(9)
    K = exact.all_states(prob.N, prob.Q)
    P, _ = mhgd.transition_matrix(prob, K)
    S = len(K)
    code = prob.Q ** np.arange(prob.N - 1, -1, -1)
    C = 20000
    p0 = np.full(S, 1.0 / S)
    for T in (1, 3, 10):
        r = mhgd.mhgd_sample(prob, 77 + T, 0, C, T)
        emp = np.bincount(r["k"] @ code, minlength=S) / C
        pt = p0 @ np.linalg.matrix_power(P, T)
        se = np.sqrt(pt * (1 - pt) / C)
        assert np.all(np.abs(emp - pt) <= 5 * se + 1e-4), (T, np.abs(emp - pt).max())


def test_missing_proposal_ratio_biases_the_stationary_law():
    tv_mhgd, tv_dmala = [], []
    for seed in range(20):
        prob = _prob(seed)
        K = exact.all_states(prob.N, prob.Q)
        pi = np.exp(exact.log_target(prob, K))
        P, _ = mhgd.transition_matrix(prob, K)
        Pd, _, _ = exact.transition_matrix(prob, K)
        Pr, _ = mhgd.transition_matrix(prob, K, with_reverse=True)
        np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-12)
        # with the proposal ratio restored: exact MH, reversible w.r.t. pi, pi stationary
        F = pi[:, None] * Pr
        assert np.abs(F - F.T).max() < 1e-12
        assert exact.tv(mhgd.stationary(Pr), pi) < 1e-10
        tv_mhgd.append(exact.tv(mhgd.stationary(P), pi))
        tv_dmala.append(exact.tv(mhgd.stationary(Pd), pi))
        if tv_mhgd[-1] > 0.05:
            # not reversible w.r.t. pi, and the TV distance of the chain's law levels off at that bias
            assert np.abs(pi[:, None] * P - (pi[:, None] * P).T).max() > 1e-4
            pt = np.full(len(K), 1.0 / len(K)) @ np.linalg.matrix_power(P, 1 << 16)
            assert abs(exact.tv(pt, pi) - tv_mhgd[-1]) < 1e-6
    assert max(tv_dmala) < 1e-10
    assert np.median(tv_mhgd) > 0.01 and max(tv_mhgd) > 0.1
