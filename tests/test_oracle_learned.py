"""Pins of the learned-proposal oracle (CPU only).

Each check ties the oracle to something other than itself: a library routine
(torch's bfloat16 conversion and Adam), finite differences, closed forms for
diagonal channels, the plain kernel it must reduce to, and the exact
transition matrix on enumerable problems (detailed balance, the chain's law).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from oracle import exact as ex
from oracle import learned as ol


def _prob(nt, nr, M, snr, seed, inst=0):
    b = W.make_batch(nt, nr, M, snr, inst + 1, seed)
    return odm.Problem(b.H[inst], b.y[inst], b.sigma2[inst], M)


def _rand_params(seed, scale=1.0):
    P = ol.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    P["W3"] = rng.standard_normal(P["W3"].shape) * 0.3 * scale
    P["b3"] = rng.standard_normal(4) * 0.2 * scale
    P["b1"] = rng.standard_normal(ol.HID) * 0.1
    P["b2"] = rng.standard_normal(ol.HID) * 0.1
    return {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-20, 20, 20000))).astype(np.float32)
    # exact ties between two bfloat16 neighbours, both parities
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(2.0 + 2.0 ** -7), 0.0], dtype=np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ol.bf16(x.astype(np.float64)), ref)
    assert ol.bf16(1.0 + 2.0 ** -8) == 1.0 and ol.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_plain_index_params_reproduce_the_preconditioned_proposal():
    prob = _prob(3, 4, 16, 12.0, 3)
    k = np.random.default_rng(1).integers(0, prob.Q, (5, prob.N))
    a = odm.log_softmax(prob.proposal_logits(prob.x_of(k)))
    b = odm.log_softmax(ol.plain_logits(prob, k))
    np.testing.assert_allclose(a, b, atol=1e-12)
    # the default parameters fix kappa = 2 (natural log units)
    assert abs(ol.plain_index_params(prob, k)[1] - 2.0) < 1e-12


def test_antenna_constants_closed_form_for_a_diagonal_channel():
    h = np.array([0.8 + 0.3j, -0.2 + 1.1j, 0.5 - 0.5j])
    sigma2, M = 0.05, 64
    prob = odm.Problem(np.diag(h), np.zeros(3, complex), sigma2, M)
    s = np.sqrt(3.0 / (2.0 * (M - 1)))
    gam = sigma2 / (2 * s * s)
    g = np.abs(h) ** 2
    c = ol.antenna_constants(prob)
    np.testing.assert_allclose(c[:, 0], np.log2(sigma2 / (g + gam) / (8 * s * s)) / 8, rtol=1e-12)
    np.testing.assert_allclose(c[:, 1], np.log2(sigma2 / (8 * s * s * g)) / 8, rtol=1e-12)
    np.testing.assert_allclose(c[:, 2], 0.75)


def test_features_layout():
    prob = _prob(2, 2, 16, 15.0, 4)
    k = np.array([[0, 3, 1, 2]])
    mu, _ = ol.plain_index_params(prob, k)
    f = ol.features(prob, k)
    assert f.shape == (1, 2, 7)
    np.testing.assert_allclose(f[0, :, 2], (k[0, 0::2] - 1.5) / 2)
    np.testing.assert_allclose(f[0, :, 3], (k[0, 1::2] - 1.5) / 2)
    np.testing.assert_allclose(f[0, :, 0], (mu[0, 0::2] - 1.5) / 2)
    np.testing.assert_allclose(f[0, :, 1], (mu[0, 1::2] - 1.5) / 2)


def test_zero_output_layer_gives_the_plain_chain():
    prob = _prob(4, 4, 16, 14.0, 5)
    P = ol.init_params(7, zero_last=True)
    k = np.random.default_rng(2).integers(0, 4, (3, prob.N))
    np.testing.assert_allclose(odm.log_softmax(ol.learned_logits(prob, k, P)),
                               odm.log_softmax(ol.plain_logits(prob, k)), atol=1e-12)
    for eps in (0.0, 0.3, 1.0):
        a = ol.mixture_sample(prob, P, eps, 11, 2, 8, 15)
        b = odm.dmala_sample(prob, 11, 2, 8, 15)
        np.testing.assert_array_equal(a["k"], b["k"])
        np.testing.assert_array_equal(a["n_acc"], b["n_acc"])
        np.testing.assert_array_equal(a["best_k"], b["best_k"])


def test_mixture_choice_frequency():
    prob = _prob(2, 2, 4, 10.0, 6)
    P = _rand_params(3)
    r = ol.mixture_sample(prob, P, 0.25, 5, 0, 400, 20)
    frac = r["n_learned"].sum() / (400 * 20)
    assert abs(frac - 0.75) < 4 * np.sqrt(0.75 * 0.25 / 8000)


@pytest.mark.parametrize("nt,M", [(2, 4), (1, 16), (2, 16)])
def test_learned_and_mixture_kernels_satisfy_detailed_balance(nt, M):
    prob = _prob(nt, nt + 1, M, 8.0, 10 + M)
    P = _rand_params(M, scale=3.0)
    K = ex.all_states(prob.N, prob.Q)
    lpi = ex.log_target(prob, K, tempered=True)
    Pm, Pp, Pl, LQl = ol.mixture_transition_matrix(prob, P, 0.3, K)
    pi = np.exp(lpi)
    for T in (Pm, Pp, Pl):
        F = pi[:, None] * T
        np.testing.assert_allclose(F, F.T, atol=1e-13)
        np.testing.assert_allclose(pi @ T, pi, atol=1e-12)
    # the learned kernel really differs from the plain one
    assert np.abs(Pl - Pp).max() > 1e-3
    # planted mistake: reverse proposal taken equal to the forward one -> no detailed balance
    ft = prob.f(prob.x_of(K)) / prob.tau
    bad = np.exp(LQl + np.minimum(0.0, ft[None, :] - ft[:, None]))
    np.fill_diagonal(bad, 0.0)
    bad[np.diag_indices_from(bad)] = 1.0 - bad.sum(axis=1)
    Fb = pi[:, None] * bad
    off = ~np.eye(len(K), dtype=bool)
    rel = np.abs(Fb - Fb.T)[off] / np.maximum(Fb + Fb.T, 1e-300)[off]
    assert rel.max() > 1e-3


def test_mixture_chain_law_matches_the_exact_kernel():
    prob = _prob(1, 2, 16, 6.0, 21)
    P = _rand_params(5, scale=2.0)
    K = ex.all_states(prob.N, prob.Q)
    Pm, _, _, _ = ol.mixture_transition_matrix(prob, P, 0.4, K)
    C, T = 6000, 4
    r = ol.mixture_sample(prob, P, 0.4, 99, 3, C, T)
    idx = r["k"][:, 0] * prob.Q + r["k"][:, 1]
    emp = np.bincount(idx, minlength=len(K)) / C
    p0 = np.full(len(K), 1.0 / len(K))
    pt = p0 @ np.linalg.matrix_power(Pm, T)
    # chains are independent: chi-square with 15 degrees of freedom
    chi2 = C * np.sum((emp - pt) ** 2 / np.maximum(pt, 1e-12))
    assert chi2 < 40.0, chi2


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = _rand_params(9)
    X = rng.standard_normal((6, ol.N_FEAT))
    d_out = rng.standard_normal((6, ol.N_OUT))
    _, cache = ol.mlp_forward(P, X, rounded=False)
    g = ol.mlp_backward(P, cache, d_out)
    h = 1e-6
    for name, shp in ol.PARAM_SHAPES:
        for _ in range(4):
            i = tuple(rng.integers(0, s) for s in shp)
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][i] += h
            Pm[name][i] -= h
            fd = (np.sum(d_out * ol.mlp_forward(Pp, X, False)[0]) - np.sum(d_out * ol.mlp_forward(Pm, X, False)[0])) / (2 * h)
            assert abs(fd - g[name][i]) < 1e-6 * max(1.0, abs(fd)), (name, i, fd, g[name][i])


def test_cross_entropy_derivatives_match_finite_differences():
    rng = np.random.default_rng(4)
    R, Q = 50, 8
    mu = rng.uniform(-2, Q + 1, R)
    kap = rng.uniform(0.1, 5.0, R)
    t = rng.integers(0, Q, R)
    _, dm, dk = ol.proposal_xent(mu, kap, Q, t)
    h = 1e-6
    fdm = (ol.proposal_xent(mu + h, kap, Q, t)[0] - ol.proposal_xent(mu - h, kap, Q, t)[0]) / (2 * h)
    fdk = (ol.proposal_xent(mu, kap + h, Q, t)[0] - ol.proposal_xent(mu, kap - h, Q, t)[0]) / (2 * h)
    np.testing.assert_allclose(dm, fdm, atol=1e-6)
    np.testing.assert_allclose(dk, fdk, atol=1e-6)
    # Q = 2 with kappa -> 0 is a fair coin
    l, _, _ = ol.proposal_xent(np.array([0.3]), np.array([1e-12]), 2, np.array([1]))
    assert abs(l[0] - np.log(2.0)) < 1e-9


def test_training_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    P = _rand_params(12, scale=4.0)
    R = 40
    X = rng.standard_normal((R, ol.N_FEAT))
    mu = rng.uniform(0, 7, (R, 2))
    kap = np.full(R, 2.0)
    Q = np.where(np.arange(R) % 2 == 0, 8, 4)
    tgt = np.stack([rng.integers(0, Q), rng.integers(0, Q)], axis=-1)
    L, G = ol.training_loss(P, X, mu, kap, Q, tgt, grad=True)
    h = 1e-6
    for name, shp in ol.PARAM_SHAPES:
        for _ in range(4):
            i = tuple(rng.integers(0, s) for s in shp)
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][i] += h
            Pm[name][i] -= h
            fd = (ol.training_loss(Pp, X, mu, kap, Q, tgt) - ol.training_loss(Pm, X, mu, kap, Q, tgt)) / (2 * h)
            assert abs(fd - G[name][i]) < 1e-6 * max(1.0, abs(fd)), (name, i, fd, G[name][i])


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(6)
    P = _rand_params(13)
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    tp = [torch.tensor(P[n].copy(), dtype=torch.float64, requires_grad=True) for n, _ in ol.PARAM_SHAPES]
    opt = torch.optim.Adam(tp, lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        G = {n: rng.standard_normal(s) for n, s in ol.PARAM_SHAPES}
        ol.adam_step(P, G, m, v, step, 3e-3)
        for t, (n, _) in zip(tp, ol.PARAM_SHAPES):
            t.grad = torch.from_numpy(G[n].copy())
        opt.step()
    for t, (n, _) in zip(tp, ol.PARAM_SHAPES):
        np.testing.assert_allclose(P[n], t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_training_lowers_the_loss():
    rng = np.random.default_rng(7)
    probs = [_prob(4, 4, 16, 18.0, 30, i) for i in range(6)]
    Xs, mus, tg = [], [], []
    for i, prob in enumerate(probs):
        b = W.make_batch(4, 4, 16, 18.0, i + 1, 30)
        k = rng.integers(0, 4, (8, prob.N))
        mu, _ = ol.plain_index_params(prob, k)
        Xs.append(ol.features(prob, k).reshape(-1, 7))
        mus.append(np.stack([mu[:, 0::2], mu[:, 1::2]], axis=-1).reshape(-1, 2))
        xi = b.x_idx[i]
        tg.append(np.tile(np.stack([xi // 4, xi % 4], axis=-1), (8, 1)))
    X, mu, tg = np.concatenate(Xs), np.concatenate(mus), np.concatenate(tg)
    kap = np.full(len(X), 2.0)
    P = ol.init_params(1, zero_last=True)
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    L0 = ol.training_loss(P, X, mu, kap, 4, tg)
    for step in range(1, 61):
        _, G = ol.training_loss(P, X, mu, kap, 4, tg, grad=True)
        ol.adam_step(P, G, m, v, step, 1e-2)
    assert ol.training_loss(P, X, mu, kap, 4, tg) < 0.8 * L0
