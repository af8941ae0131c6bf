"""Pins of the float64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: published
known answers, closed forms, invariants proved in the paper (Lemma 1,
detailed balance in Appendix A), exhaustive enumeration, or an independent
formulation (the continuous Langevin Gaussian of eq. proposal_cont restricted
to the lattice; numerical differentiation of f; scipy's Gaussian density).
"""
import os

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import philox, dmala, exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _prob(nt, nr, M, snr, seed, variant=dmala.PRECOND, tau=2.0, **kw):
    b = W.make_batch(nt, nr, M, snr, 1, seed)
    return dmala.Problem(b.H[0], b.y[0], b.sigma2[0], M, variant, tau, **kw)


# ----------------------------------------------------------------- Philox

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for r in rows:
        v = [int(x, 16) for x in r[1:]]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:], r


def test_philox_uniformity_and_counter_independence():
    w = philox.words(12345, 7, np.arange(4096), 3, 64)      # 4096 x 64 words
    u = philox.uniform24(w).reshape(-1)
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = stats.chisquare(hist)
    assert chi2.pvalue > 1e-4
    # streams of neighbouring counters are uncorrelated
    w2 = philox.words(12345, 7, np.arange(4096), 4, 64)
    c = np.corrcoef(u, philox.uniform24(w2).reshape(-1))[0, 1]
    assert abs(c) < 0.01
    # the draw uniform: midpoints of the 23-bit cells, in (0, 1) and exact in fp32
    ud = philox.uniform_draw(np.array([0, 0x1FF, 0x200, 0xFFFFFFFF], np.uint32))
    np.testing.assert_array_equal(ud, [2.0 ** -24, 2.0 ** -24, 3 * 2.0 ** -24, 1 - 2.0 ** -24])
    ua = philox.uniform_draw(w).reshape(-1)
    assert np.all(ua.astype(np.float32) == ua)
    assert stats.kstest(ua, "uniform").pvalue > 1e-4
    # low-byte MH uniforms are uniform too
    um = philox.low_byte_uniform(w, 0)
    assert stats.kstest(um, "uniform").pvalue > 1e-4


def test_init_levels_uniform():
    w = philox.words(99, 0, np.arange(20000), 0, 8)
    for Q in (2, 4, 8, 16):
        k = philox.init_level_index(w[:, :8], Q).reshape(-1)
        assert k.min() == 0 and k.max() == Q - 1
        assert stats.chisquare(np.bincount(k, minlength=Q)).pvalue > 1e-4


# ----------------------------------------------------------------- constellation

@pytest.mark.parametrize("M", [4, 16, 64, 256])
def test_constellation_unit_energy_and_dmin(M):
    Q = int(np.sqrt(M))
    lv, s = dmala.pam_levels(Q)
    pts = (lv[:, None] + 1j * lv[None, :]).reshape(-1)
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) < 1e-12          # unit average power
    d = np.abs(pts[:, None] - pts[None, :])
    dmin = d[d > 0].min()
    assert abs(dmin / 2 - s) < 1e-12                            # dmin = half min distance
    # independent generator of the inputs agrees on the points
    np.testing.assert_allclose(W.qam_points(M), pts, atol=1e-15)


@pytest.mark.parametrize("Q", [2, 4, 8, 16])
def test_gray_labels(Q):
    nb = int(np.log2(Q))
    k = np.arange(Q)
    bits = dmala.gray_bits(k, nb)
    codes = bits @ (1 << np.arange(nb)[::-1])
    assert len(set(codes.tolist())) == Q                          # bijective
    assert np.all(np.sum(bits[1:] != bits[:-1], axis=1) == 1)     # neighbours differ in one bit
    assert np.array_equal(dmala.level_from_gray_bits(bits), k)


# ----------------------------------------------------------------- model

def test_real_equivalent_model():
    p = _prob(3, 5, 16, 10.0, 1)
    rng = np.random.default_rng(0)
    xc = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    x = np.zeros(6)
    x[0::2], x[1::2] = xc.real, xc.imag
    yc = p.H_c @ xc                                              # complex product
    y = p.H @ x
    np.testing.assert_allclose(y[0::2], yc.real, atol=1e-13)
    np.testing.assert_allclose(y[1::2], yc.imag, atol=1e-13)


def test_f_is_gaussian_log_likelihood():
    """eq. f equals log p(y|x) with N(0, sigma^2/2) noise per real element, up to a constant."""
    p = _prob(2, 3, 16, 8.0, 2)
    K = exact.all_states(p.N, p.Q)[::37]
    X = p.x_of(K)
    ll = np.sum(stats.norm.logpdf(p.y[None, :], loc=X @ p.H.T, scale=np.sqrt(p.sigma2 / 2)), axis=1)
    diff = ll - p.f(X)
    assert np.ptp(diff) < 1e-9


@pytest.mark.parametrize("variant", [dmala.NAIVE, dmala.PRECOND])
def test_gradient_matches_finite_differences(variant):
    p = _prob(3, 4, 16, 12.0, 3, variant)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(p.N) * 0.5
    g = p.grad_f(x)
    h = 1e-5
    fd = np.array([(p.f(x + h * e) - p.f(x - h * e)) / (2 * h) for e in np.eye(p.N)])
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6 * np.abs(g).max())


def test_preconditioner_inverts_damped_hessian():
    p = _prob(4, 4, 64, 20.0, 4)
    np.testing.assert_allclose(p.Mpre @ (p.H.T @ p.H + p.gamma * np.eye(p.N)), np.eye(p.N), atol=1e-10)
    assert abs(p.gamma - p.sigma2 / (2 * p.s ** 2)) < 1e-15
    assert abs(p.alpha * p.beta - p.s ** 2) < 1e-15


@pytest.mark.parametrize("variant,tau", [(dmala.NAIVE, 1.0), (dmala.NAIVE, 2.0), (dmala.PRECOND, 2.0), (dmala.PRECOND, 1.0)])
def test_factorised_proposal_equals_restricted_langevin_gaussian(variant, tau):
    """Pi_n q_n (eq. dis_prop_fac1) == N(x + a/2 [M] grad, a[b] I) restricted to A^N and renormalised."""
    p = _prob(2, 2, 16, 6.0, 5, variant, tau)
    K = exact.all_states(p.N, p.Q)
    X = p.x_of(K)
    rng = np.random.default_rng(2)
    for _ in range(3):
        k0 = rng.integers(0, p.Q, p.N)
        x0 = p.x_of(k0)
        # gradient of f/tau by central differences (independent of grad_f)
        h = 1e-6
        g = np.array([(p.f(x0 + h * e) - p.f(x0 - h * e)) / (2 * h) for e in np.eye(p.N)]) / tau
        if variant == dmala.NAIVE:
            mean, cov = x0 + p.alpha / 2 * g, p.alpha
        else:
            mean, cov = x0 + p.alpha / 2 * (p.Mpre @ g), p.alpha * p.beta
        lg = stats.multivariate_normal(mean=mean, cov=cov * np.eye(p.N)).logpdf(X)
        joint = lg - np.log(np.sum(np.exp(lg - lg.max()))) - lg.max()
        logq = dmala.log_softmax(p.proposal_logits(x0[None]))[0]
        fact = np.zeros(len(K))
        for n in range(p.N):
            fact += logq[n, K[:, n]]
        np.testing.assert_allclose(fact, joint, atol=1e-5)


def test_inverse_cdf_semantics():
    rng = np.random.default_rng(3)
    logits = rng.standard_normal((500, 7)) * 2
    u = rng.random(500)
    idx, margin = dmala.inverse_cdf(logits, u)
    p = np.exp(dmala.log_softmax(logits))
    ref = np.array([np.searchsorted(np.cumsum(pi), ui, side="right") for pi, ui in zip(p, u)])
    np.testing.assert_array_equal(idx, np.minimum(ref, 6))
    assert np.all(margin >= 0)
    # frequencies follow the probabilities
    lg = np.array([0.3, -1.0, 2.0, 0.0])
    uu = philox.uniform_draw(philox.words(1, 0, np.arange(40000), 1, 4)[:, 0])
    ii, _ = dmala.inverse_cdf(np.broadcast_to(lg, (40000, 4)), uu)
    exp_p = np.exp(dmala.log_softmax(lg))
    assert stats.chisquare(np.bincount(ii, minlength=4), 40000 * exp_p).pvalue > 1e-4


# ----------------------------------------------------------------- MH kernel

CASES = [(1, 1, 4), (2, 2, 4), (1, 2, 16), (2, 2, 16), (1, 1, 64)]


@pytest.mark.parametrize("variant", [dmala.NAIVE, dmala.PRECOND])
@pytest.mark.parametrize("nt,nr,M", CASES)
def test_transition_matrix_properties(variant, nt, nr, M):
    """Lemma 1 and Appendix A: stochastic, detailed balance, stationary pi_a, irreducible, aperiodic."""
    p = _prob(nt, nr, M, 8.0, 10 + nt + M, variant)
    K = exact.all_states(p.N, p.Q)
    P, LQ, LA = exact.transition_matrix(p, K)
    pi = np.exp(exact.log_target(p, K, tempered=True))
    assert np.abs(P.sum(1) - 1).max() < 1e-12
    F = pi[:, None] * P
    assert np.abs(F - F.T).max() < 1e-12 * max(1.0, F.max())
    assert np.abs(pi @ P - pi).max() < 1e-12
    off = P[~np.eye(len(K), dtype=bool)]
    assert off.min() > 0                                          # irreducible in one step
    assert np.diag(P).min() > 0                                   # aperiodic
    assert exact.second_eigenvalue(P) < 1.0


def test_wrong_acceptance_breaks_detailed_balance():
    """A kernel without the reverse-proposal term (a plausible slip) is caught by the balance check."""
    p = _prob(2, 2, 4, 8.0, 11)
    K = exact.all_states(p.N, p.Q)
    _, LQ, _ = exact.transition_matrix(p, K)
    ft = p.f(p.x_of(K)) / p.tau
    bad = np.exp(LQ + np.minimum(0.0, ft[None, :] - ft[:, None]))
    np.fill_diagonal(bad, 0)
    pi = np.exp(exact.log_target(p, K))
    F = pi[:, None] * bad
    assert np.abs(F - F.T).max() > 1e-6


def test_zero_channel_uniform_posterior():
    """H = 0: pi is uniform, every marginal is 1/M and the chain keeps the uniform law."""
    b = W.make_batch(2, 2, 16, 10.0, 1, 3)
    p = dmala.Problem(np.zeros_like(b.H[0]), b.y[0], b.sigma2[0], 16)
    K = exact.all_states(p.N, p.Q)
    m = exact.exact_marginals(p, K)
    np.testing.assert_allclose(m, 1.0 / 16, atol=1e-12)
    P, _, _ = exact.transition_matrix(p, K)
    u = np.full(len(K), 1.0 / len(K))
    np.testing.assert_allclose(u @ P, u, atol=1e-12)


@pytest.mark.parametrize("variant", [dmala.NAIVE, dmala.PRECOND])
def test_sampler_law_matches_exact_kernel_powers(variant):
    """Theorem 1 / Fig. 2 setting: 2x2 QPSK at 8 dB; empirical law of many chains vs uniform-init P^t."""
    p = _prob(2, 2, 4, 8.0, 21, variant)
    K = exact.all_states(p.N, p.Q)
    P, _, _ = exact.transition_matrix(p, K)
    S = 20000
    code = lambda k: (k * (p.Q ** np.arange(p.N)[::-1])).sum(-1)
    r = dmala.dmala_sample(p, 77, 0, S, 12)
    r2 = dmala.dmala_sample(p, 77, 0, S, 3)
    p0 = np.full(len(K), 1.0 / len(K))
    pi = np.exp(exact.log_target(p, K))
    lam = exact.second_eigenvalue(P)
    for T, res in ((3, r2), (12, r)):
        pt = p0 @ np.linalg.matrix_power(P, T)
        emp = np.bincount(code(res["k"]), minlength=len(K)) / S
        noise = 0.5 * np.sum(np.sqrt(pt * (1 - pt) / S))
        assert exact.tv(emp, pt) < 4 * noise + 1e-3, (T, exact.tv(emp, pt), noise)
    # exponential convergence of the exact kernel
    tvs = [exact.tv(p0 @ np.linalg.matrix_power(P, t), pi) for t in range(1, 40)]
    assert tvs[-1] < 1e-3 or tvs[-1] < tvs[0] * lam ** 30


# ----------------------------------------------------------------- estimators

@pytest.mark.parametrize("tau", [1.0, 2.0, 3.0])
@pytest.mark.parametrize("nt,M", [(2, 4), (2, 16), (1, 64)])
def test_is_llr_is_exact_under_exact_expectation(tau, nt, M):
    """Appendix C: replacing the sample mean by the exact expectation under pi_a gives eq. exact_llr."""
    p = _prob(nt, 2, M, 9.0, 30 + nt, tau=tau)
    K = exact.all_states(p.N, p.Q)
    lw = exact.log_target(p, K, tempered=True)
    np.testing.assert_allclose(dmala.llr_is(p, K, lw), exact.exact_llr(p, K), atol=1e-9)


@pytest.mark.parametrize("tau", [1.0, 2.0])
def test_is_marginals_exact_under_exact_expectation(tau):
    p = _prob(2, 2, 16, 9.0, 40, tau=tau)
    K = exact.all_states(p.N, p.Q)
    lw = exact.log_target(p, K, tempered=True)
    np.testing.assert_allclose(dmala.marginals_is(p, K, lw), exact.exact_marginals(p, K), atol=1e-12)
    # plain MC with the exact posterior weights is exact too (eq. mc)
    lw1 = exact.log_target(p, K, tempered=False)
    np.testing.assert_allclose(dmala.marginals_mc(p.Q, p.Nt, K, lw1), exact.exact_marginals(p, K), atol=1e-12)


def test_llr_sign_flips_with_label():
    """A wrong +/- assignment would flip every sign: check against the hard MAP symbol's bits."""
    p = _prob(2, 2, 16, 25.0, 41)
    L = exact.exact_llr(p)
    sym, _ = exact.map_detect(p)
    kI, kQ = sym // p.Q, sym % p.Q
    bits = np.concatenate([dmala.gray_bits(kI, 2), dmala.gray_bits(kQ, 2)], axis=1)
    # at high SNR the MAP bits agree with the LLR signs: b=+1 <-> bit 0 <-> L > 0
    assert np.all((L > 0) == (bits == 0))


def test_c1_estimates_converge_to_exact_posterior():
    """Small 4x4 16-QAM case: many-chain estimates vs enumeration (65,536 states)."""
    b = W.c1_small(n_inst=2)
    p = dmala.Problem(b.H[0], b.y[0], b.sigma2[0], 16)
    K = exact.all_states(p.N, p.Q)
    ex = exact.exact_marginals(p, K)
    exl = exact.exact_llr(p, K)
    errs = []
    for C in (16, 256, 2048):
        r = dmala.dmala_sample(p, 1000 + C, 0, C, 50)
        errs.append(np.abs(dmala.marginals_is(p, r["k"]) - ex).mean())
    assert errs[2] < errs[0]
    assert errs[2] < 0.01
    r = dmala.dmala_sample(p, 5, 0, 2048, 50)
    L = dmala.llr_is(p, r["k"])
    assert np.median(np.abs(L - exl)) < 0.15


def test_c1_hard_decision_vs_map():
    b = W.c1_small(n_inst=12)
    same = 0
    for i in range(12):
        p = dmala.Problem(b.H[i], b.y[i], b.sigma2[i], 16)
        r = dmala.dmala_sample(p, 3, i, 16, 50)
        sym, E, c = dmala.hard_decision(p.Q, r["best_E"], r["best_k"])
        ms, mE = exact.map_detect(p)
        assert E >= mE - 1e-12                                    # MAP is a lower bound
        assert abs(p.energy(p.x_of(r["best_k"][c])) - E) < 1e-12  # reported energy is the state's
        same += np.array_equal(sym, ms)
    assert same >= 9


def test_trace_consistency():
    p = _prob(4, 4, 16, 10.0, 50)
    r = dmala.dmala_sample(p, 9, 3, 16, 30, trace=True)
    tr = r["trace"]
    assert np.array_equal(tr["accept"].sum(0), r["n_acc"])
    assert np.array_equal(tr["hash"][-1], dmala.state_hash(r["k"]))
    # accept decisions agree with the log ratio and margins are positive
    assert np.all(tr["mh_margin"] > 0)
    # rejection keeps the hash
    prev = np.concatenate([tr["init_hash"][None], tr["hash"][:-1]])
    assert np.all((tr["hash"] == prev) | tr["accept"])


def test_imperfect_csi_has_the_requested_nmse():
    b = W.make_batch(16, 16, 16, 16.5, 400, seed=91)
    for nmse in (-20.0, -10.0):
        e = W.imperfect_csi(b, nmse, seed=1)
        ratio = np.sum(np.abs(e.H - b.H) ** 2) / np.sum(np.abs(b.H) ** 2)
        assert abs(10 * np.log10(ratio) - nmse) < 0.1
        np.testing.assert_array_equal(e.y, b.y)
        np.testing.assert_array_equal(e.meta["H_true"], b.H)


def test_list_llr_over_the_whole_lattice_is_exact():
    """eq. llr_approx_app with the list equal to A^N is eq. exact_llr."""
    b = W.make_batch(2, 2, 16, 12.0, 3, seed=44)
    for i in range(3):
        prob = dmala.Problem(b.H[i], b.y[i], b.sigma2[i], 16)
        K = exact.all_states(prob.N, prob.Q)
        np.testing.assert_allclose(dmala.llr_list(prob, K, clip=1e9), exact.exact_llr(prob, K), atol=1e-9)
        # duplicates do not count; a one-sided list clips
        dup = np.concatenate([K, K[:7]])
        np.testing.assert_allclose(dmala.llr_list(prob, dup, clip=1e9), exact.exact_llr(prob, K), atol=1e-9)
        one = dmala.llr_list(prob, K[:1])
        assert np.all(np.abs(one) == dmala.LLR_CLIP)


def test_mc_llr_with_exact_frequencies_is_exact():
    """eq. mc on the bit indicators with every state repeated in proportion to pi tends to eq. exact_llr."""
    b = W.make_batch(1, 2, 16, 10.0, 2, seed=45)
    for i in range(2):
        prob = dmala.Problem(b.H[i], b.y[i], b.sigma2[i], 16, tau=1.0)
        K = exact.all_states(prob.N, prob.Q)
        p = np.exp(exact.log_target(prob, K, tempered=False))
        reps = np.round(p * 1e6).astype(int)
        samples = np.repeat(K, reps, axis=0)
        ex = exact.exact_llr(prob, K)
        mc = dmala.llr_mc(prob, samples, clip=1e9)
        ok = np.abs(ex) < 8          # bits whose rarer side has at least ~300 samples
        np.testing.assert_allclose(mc[ok], ex[ok], atol=5e-3)
        assert dmala.llr_mc(prob, K[:1]).max() == dmala.LLR_CLIP
