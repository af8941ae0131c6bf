"""Exhaustive enumeration over the lattice A^N for tiny systems (test oracle).

TEST INFRASTRUCTURE ONLY.

* posterior pi (eq. post) and tempered pi_a (eq. aux);
* exact bit LLRs (eq. exact_llr) and exact symbol marginals;
* MAP / ML hard decision by brute force;
* the exact transition matrix P of the DMALA chain (eq. trans_prob_1) and its
  second-largest eigenvalue modulus, the convergence rate r of Theorem 1;
* total-variation distance (definition in Theorem 1).
"""
import itertools

import numpy as np

from .dmala import log_softmax, gray_bits, symbols_of


def all_states(N, Q):
    """Every level-index vector in lexicographic order, shape (Q^N, N)."""
    return np.array(list(itertools.product(range(Q), repeat=N)), dtype=np.int64)


def log_target(prob, K, tempered=True):
    """Normalised log pi (tau=1) or log pi_a over the rows of K."""
    f = prob.f(prob.x_of(K))
    if tempered:
        f = f / prob.tau
    mx = np.max(f)
    return f - (mx + np.log(np.sum(np.exp(f - mx))))


def exact_llr(prob, K=None):
    """eq. exact_llr by enumeration: (Nt, 2*log2 Q), b=+1 <-> Gray label bit 0."""
    if K is None:
        K = all_states(prob.N, prob.Q)
    f = prob.f(prob.x_of(K))
    nb = prob.nbits_axis
    labels = gray_bits(K, nb)                               # (S, N, nb)
    out = np.zeros((prob.Nt, 2 * nb))
    for n in range(prob.N):
        for b in range(nb):
            plus = labels[:, n, b] == 0
            fp, fm = f[plus], f[~plus]
            mp, mm = fp.max(), fm.max()
            out[n // 2, (n % 2) * nb + b] = (mp + np.log(np.sum(np.exp(fp - mp)))) - (mm + np.log(np.sum(np.exp(fm - mm))))
    return out


def exact_marginals(prob, K=None, tempered=False):
    """Symbol posterior marginals p(x_m = a | y) by enumeration, (Nt, M)."""
    if K is None:
        K = all_states(prob.N, prob.Q)
    p = np.exp(log_target(prob, K, tempered=tempered))
    sym = symbols_of(prob.Q, K)
    out = np.zeros((prob.Nt, prob.M))
    for m in range(prob.Nt):
        np.add.at(out[m], sym[:, m], p)
    return out


def map_detect(prob, K=None):
    """Brute-force MAP (= ML under the uniform prior): argmin ||y - Hx||^2."""
    if K is None:
        K = all_states(prob.N, prob.Q)
    E = prob.energy(prob.x_of(K))
    i = int(np.argmin(E))
    return symbols_of(prob.Q, K[i]), float(E[i])


def transition_matrix(prob, K=None):
    """Exact DMALA kernel P(x'|x) (eq. trans_prob_1) on pi_a, rows = current state."""
    if K is None:
        K = all_states(prob.N, prob.Q)
    X = prob.x_of(K)
    logq = log_softmax(prob.proposal_logits(X))              # (S, N, Q)
    S, N = K.shape
    # log q(x_j | x_i) = sum_n logq[i, n, K[j, n]]
    LQ = np.zeros((S, S))
    for n in range(N):
        LQ += logq[:, n, :][:, K[:, n]]
    ft = prob.f(X) / prob.tau
    logA = np.minimum(0.0, ft[None, :] - ft[:, None] + LQ.T - LQ)   # eq. acc_prob
    Pm = np.exp(LQ + logA)
    np.fill_diagonal(Pm, 0.0)
    stay = 1.0 - Pm.sum(axis=1)
    Pm[np.arange(S), np.arange(S)] = stay
    return Pm, LQ, logA


def tv(p1, p2):
    return 0.5 * np.sum(np.abs(np.asarray(p1) - np.asarray(p2)), axis=-1)


def second_eigenvalue(P):
    ev = np.linalg.eigvals(P)
    ev = ev[np.argsort(-np.abs(ev))]
    return float(np.abs(ev[1]))
