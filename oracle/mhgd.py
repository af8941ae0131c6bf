"""The earlier gradient-based MCMC detector that the paper compares against (MHGD) -- test oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Section III-A (the Remark on Fig. 1(a)) describes how those detectors make a
candidate: a gradient step in the continuous relaxation, a Gaussian random walk,
and a deterministic mapping of the result to its nearest lattice point; because
the mapping has no proposal probability attached, the MH test cannot contain the
proposal ratio, and the chain samples a biased distribution (Section III-B,
fig. tv_theory: its total-variation distance to the target levels off near 0.2 on 2x2
QPSK while DMALA's goes to zero).  The paper gives no further detail, so this
oracle takes these readings (listed in the design notes):

* the continuous candidate is the preconditioned Langevin step of the Remark
  after Algorithm 1, on the tempered metric f/tau:
      x~ = x + (alpha/2) M grad(f/tau)(x) + sqrt(alpha beta) w,   w ~ N(0, I_N),
  with the Section IV-A parameters (alpha = sigma^2, beta = dmin^2/sigma^2,
  gamma = sigma^2/(2 dmin^2), which the paper takes from the MHGD reference);
  one gradient step per transition, no step-size search;
* the mapping takes every real dimension to its nearest PAM level (the square
  QAM lattice is a product of PAM alphabets), edge cells extending to infinity;
* the MH test accepts with min(1, pi_a(x') / pi_a(x)), i.e. the symmetric-proposal
  form with the missing proposal ratio left out.

Random numbers follow the detector's word layout (see philox.py): word n of
transition t drives dimension n through w_n = Phi^-1(u_n), u_n the word's high
24 bits plus one half, times 2^-24 (so 0 < u_n < 1); the MH uniform and the
initial state are those of the DMALA sampler.

Exact kernel: the candidate law factorises over dimensions, each the Gaussian
N(c_n, alpha beta) integrated over the cells of the nearest-level mapping, so the
transition matrix of the chain follows in closed form (eq. trans_prob_1 with this
q and the acceptance above).
"""
import numpy as np
from scipy.special import ndtr, ndtri

from . import philox
from .dmala import Problem, PRECOND, state_hash


def candidate_centre(prob, x):
    """Mean of the continuous candidate: x + (alpha/2) M grad(f/tau)(x), shape (..., N)."""
    g = prob.grad_f(x) / prob.tau
    return x + 0.5 * prob.alpha * (g @ prob.Mpre.T)


def noise_std(prob):
    return np.sqrt(prob.alpha * prob.beta)


def cell_edges(prob):
    """Boundaries of the nearest-level cells: midpoints between adjacent levels, (Q-1,)."""
    return 0.5 * (prob.levels[1:] + prob.levels[:-1])


def nearest_level(prob, xt):
    """Index of the nearest level of every entry (the QAM mapping per real dimension) and the
    distance of the entry to its nearest cell boundary, in units of the level spacing 2 s."""
    e = cell_edges(prob)
    k = np.searchsorted(e, xt, side="right")                  # number of edges <= xt
    margin = np.min(np.abs(xt[..., None] - e), axis=-1) / (2.0 * prob.s) if len(e) else np.full(xt.shape, np.inf)
    return k, margin


def gaussian_uniform(w):
    """The uniform in (0, 1) of a word: (high 24 bits + 1/2) * 2^-24."""
    return ((np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def cell_probs(prob, c):
    """Probability of each level under N(c_n, alpha beta) mapped to the nearest level, (..., N, Q)."""
    sd = noise_std(prob)
    e = np.concatenate([[-np.inf], cell_edges(prob), [np.inf]])
    z = (e[None, :] - np.asarray(c)[..., None]) / sd            # (..., N, Q+1)
    # upper-tail form on the right of the centre keeps small cell probabilities accurate
    lo, hi = z[..., :-1], z[..., 1:]
    right = lo > 0
    return np.where(right, ndtr(-lo) - ndtr(-hi), ndtr(hi) - ndtr(lo))


def mhgd_sample(prob, seed, instance, n_chains, n_iters, trace=False):
    """n_chains independent MHGD chains (readings above), vectorised over chains.

    Returns final levels, accept counts, best (minimum-residual) states and energies,
    and with trace=True per-transition accept flags, state hashes, the energies after
    the transition and of the candidate, and the decision margins: the candidate's
    distance to the nearest cell boundary (level-spacing units) and |log u - log A|.
    """
    N, tau = prob.N, prob.tau
    chains = np.arange(n_chains)
    w = philox.words(seed, instance, chains, 0, N)
    k = philox.init_level_index(w[:, :N], prob.Q)
    x = prob.x_of(k)
    f_x = prob.f(x) / tau
    E = prob.energy(x)
    best_E, best_k = E.copy(), k.copy()
    n_acc = np.zeros(n_chains, dtype=np.int64)
    tr = None
    if trace:
        tr = dict(accept=np.zeros((n_iters, n_chains), bool), hash=np.zeros((n_iters, n_chains), np.uint32),
                  cat_margin=np.zeros((n_iters, n_chains)), mh_margin=np.zeros((n_iters, n_chains)),
                  E=np.zeros((n_iters, n_chains)), E_prop=np.zeros((n_iters, n_chains)),
                  init_hash=state_hash(k), init_E=E.copy())
    sd = noise_std(prob)
    for t in range(1, n_iters + 1):
        w = philox.words(seed, instance, chains, t, N)
        # gradient step, Gaussian random walk, nearest-point mapping
        xt = candidate_centre(prob, x) + sd * ndtri(gaussian_uniform(w[:, :N]))
        kp, cmarg = nearest_level(prob, xt)
        xp = prob.x_of(kp)
        f_p = prob.f(xp) / tau
        # MH test without the proposal ratio
        R = f_p - f_x
        u_mh = philox.low_byte_uniform(w, 0)
        acc = np.exp(np.minimum(0.0, R)) > u_mh
        E_p = prob.energy(xp)
        k = np.where(acc[:, None], kp, k)
        x = prob.x_of(k)
        f_x = np.where(acc, f_p, f_x)
        E = np.where(acc, E_p, E)
        n_acc += acc
        better = E < best_E
        best_E = np.where(better, E, best_E)
        best_k = np.where(better[:, None], k, best_k)
        if trace:
            with np.errstate(divide="ignore"):
                lu = np.log(u_mh)
            tr["accept"][t - 1] = acc
            tr["hash"][t - 1] = state_hash(k)
            tr["cat_margin"][t - 1] = np.min(cmarg, axis=-1)
            tr["mh_margin"][t - 1] = np.abs(R - lu)
            tr["E"][t - 1] = E
            tr["E_prop"][t - 1] = E_p
    return dict(k=k, best_k=best_k, best_E=best_E, n_acc=n_acc, trace=tr)


def transition_matrix(prob, K, with_reverse=False):
    """Exact kernel of the MHGD chain over the states K (rows = current state).

    q(x'|x) = prod_n P(nearest level of N(c_n(x), alpha beta) = x'_n); acceptance
    min(1, pi_a(x')/pi_a(x)), or with with_reverse=True the exact MH acceptance
    min(1, pi_a(x') q(x|x') / (pi_a(x) q(x'|x))) that the mapping's missing
    probability would allow.  Returns (P, log q matrix).
    """
    X = prob.x_of(K)
    cp = cell_probs(prob, candidate_centre(prob, X))               # (S, N, Q)
    S, N = K.shape
    with np.errstate(divide="ignore"):
        lcp = np.log(cp)
    LQ = np.zeros((S, S))
    for n in range(N):
        LQ += lcp[:, n, :][:, K[:, n]]
    ft = prob.f(X) / prob.tau
    R = ft[None, :] - ft[:, None]
    if with_reverse:
        R = R + LQ.T - LQ
    P = np.exp(LQ + np.minimum(0.0, R))
    np.fill_diagonal(P, 0.0)
    P[np.arange(S), np.arange(S)] = 1.0 - P.sum(axis=1)
    return P, LQ


def stationary(P):
    """Stationary distribution of a row-stochastic matrix (left eigenvector for eigenvalue 1)."""
    ev, V = np.linalg.eig(P.T)
    i = int(np.argmin(np.abs(ev - 1.0)))
    v = np.real(V[:, i])
    return v / v.sum()


def make_problem(H_c, y_c, sigma2, M, tau=2.0):
    """The preconditioned problem of eq. sys_model with the Section IV-A parameters."""
    return Problem(H_c, y_c, sigma2, M, PRECOND, tau)
