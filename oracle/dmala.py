"""DMALA-based soft MIMO detection in float64 -- the test oracle.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import this package; the product path never does.

Plain, slow, direct transcription of the method of Zhou et al., "Near-Optimal
MIMO Detection Using Gradient-Based MCMC in Discrete Spaces":

* real-valued system model and posterior: Section II-A, eqs. sys_model, post, f;
* discrete Langevin proposal and its element-wise factorisation: Section III-A,
  eqs. dis_prop, dis_prop_fac1, dis_prop_fac2, exp_fac, softmax; the
  preconditioned variant (nu instead of mu): the Remark after Algorithm 1;
* MH correction: eq. acc_prob; sampler: Algorithm 1;
* tempered target and IS-based LLR: Section III-C, eqs. aux, llr_is (log-sum-exp
  form of eq. llr_simple with F(a) = log(1+e^a) evaluated exactly); soft
  detection: Algorithm 2;
* hard decision: the minimum-residual sample (text after Algorithm 1);
* parameters: Section IV-A (alpha = sigma^2, beta = dmin^2/sigma^2,
  gamma = sigma^2/(2 dmin^2), tau = 2, final sample of each of the parallel
  samplers used for the soft output).

Readings where the paper is silent (each is listed in the design notes):
* the real-equivalent vector interleaves Re/Im per antenna (x_{2m} = Re x_m);
* dmin is half the minimum distance, i.e. the level step s of unit-energy QAM;
* tempering divides f (and its gradient) by tau; alpha, beta, gamma are not
  rescaled; the preconditioner M does not depend on tau;
* n_iters is the number of MH transitions (the paper's T is n_iters + 1);
* the hard decision ranges over every state visited by every chain, including
  the initial one; ties go to the earliest iteration, then the lowest chain;
* bits: per-axis binary-reflected Gray label of the level index, MSB first,
  antenna bits ordered [I bits, Q bits]; b = +1 <-> label bit 0;
* symbol marginals (not defined in the paper) use the symbol-level analogue of
  the IS estimator of Appendix C:
      p_m(a) propto sum_s pi_a(a | x^{[s]}_{-m}) exp(((tau-1)/tau) f(x^{[s]}_{m<-a})).
"""
import numpy as np

from . import philox

NAIVE = "naive"
PRECOND = "precond"


# ---------------------------------------------------------------- constellation

def pam_levels(Q):
    """Real PAM alphabet A of unit-average-energy square Q^2-QAM (ascending)."""
    M = Q * Q
    s = np.sqrt(3.0 / (2.0 * (M - 1)))
    return s * (2.0 * np.arange(Q) - Q + 1), s


def gray(k):
    k = np.asarray(k)
    return k ^ (k >> 1)


def gray_bits(k, nbits):
    """Gray label bits of level index k, MSB first. Shape (..., nbits)."""
    g = gray(np.asarray(k, dtype=np.int64))
    return np.stack([(g >> (nbits - 1 - b)) & 1 for b in range(nbits)], axis=-1)


def level_from_gray_bits(bits):
    """Inverse of gray_bits: the level index whose Gray label is `bits`."""
    bits = np.asarray(bits, dtype=np.int64)
    nb = bits.shape[-1]
    g = np.zeros(bits.shape[:-1], dtype=np.int64)
    for b in range(nb):
        g = (g << 1) | bits[..., b]
    k = g.copy()
    shift = g >> 1
    while np.any(shift):
        k ^= shift
        shift >>= 1
    return k


# ---------------------------------------------------------------- the problem

class Problem:
    """One detection problem in the real-valued model of eq. sys_model."""

    def __init__(self, H_c, y_c, sigma2, M, variant=PRECOND, tau=2.0,
                 alpha=None, beta=None, gamma=None):
        H_c = np.asarray(H_c, dtype=np.complex128)
        y_c = np.asarray(y_c, dtype=np.complex128)
        Nr, Nt = H_c.shape
        Q = int(round(np.sqrt(M)))
        if Q * Q != M:
            raise ValueError("square QAM only")
        if not sigma2 > 0:
            raise ValueError("sigma^2 must be positive (Lemma 1)")
        self.Nt, self.Nr, self.M, self.Q = Nt, Nr, M, Q
        self.N = 2 * Nt
        self.nbits_axis = int(round(np.log2(Q)))
        self.levels, self.s = pam_levels(Q)
        self.dmin = self.s
        self.sigma2 = float(sigma2)
        self.tau = float(tau)
        self.variant = variant
        # Section IV-A defaults
        self.alpha = float(alpha) if alpha is not None else self.sigma2
        self.beta = float(beta) if beta is not None else self.dmin ** 2 / self.sigma2
        self.gamma = float(gamma) if gamma is not None else self.sigma2 / (2.0 * self.dmin ** 2)
        # equivalent real-valued model, Re/Im interleaved per antenna
        H = np.zeros((2 * Nr, 2 * Nt))
        H[0::2, 0::2] = H_c.real
        H[0::2, 1::2] = -H_c.imag
        H[1::2, 0::2] = H_c.imag
        H[1::2, 1::2] = H_c.real
        y = np.zeros(2 * Nr)
        y[0::2] = y_c.real
        y[1::2] = y_c.imag
        self.H, self.y = H, y
        self.H_c, self.y_c = H_c, y_c
        if variant == PRECOND:
            # damped-Hessian preconditioner M = (H^T H + gamma I)^-1 (Remark, Sec. III-A)
            self.Mpre = np.linalg.inv(H.T @ H + self.gamma * np.eye(self.N))
        elif variant == NAIVE:
            self.Mpre = None
        else:
            raise ValueError(variant)

    # eq. f
    def f(self, x):
        r = self.y - x @ self.H.T
        return -np.sum(r * r, axis=-1) / self.sigma2

    def energy(self, x):
        r = self.y - x @ self.H.T
        return np.sum(r * r, axis=-1)

    # eq. grad
    def grad_f(self, x):
        return (2.0 / self.sigma2) * ((self.y - x @ self.H.T) @ self.H)

    def x_of(self, k):
        """Real vector from level indices."""
        return self.levels[np.asarray(k)]

    def proposal_logits(self, x):
        """Logits of the factorised proposal q_n(. | x_n) over the alphabet.

        Uses f/tau (Algorithm 2 runs Algorithm 1 on the tempered target).
        naive:   mu(a) = 1/2 [grad]_n (a - x_n) - (a - x_n)^2 / (2 alpha)      (eq. exp_fac)
        precond: nu(a) = 1/(2 beta) [M grad]_n (a - x_n) - (a - x_n)^2 / (2 alpha beta)
        Returns shape (..., N, Q).
        """
        g = self.grad_f(x) / self.tau
        d = self.levels[None, :] - x[..., None]
        if self.variant == NAIVE:
            return 0.5 * g[..., None] * d - d * d / (2.0 * self.alpha)
        mg = g @ self.Mpre.T
        ab = self.alpha * self.beta
        return (1.0 / (2.0 * self.beta)) * mg[..., None] * d - d * d / (2.0 * ab)


def log_softmax(logits):
    """eq. softmax in the log domain, over the last axis."""
    mx = np.max(logits, axis=-1, keepdims=True)
    return logits - (mx + np.log(np.sum(np.exp(logits - mx), axis=-1, keepdims=True)))


def sum_log_q(logq, k):
    """log q(x'|x) = sum_n log q_n(x'_n | x_n) (eq. dis_prop_fac1); logq (..., N, Q), k (..., N)."""
    return np.sum(np.take_along_axis(logq, np.asarray(k)[..., None], axis=-1)[..., 0], axis=-1)


def inverse_cdf(logits, u):
    """Draw index j = smallest j with u * W < sum_{i<=j} w_i, w = exp(logits - max), W = sum w.

    logits (..., K), u (...,).  Returns (index, margin) where margin is the
    distance of u to the nearest internal CDF boundary (probability units).
    If rounding leaves no qualifying j, the last index is taken.
    """
    mx = np.max(logits, axis=-1, keepdims=True)
    w = np.exp(logits - mx)
    cw = np.cumsum(w, axis=-1)
    W = cw[..., -1:]
    hit = (u[..., None] * W) < cw
    K = logits.shape[-1]
    idx = np.where(np.any(hit, axis=-1), np.argmax(hit, axis=-1), K - 1)
    if K > 1:
        margin = np.min(np.abs(u[..., None] - cw[..., :-1] / W), axis=-1)
    else:
        margin = np.full(u.shape, np.inf)
    return idx, margin


def state_hash(k):
    """32-bit state fingerprint sum_n (k_n + 1) * ((2n+1) * 0x9E3779B1) mod 2^32."""
    k = np.asarray(k, dtype=np.uint64)
    n = np.arange(k.shape[-1], dtype=np.uint64)
    mult = ((2 * n + 1) * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    return (np.sum((k + np.uint64(1)) * mult, axis=-1) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


# ---------------------------------------------------------------- Algorithm 1

def dmala_sample(prob, seed, instance, n_chains, n_iters, trace=False):
    """Algorithm 1 on the tempered metric f/tau for n_chains parallel samplers.

    Chains are independent (their random words differ by the chain counter); the
    loop is vectorised over chains only.  Returns a dict with the final level
    indices, best (minimum-residual) states and energies, accept counts and,
    when trace is true, per-transition accept flags, state hashes, the energies of
    the state after the transition and of the proposal, and the decision margins of
    every draw; trace="states" also records the state before and the proposal of
    every transition (int8 level indices) and the energy before.
    """
    N, Q, tau = prob.N, prob.Q, prob.tau
    chains = np.arange(n_chains)
    w = philox.words(seed, instance, chains, 0, N)
    k = philox.init_level_index(w[:, :N], Q)               # initial state x^(1)
    x = prob.x_of(k)
    f_x = prob.f(x) / tau                                   # tempered metric
    logq = log_softmax(prob.proposal_logits(x))             # q_n(. | x_n^(1))
    E = prob.energy(x)
    best_E, best_k = E.copy(), k.copy()
    n_acc = np.zeros(n_chains, dtype=np.int64)
    tr = None
    if trace:
        tr = dict(accept=np.zeros((n_iters, n_chains), bool),
                  hash=np.zeros((n_iters, n_chains), np.uint32),
                  prop_hash=np.zeros((n_iters, n_chains), np.uint32),
                  cat_margin=np.zeros((n_iters, n_chains)),
                  mh_margin=np.zeros((n_iters, n_chains)),
                  log_ratio=np.zeros((n_iters, n_chains)),
                  E=np.zeros((n_iters, n_chains)), E_prop=np.zeros((n_iters, n_chains)),
                  init_hash=state_hash(k), init_E=E.copy())
        if trace == "states":
            tr["k_from"] = np.zeros((n_iters, n_chains, N), np.int8)
            tr["k_prop"] = np.zeros((n_iters, n_chains, N), np.int8)
            tr["E_from"] = np.zeros((n_iters, n_chains))
    for t in range(1, n_iters + 1):
        w = philox.words(seed, instance, chains, t, N)
        u = philox.uniform_draw(w[:, :N])
        # sample x'_n ~ q_n(. | x_n) for every n in parallel
        kp, cmarg = inverse_cdf(logq, u)
        # q(x' | x)
        lq_f = sum_log_q(logq, kp)
        xp = prob.x_of(kp)
        # grad f(x'), proposal at x', and q(x | x')
        logq_p = log_softmax(prob.proposal_logits(xp))
        lq_r = sum_log_q(logq_p, k)
        # f(x')
        f_p = prob.f(xp) / tau
        # acceptance (eq. acc_prob) against u ~ U(0,1)
        R = f_p - f_x + lq_r - lq_f
        A = np.exp(np.minimum(0.0, R))
        u_mh = philox.low_byte_uniform(w, 0)
        acc = A > u_mh
        E_p = prob.energy(xp)
        if trace == "states":
            tr["k_from"][t - 1] = k
            tr["k_prop"][t - 1] = kp
            tr["E_from"][t - 1] = E
        k = np.where(acc[:, None], kp, k)
        f_x = np.where(acc, f_p, f_x)
        logq = np.where(acc[:, None, None], logq_p, logq)
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
            tr["prop_hash"][t - 1] = state_hash(kp)
            tr["cat_margin"][t - 1] = np.min(cmarg, axis=-1)
            tr["mh_margin"][t - 1] = np.abs(R - lu)
            tr["log_ratio"][t - 1] = R
            tr["E"][t - 1] = E
            tr["E_prop"][t - 1] = E_p
    return dict(k=k, best_k=best_k, best_E=best_E, n_acc=n_acc, trace=tr)


# ---------------------------------------------------------------- estimators

def _lse(a, axis):
    mx = np.max(a, axis=axis, keepdims=True)
    mx = np.where(np.isfinite(mx), mx, 0.0)
    return np.squeeze(mx, axis=axis) + np.log(np.sum(np.exp(a - mx), axis=axis))


def llr_is(prob, k_samples, log_w=None, antennas=None):
    """IS-based bit LLRs (eq. llr_is, computed as eq. llr_simple in the log domain).

    k_samples: (S, N) level indices of samples from pi_a.  log_w: optional
    per-sample log weights replacing the uniform 1/S (used to pin the
    estimator to the exact expectation).  Returns (Nt, 2*log2(Q)) LLRs,
    L = log p(b=+1)/p(b=-1), bits ordered [I MSB..LSB, Q MSB..LSB]; with
    `antennas` only those rows are computed (the others are NaN).
    """
    k_samples = np.asarray(k_samples)
    S = k_samples.shape[0]
    lw = np.zeros(S) if log_w is None else np.asarray(log_w, dtype=np.float64)
    nb, tau = prob.nbits_axis, prob.tau
    c = (tau - 1.0) / tau
    out = np.full((prob.Nt, 2 * nb), np.nan)
    labels = gray_bits(k_samples, nb)                       # demap: (S, N, nb)
    ants = range(prob.Nt) if antennas is None else antennas
    for n in [2 * m + ax for m in ants for ax in (0, 1)]:
        m, axis = n // 2, n % 2
        for b in range(nb):
            lab_p = labels[:, n, :].copy()
            lab_p[:, b] = 0                                  # b_k = +1
            lab_m = labels[:, n, :].copy()
            lab_m[:, b] = 1                                  # b_k = -1
            kp = k_samples.copy()
            kp[:, n] = level_from_gray_bits(lab_p)
            km = k_samples.copy()
            km[:, n] = level_from_gray_bits(lab_m)
            fp = prob.f(prob.x_of(kp))
            fm = prob.f(prob.x_of(km))
            g = (fp - fm) / tau
            num = _lse(lw + c * fp - np.logaddexp(0.0, -g), axis=0)
            den = _lse(lw + c * fm - np.logaddexp(0.0, g), axis=0)
            out[m, axis * nb + b] = num - den
    return out


LLR_CLIP = 20.0


def llr_list(prob, k_samples, clip=LLR_CLIP):
    """List-based LLRs (eq. llr_approx_app): the APP sums of eq. exact_llr restricted
    to the distinct samples of the list, log sum over the list's x with b_k = +1 of
    exp f(x) minus the same over b_k = -1.  A side with no sample gives +-clip (the
    paper leaves the empty case open; the result is also clipped to [-clip, clip])."""
    k = np.unique(np.asarray(k_samples), axis=0)             # the list: distinct samples
    nb = prob.nbits_axis
    f = prob.f(prob.x_of(k))
    labels = gray_bits(k, nb)                                # (L, N, nb)
    out = np.zeros((prob.Nt, 2 * nb))
    for n in range(prob.N):
        for b in range(nb):
            plus = labels[:, n, b] == 0
            if not plus.any():
                v = -clip
            elif plus.all():
                v = clip
            else:
                v = _lse(f[plus], axis=0) - _lse(f[~plus], axis=0)
            out[n // 2, (n % 2) * nb + b] = np.clip(v, -clip, clip)
    return out


def llr_mc(prob, k_samples, clip=LLR_CLIP):
    """Plain Monte Carlo LLRs (eq. mc on the bit indicators): log of the number of
    samples with b_k = +1 over the number with b_k = -1, duplicates counted; with
    samples from pi (tau = 1) this tends to eq. exact_llr.  Clipped to [-clip, clip]."""
    k = np.asarray(k_samples)
    nb = prob.nbits_axis
    labels = gray_bits(k, nb)
    out = np.zeros((prob.Nt, 2 * nb))
    for n in range(prob.N):
        for b in range(nb):
            npl = int(np.sum(labels[:, n, b] == 0))
            nmi = len(k) - npl
            v = clip if nmi == 0 else (-clip if npl == 0 else np.log(npl) - np.log(nmi))
            out[n // 2, (n % 2) * nb + b] = np.clip(v, -clip, clip)
    return out


def marginals_is(prob, k_samples, log_w=None, antennas=None):
    """Symbol posterior marginals, IS estimator at symbol level (see module doc).

    Returns (Nt, M) probabilities over points indexed k_I * Q + k_Q; with
    `antennas` only those rows are computed (the others are NaN).
    """
    k_samples = np.asarray(k_samples)
    S = k_samples.shape[0]
    lw = np.zeros(S) if log_w is None else np.asarray(log_w, dtype=np.float64)
    Q, tau = prob.Q, prob.tau
    c = (tau - 1.0) / tau
    kI, kQ = np.meshgrid(np.arange(Q), np.arange(Q), indexing="ij")
    kI, kQ = kI.reshape(-1), kQ.reshape(-1)                  # point a = kI*Q + kQ
    out = np.full((prob.Nt, Q * Q), np.nan)
    for m in (range(prob.Nt) if antennas is None else antennas):
        ks = np.repeat(k_samples[:, None, :], Q * Q, axis=1)  # (S, M, N)
        ks[:, :, 2 * m] = kI[None, :]
        ks[:, :, 2 * m + 1] = kQ[None, :]
        phi = prob.f(prob.x_of(ks))                           # f(x_{m<-a}), (S, M)
        log_cond = phi / tau - _lse(phi / tau, axis=1)[:, None]  # log pi_a(a | x_-m)
        lp = _lse(lw[:, None] + log_cond + c * phi, axis=0)
        lp -= _lse(lp, axis=0)
        out[m] = np.exp(lp)
    return out


def marginals_mc(Q, Nt, k_samples, log_w=None):
    """Plain Monte Carlo (eq. mc) histogram of the samples' symbols."""
    k_samples = np.asarray(k_samples)
    S = k_samples.shape[0]
    w = np.full(S, 1.0 / S) if log_w is None else np.exp(np.asarray(log_w) - _lse(np.asarray(log_w), 0))
    out = np.zeros((Nt, Q * Q))
    for m in range(Nt):
        idx = k_samples[:, 2 * m] * Q + k_samples[:, 2 * m + 1]
        np.add.at(out[m], idx, w)
    return out


def symbols_of(Q, k):
    k = np.asarray(k)
    return k[..., 0::2] * Q + k[..., 1::2]


def hard_decision(Q, best_E, best_k):
    """Minimum-residual sample over chains (lowest chain on ties)."""
    c = int(np.argmin(best_E))
    return symbols_of(Q, best_k[c]), float(best_E[c]), c


# ---------------------------------------------------------------- Algorithm 2

def detect(H_c, y_c, sigma2, M, n_chains, n_iters, seed, instance=0,
           variant=PRECOND, tau=2.0, alpha=None, beta=None, gamma=None,
           trace=False, estimators=True):
    """Algorithm 2: sample pi_a with Algorithm 1, then hard and soft outputs."""
    prob = Problem(H_c, y_c, sigma2, M, variant, tau, alpha, beta, gamma)
    r = dmala_sample(prob, seed, instance, n_chains, n_iters, trace=trace)
    sym, bestE, _ = hard_decision(prob.Q, r["best_E"], r["best_k"])
    out = dict(problem=prob, symbols=sym, best_energy=bestE, **r)
    if estimators:
        out["llr"] = llr_is(prob, r["k"])
        out["marginals"] = marginals_is(prob, r["k"])
        out["marginals_mc"] = marginals_mc(prob.Q, prob.Nt, r["k"])
    return out
