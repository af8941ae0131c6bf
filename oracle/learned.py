"""Learned proposal for the DMALA chain, its mixture with the plain kernel, and
the training of its network, in float64 (test oracle).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import this module; the product path never does.

The paper does not define a learned proposal: its conclusion (Section V)
names the combination of model-driven and data-driven methods as future work.
What makes one admissible is the MH construction of Section III-A (eq.
acc_prob, eq. acc_prob_general): a proposal q(. | x) that is a fixed function
of the current state, positive on the whole alphabet, and used for both the
forward and the reverse term leaves the target pi_a (eq. aux) invariant; and a
random choice between two such kernels, made independently of the state,
keeps pi_a invariant as well (the mixture of two pi_a-invariant kernels).

Everything below works in index units: level j in 0..Q-1 is the point
x = s (2 j - Q + 1) of the per-axis PAM alphabet.

Plain preconditioned proposal (the Remark after Algorithm 1, eq. nu, on f/tau):
in index units it is a discretised Gaussian per real dimension n,
    log q_n(j) = -kappa (j - mu_n)^2 - log Z_n,
    mu_n  = k_n + alpha [M grad(f/tau)(x)]_n / (4 s),   kappa = 2 s^2 / (alpha beta).

Learned proposal: the same family with the centre and the precision of every
dimension set by a small network per antenna m (dimensions 2m = Re, 2m+1 = Im):
    (D_re, D_im, b_re, b_im) = MLP(phi_m),
    mu^L_n = mu_n + D_n,  kappa^L_n = kappa 2^{clamp(b_n, -4, 4)}.
With a zero output layer the learned proposal is the plain one.

Features phi_m (7 values; the network sees an 8th input fixed at 1 for the
first layer's bias), c = (Q-1)/2, h = Q/2:
    (mu_re - c)/h, (mu_im - c)/h, (k_re - c)/h, (k_im - c)/h,
    log2(sigma^2 M_nn / (8 s^2)) / 8   -- variance of the damped LS estimate of
                                          the antenna, in index units^2,
    log2(sigma^2 / (8 s^2 G_nn)) / 8   -- variance of one axis given the others,
    log2(Q) / 4
(n = 2m; the real-equivalent M and G have equal diagonal entries at 2m, 2m+1).

Network: 8 -> 64 -> 64 -> 4, ReLU after the two hidden layers.  Parameters are
held in float32 by the caller.  Inference (inside the chain) rounds the
parameters, the inputs and the hidden activations to bfloat16 (round to
nearest, ties to even) and sums the products exactly (float64 here);
training uses the unrounded network.

Mixture (one kernel per chain and transition): with u the 24-bit uniform from
the low bytes of words 4, 5, 6 of the transition's random stream, the plain
kernel is used when u < eps and the learned kernel otherwise; each kernel does
a full MH step with its own forward and reverse proposal.

Training: cross-entropy of the learned proposal at the transmitted levels,
averaged over rows (one row per antenna of a chain state), Adam (Kingma & Ba,
ICLR 2015) with bias correction.
"""
import numpy as np

from . import philox
from .dmala import Problem, PRECOND, log_softmax, sum_log_q, inverse_cdf, state_hash

N_FEAT = 7
HID = 64
N_OUT = 4
B_CLAMP = 4.0
LN2 = np.log(2.0)

PARAM_SHAPES = (("W1", (HID, N_FEAT)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
                ("W3", (N_OUT, HID)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


# ---------------------------------------------------------------- parameters

def unflatten(flat):
    """Flat float array (W1, b1, W2, b2, W3, b3, row-major) -> dict of float64 arrays."""
    flat = np.asarray(flat, dtype=np.float64).reshape(-1)
    if flat.size != N_PARAMS:
        raise ValueError("expected %d parameters" % N_PARAMS)
    out, o = {}, 0
    for name, shp in PARAM_SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp).copy()
        o += n
    return out


def flatten(P):
    return np.concatenate([np.asarray(P[name], dtype=np.float64).reshape(-1) for name, _ in PARAM_SHAPES])


def init_params(seed, zero_last=False):
    """He-normal hidden layers, small output layer; float32-representable values."""
    rng = np.random.default_rng(seed)
    P = {"W1": rng.standard_normal((HID, N_FEAT)) * np.sqrt(2.0 / (N_FEAT + 1)), "b1": np.zeros(HID),
         "W2": rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID), "b2": np.zeros(HID),
         "W3": rng.standard_normal((N_OUT, HID)) * (0.0 if zero_last else 0.01), "b3": np.zeros(N_OUT)}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                     # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)


# ---------------------------------------------------------------- the network

def mlp_forward(P, X, rounded=True):
    """Outputs (R, 4) of the network on feature rows X (R, 7) and the layer cache."""
    r = bf16 if rounded else (lambda v: np.asarray(v, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    a0 = r(X)
    z1 = a0 @ r(P["W1"]).T + r(P["b1"])
    a1 = r(np.maximum(z1, 0.0))
    z2 = a1 @ r(P["W2"]).T + r(P["b2"])
    a2 = r(np.maximum(z2, 0.0))
    out = a2 @ r(P["W3"]).T + r(P["b3"])
    return out, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2)


def mlp_backward(P, cache, d_out):
    """Gradients of sum(d_out * out) with respect to the parameters (unrounded network)."""
    g = {}
    g["W3"] = d_out.T @ cache["a2"]
    g["b3"] = d_out.sum(axis=0)
    d2 = (d_out @ P["W3"]) * (cache["z2"] > 0)
    g["W2"] = d2.T @ cache["a1"]
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (cache["z1"] > 0)
    g["W1"] = d1.T @ cache["a0"]
    g["b1"] = d1.sum(axis=0)
    return g


def head(out):
    """Network outputs -> centre offsets (R, 2) and log2 precision factors (R, 2), clamped."""
    return out[:, 0:2], np.clip(out[:, 2:4], -B_CLAMP, B_CLAMP)


# ---------------------------------------------------------------- proposal parameters

def plain_index_params(prob, k):
    """Centre mu (..., N) and precision kappa (natural log units) of the plain proposal."""
    if prob.variant != PRECOND:
        raise ValueError("the learned proposal extends the preconditioned one")
    x = prob.x_of(k)
    mg = (prob.grad_f(x) / prob.tau) @ prob.Mpre.T
    mu = np.asarray(k, dtype=np.float64) + prob.alpha * mg / (4.0 * prob.s)
    kappa = 2.0 * prob.s ** 2 / (prob.alpha * prob.beta)
    return mu, kappa


def antenna_constants(prob):
    """Per-antenna feature constants (Nt, 3): LS variance, conditional variance, order."""
    G = prob.H.T @ prob.H
    d = np.arange(prob.Nt) * 2
    v_ls = np.log2(prob.sigma2 * prob.Mpre[d, d] / (8.0 * prob.s ** 2)) / 8.0
    v_c = np.log2(prob.sigma2 / (8.0 * prob.s ** 2 * G[d, d])) / 8.0
    return np.stack([v_ls, v_c, np.full(prob.Nt, np.log2(prob.Q) / 4.0)], axis=-1)


def features(prob, k, mu=None):
    """Feature rows phi (..., Nt, 7) at level-index states k (..., N)."""
    k = np.asarray(k)
    if mu is None:
        mu, _ = plain_index_params(prob, k)
    c, hq = (prob.Q - 1) / 2.0, prob.Q / 2.0
    lead = k.shape[:-1]
    f = np.empty(lead + (prob.Nt, N_FEAT))
    f[..., 0] = (mu[..., 0::2] - c) / hq
    f[..., 1] = (mu[..., 1::2] - c) / hq
    f[..., 2] = (k[..., 0::2] - c) / hq
    f[..., 3] = (k[..., 1::2] - c) / hq
    f[..., 4:7] = np.broadcast_to(antenna_constants(prob), lead + (prob.Nt, 3))
    return f


def learned_index_params(prob, k, P, rounded=True):
    """Centre (..., N) and precision (..., N) (natural log units) of the learned proposal."""
    k = np.asarray(k)
    mu, kappa = plain_index_params(prob, k)
    phi = features(prob, k, mu)
    lead = k.shape[:-1]
    out, _ = mlp_forward(P, phi.reshape(-1, N_FEAT), rounded)
    D, b = head(out)
    D = D.reshape(lead + (prob.Nt, 2)).reshape(lead + (prob.N,))
    b = b.reshape(lead + (prob.Nt, 2)).reshape(lead + (prob.N,))
    return mu + D, kappa * np.exp2(b)


def gaussian_logits(mu, kappa, Q):
    """Unnormalised natural-log logits -kappa (j - mu)^2 over j = 0..Q-1, shape (..., N, Q)."""
    j = np.arange(Q, dtype=np.float64)
    t = j - np.asarray(mu)[..., None]
    return -np.asarray(kappa)[..., None] * t * t if np.ndim(kappa) else -kappa * t * t


def learned_logits(prob, k, P, rounded=True):
    mu, kap = learned_index_params(prob, k, P, rounded)
    return gaussian_logits(mu, kap, prob.Q)


def plain_logits(prob, k):
    mu, kap = plain_index_params(prob, k)
    return gaussian_logits(mu, kap, prob.Q)


# ---------------------------------------------------------------- the mixture chain

def mixture_uniform(w):
    """Kernel-choice uniform: low bytes of words 4, 5, 6."""
    return philox.low_byte_uniform(w, 4)


def mixture_sample(prob, P, eps, seed, instance, n_chains, n_iters, trace=False):
    """Algorithm 1 on f/tau where every transition of every chain uses the plain
    kernel with probability eps and the learned one otherwise (the choice is
    made from the chain's random stream, independently of the state)."""
    N, Q, tau = prob.N, prob.Q, prob.tau
    chains = np.arange(n_chains)
    w = philox.words(seed, instance, chains, 0, N)
    k = philox.init_level_index(w[:, :N], Q)
    x = prob.x_of(k)
    f_x = prob.f(x) / tau
    lq_plain = log_softmax(plain_logits(prob, k))
    lq_learn = log_softmax(learned_logits(prob, k, P))
    E = prob.energy(x)
    best_E, best_k = E.copy(), k.copy()
    n_acc = np.zeros(n_chains, dtype=np.int64)
    n_learn = np.zeros(n_chains, dtype=np.int64)
    tr = None
    if trace:
        tr = dict(accept=np.zeros((n_iters, n_chains), bool), hash=np.zeros((n_iters, n_chains), np.uint32),
                  use_learned=np.zeros((n_iters, n_chains), bool),
                  cat_margin=np.zeros((n_iters, n_chains)), mh_margin=np.zeros((n_iters, n_chains)),
                  mix_margin=np.zeros((n_iters, n_chains)), init_hash=state_hash(k))
    for t in range(1, n_iters + 1):
        w = philox.words(seed, instance, chains, t, N)
        u = philox.uniform_draw(w[:, :N])
        um = mixture_uniform(w)
        use_l = um >= eps
        logq = np.where(use_l[:, None, None], lq_learn, lq_plain)
        kp, cmarg = inverse_cdf(logq, u)
        lq_f = sum_log_q(logq, kp)
        xp = prob.x_of(kp)
        lqp_plain = log_softmax(plain_logits(prob, kp))
        lqp_learn = log_softmax(learned_logits(prob, kp, P))
        lq_r = sum_log_q(np.where(use_l[:, None, None], lqp_learn, lqp_plain), k)
        f_p = prob.f(xp) / tau
        R = f_p - f_x + lq_r - lq_f
        u_mh = philox.low_byte_uniform(w, 0)
        acc = np.exp(np.minimum(0.0, R)) > u_mh
        E_p = prob.energy(xp)
        k = np.where(acc[:, None], kp, k)
        f_x = np.where(acc, f_p, f_x)
        lq_plain = np.where(acc[:, None, None], lqp_plain, lq_plain)
        lq_learn = np.where(acc[:, None, None], lqp_learn, lq_learn)
        E = np.where(acc, E_p, E)
        n_acc += acc
        n_learn += use_l
        better = E < best_E
        best_E = np.where(better, E, best_E)
        best_k = np.where(better[:, None], k, best_k)
        if trace:
            with np.errstate(divide="ignore"):
                lu = np.log(u_mh)
            tr["accept"][t - 1] = acc
            tr["hash"][t - 1] = state_hash(k)
            tr["use_learned"][t - 1] = use_l
            tr["cat_margin"][t - 1] = np.min(cmarg, axis=-1)
            tr["mh_margin"][t - 1] = np.abs(R - lu)
            tr["mix_margin"][t - 1] = np.abs(um - eps)
    return dict(k=k, best_k=best_k, best_E=best_E, n_acc=n_acc, n_learned=n_learn, trace=tr)


def kernel_matrix(prob, K, logq_rows):
    """MH transition matrix on the states K for a proposal given as log q rows (S, N, Q)."""
    S, N = K.shape
    LQ = np.zeros((S, S))
    for n in range(N):
        LQ += logq_rows[:, n, :][:, K[:, n]]
    ft = prob.f(prob.x_of(K)) / prob.tau
    logA = np.minimum(0.0, ft[None, :] - ft[:, None] + LQ.T - LQ)
    Pm = np.exp(LQ + logA)
    np.fill_diagonal(Pm, 0.0)
    Pm[np.arange(S), np.arange(S)] = 1.0 - Pm.sum(axis=1)
    return Pm, LQ


def mixture_transition_matrix(prob, P, eps, K):
    """Exact kernel eps P_plain + (1 - eps) P_learned on the enumerated states K."""
    Pp, _ = kernel_matrix(prob, K, log_softmax(plain_logits(prob, K)))
    Pl, LQl = kernel_matrix(prob, K, log_softmax(learned_logits(prob, K, P)))
    return eps * Pp + (1.0 - eps) * Pl, Pp, Pl, LQl


# ---------------------------------------------------------------- training

def proposal_xent(mu, kappa, Q, target):
    """Cross-entropy -log q(target) of discretised Gaussians and its derivatives.

    mu, kappa, target: (R,) arrays (natural-log precision).  Returns
    (loss (R,), d loss / d mu, d loss / d kappa)."""
    lg = gaussian_logits(mu, kappa, Q)
    lq = log_softmax(lg)
    p = np.exp(lq)
    j = np.arange(Q, dtype=np.float64)
    t = np.asarray(target)
    loss = -np.take_along_axis(lq, t[:, None], axis=-1)[:, 0]
    Ej = p @ j
    Et2 = np.sum(p * (j[None, :] - mu[:, None]) ** 2, axis=-1)
    d_mu = -2.0 * kappa * (t - Ej)
    d_kappa = (t - mu) ** 2 - Et2
    return loss, d_mu, d_kappa


def training_loss(P, X, mu, kappa, Q, target, grad=False):
    """Mean over rows of -log q^L(target) summed over the two axes of the antenna.

    X (R, 7) features, mu (R, 2) plain centres, kappa (R,) plain precision
    (natural log units), Q (R,) or scalar, target (R, 2) level indices."""
    R = X.shape[0]
    out, cache = mlp_forward(P, X, rounded=False)
    D, b = head(out)
    Qv = np.broadcast_to(np.asarray(Q), (R,))
    loss = np.zeros(R)
    d_out = np.zeros((R, N_OUT))
    for q in np.unique(Qv):
        sel = Qv == q
        for ax in range(2):
            muL = mu[sel, ax] + D[sel, ax]
            kL = kappa[sel] * np.exp2(b[sel, ax])
            l, dm, dk = proposal_xent(muL, kL, int(q), target[sel, ax])
            loss[sel] += l
            d_out[sel, ax] = dm
            inside = np.abs(out[sel, 2 + ax]) < B_CLAMP
            d_out[sel, 2 + ax] = dk * kL * LN2 * inside
    L = loss.mean()
    if not grad:
        return L
    return L, mlp_backward(P, cache, d_out / R)


def adam_step(P, G, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on P, m, v); step counts from 1."""
    for name, _ in PARAM_SHAPES:
        m[name] = b1 * m[name] + (1.0 - b1) * G[name]
        v[name] = b2 * v[name] + (1.0 - b2) * G[name] ** 2
        mh = m[name] / (1.0 - b1 ** step)
        vh = v[name] / (1.0 - b2 ** step)
        P[name] = P[name] - lr * mh / (np.sqrt(vh) + eps)
    return P, m, v
