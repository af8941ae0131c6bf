"""Convergence diagnostics of the device chain on enumerable systems.

Theorem 1 bounds the total-variation distance of the chain's law from the
target by a geometric rate r < 1; for a finite state space the rate is the
second-largest eigenvalue modulus of the transition matrix, and Section III-B
compares it for the naive and the preconditioned proposal over channel
realisations and SNRs.  Here the transition matrices are built from the
device's own proposal and acceptance (dmala_debug_eval evaluates every state
pair with the sampler's code), batched over realisations; the eigenvalue and
TV computations on the host are plain linear algebra on those matrices.
"""
import itertools

import numpy as np

from . import device_inputs, debug_eval


def all_states(N, Q):
    """Every level-index vector of N real dimensions, lexicographic order (Q^N, N)."""
    return np.array(list(itertools.product(range(Q), repeat=N)), dtype=np.int64)


def device_kernels(H, y, sigma2, M, precision="fp64", proposal="precond", tau=2.0, mlp_weights=None):
    """Exact transition matrices of the device chain, one per problem.

    H: (B, Nr, Nt) complex host array, y: (B, Nr), sigma2: (B,).  The state space
    (Q^(2 Nt) states) must have at most 32 states (<= 1024 ordered pairs).
    Returns (P (B, S, S), K (S, 2 Nt), log_pi (B, S)): log_pi is the tempered target
    as the device computes it (from its f(x') - f(x) values), normalised.
    """
    import torch
    H = np.asarray(H)
    B, Nr, Nt = H.shape
    Q = int(round(np.sqrt(M)))
    N = 2 * Nt
    S = Q ** N
    if S * S > 1024:
        raise ValueError("state space too large for one evaluation per pair (%d states)" % S)
    K = all_states(N, Q)
    xf = np.broadcast_to(np.repeat(K, S, axis=0)[None], (B, S * S, N)).copy()
    xt = np.broadcast_to(np.tile(K, (S, 1))[None], (B, S * S, N)).copy()
    Hcm, yd, s2 = device_inputs(H, y, sigma2, precision)
    out = debug_eval(Hcm, yd, s2, M, torch.from_numpy(xf).cuda(), torch.from_numpy(xt).cuda(), precision=precision,
                     proposal=proposal, tau=tau, mlp_weights=mlp_weights).cpu().numpy()
    out = out.reshape(B, S, S, 4)
    P = np.exp(out[..., 0] + np.minimum(0.0, out[..., 3]))
    idx = np.arange(S)
    P[:, idx, idx] = 0.0
    P[:, idx, idx] = 1.0 - P.sum(axis=2)
    lt = out[:, 0, :, 2]                          # f(x_j)/tau - f(x_0)/tau
    lt = lt - lt.max(axis=1, keepdims=True)
    log_pi = lt - np.log(np.exp(lt).sum(axis=1, keepdims=True))
    return P, K, log_pi


def second_eigenvalue(P):
    """Second-largest eigenvalue modulus of each transition matrix (the rate of Theorem 1)."""
    P = np.asarray(P)
    single = P.ndim == 2
    P = P[None] if single else P
    out = np.empty(len(P))
    for b in range(len(P)):
        ev = np.linalg.eigvals(P[b])
        out[b] = np.sort(np.abs(ev))[-2]
    return out[0] if single else out


def tv_curve(P, log_pi, T, start=None):
    """TV distance between the chain's law after t = 0..T transitions and the target.

    start: initial distribution (default: uniform, the sampler's initialisation)."""
    P = np.asarray(P)
    S = P.shape[-1]
    p = np.full(S, 1.0 / S) if start is None else np.asarray(start, dtype=np.float64)
    pi = np.exp(log_pi)
    out = np.empty(T + 1)
    for t in range(T + 1):
        out[t] = 0.5 * np.abs(p - pi).sum()
        p = p @ P
    return out
