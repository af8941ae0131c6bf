"""Shared helpers for the GPU parity tests (oracle runs and trajectory comparison)."""
import numpy as np

from oracle import dmala as odm

PREC_NP = {"fp64": np.float64, "fp32": np.float32, "bf16": np.float32, "fp16": np.float32}


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def run_gpu(batch, n_chains, n_iters, seed, precision="fp32", proposal="precond", tau=2.0, trace=True,
            outputs=("symbols", "marginals", "llrs", "best_energy", "final_state", "accept_count", "marginals_mc"),
            **kw):
    import torch
    import paper_2407_06042_amd as dm
    b = batch.as_precision(PREC_NP[precision])
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    det = dm.Detector(len(b.sigma2), b.nt, b.nr, b.M, n_chains, n_iters, seed, precision, proposal, tau,
                      outputs=outputs, trace=trace, **kw)
    out = det(Hcm, y, s2)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("trace_hash", "trace_accept"):
        if k in res:
            res[k] = res[k].view(np.uint32)
    return b, res


def run_oracle(b, i, n_chains, n_iters, seed, proposal="precond", tau=2.0, trace=True, estimators=True, **kw):
    return odm.detect(b.H[i], b.y[i], b.sigma2[i], b.M, n_chains, n_iters, seed, instance=i,
                      variant=proposal, tau=tau, trace=trace, estimators=estimators, **kw)


# Near-tie thresholds of the chain-identity tests (oracle decision margins below which the GPU may
# decide a draw differently).  float64 path: a few ulps.  fp32 path: from the errors measured by
# tests/test_gpu_near_ties.py on real trajectories (32x32 64-QAM at 16/22/28 dB, 128x128 256-QAM
# rho 0.5 at 30 dB), kept at least EPS32_SAFETY times above the maxima:
#   categorical draws: per-dimension |log q_fp32 - log q_fp64| <= 6.0e-6 (preconditioned),
#     2.6e-5 (naive, 28 dB); an error delta in every log-probability moves each CDF value by at
#     most about delta, so margins below 1.2e-4 are near-ties;
#   MH test: |log A_fp32 - log A_fp64| <= 1.9e-7 (E + E') / (tau sigma^2) (up to 8.5e-3 in absolute
#     terms at 128x128, 30 dB), so the threshold is max(2e-3, 2^-20 (E + E') / (tau sigma^2)).
EPS64 = (1e-9, 1e-9)
EPS32 = (1.2e-4, 2e-3)
EPS32_REL = 2.0 ** -20
EPS32_SAFETY = 4.0


def eps32_mh(scale):
    """fp32 MH near-tie threshold for tempered energy scale (E + E') / (tau sigma^2)."""
    return np.maximum(EPS32[1], EPS32_REL * np.asarray(scale))


def mh_scale(orc):
    """(E + E') / (tau sigma^2) of every transition of an oracle trace, shape (T, C)."""
    tr, prob = orc["trace"], orc["problem"]
    E_before = np.concatenate([tr["init_E"][None], tr["E"][:-1]], axis=0)
    return (E_before + tr["E_prop"]) / (prob.tau * prob.sigma2)


def compare_chains(gpu_hash, orc, eps_cat, eps_mh):
    """Per-chain agreement of a GPU trajectory with the oracle's.

    gpu_hash: (C, T) state fingerprints after each transition.  A chain passes
    if its first disagreement is at or after its first near-tie draw (oracle
    margin below eps; eps_mh may be a function of the transition's tempered
    energy scale, see eps32_mh).  Returns (n_identical, n_flagged_diverged, bad_chains).
    """
    tr = orc["trace"]
    T, C = tr["hash"].shape
    emh = eps_mh(mh_scale(orc)) if callable(eps_mh) else eps_mh
    flag = (tr["cat_margin"] < eps_cat) | (tr["mh_margin"] < emh)
    n_id, n_fd, bad = 0, 0, []
    for c in range(C):
        f = np.nonzero(flag[:, c])[0]
        first_flag = f[0] if len(f) else T
        d = np.nonzero(gpu_hash[c] != tr["hash"][:, c])[0]
        first_div = d[0] if len(d) else T
        if first_div == T:
            n_id += 1
        elif first_div >= first_flag:
            n_fd += 1
        else:
            bad.append((c, int(first_div), int(first_flag), float(tr["cat_margin"][first_div, c]),
                        float(tr["mh_margin"][first_div, c])))
    return n_id, n_fd, bad
