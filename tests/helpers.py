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


def compare_chains(gpu_hash, orc, eps_cat, eps_mh):
    """Per-chain agreement of a GPU trajectory with the oracle's.

    gpu_hash: (C, T) state fingerprints after each transition.  A chain passes
    if its first disagreement is at or after its first near-tie draw (oracle
    margin below eps).  Returns (n_identical, n_flagged_diverged, bad_chains).
    """
    tr = orc["trace"]
    T, C = tr["hash"].shape
    flag = (tr["cat_margin"] < eps_cat) | (tr["mh_margin"] < eps_mh)
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
