"""Training of the learned proposal's network with the library's kernels.

Data: accepted states of the method's own chains.  For a batch of problems
the plain preconditioned sampler runs from one seed to T1 transitions, which
exports one training row per (chain, antenna) at the chain's state x_T1
(network features, plain centre and precision: dmala_outputs.train_rows), and
again, from the same seed, to T1 + k transitions: the state x_{T1+k} of the
same chain is the target of those rows.  Chains that did not move in the k
transitions are left out.  The network thus learns where the plain chain goes
from a state with such features within k transitions, and proposes that jump
directly; inside the MH correction this only changes how fast the chain
moves, never its target distribution.

Training: Adam on mini-batches drawn uniformly from the rows
(dmala_mlp_train_step: forward, cross-entropy of the learned proposal at the
target levels, backward, Adam, all in the library's kernels).
"""
import numpy as np

from . import Detector, MlpTrainer, MLP_PARAMS, TRAIN_ROW

HID, N_IN, N_OUT = 64, 7, 4


def init_weights(seed=0, device="cuda"):
    """He-normal hidden layers, zero output layer (the learned kernel starts as the plain one)."""
    import torch
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((HID, N_IN)) * np.sqrt(2.0 / (N_IN + 1))
    W2 = rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID)
    flat = np.concatenate([W1.ravel(), np.zeros(HID), W2.ravel(), np.zeros(HID), np.zeros(N_OUT * HID), np.zeros(N_OUT)])
    assert flat.size == MLP_PARAMS
    return torch.from_numpy(flat.astype(np.float32)).to(device)


def collect(Hcm, y, sigma2, nt, nr, M, n_chains, feature_iters, k, seed, precision="fp32"):
    """Training rows (R, TRAIN_ROW) and targets (R, 2) on the device for one problem shape.

    Hcm, y, sigma2: device inputs as for Detector.  feature_iters: list of T1
    values (0 = the random initial states); k: transitions to the target state."""
    import torch
    B = Hcm.shape[0]
    rows, tgts = [], []
    for T1 in feature_iters:
        a = Detector(B, nt, nr, M, n_chains, T1, seed, precision, outputs=("train_rows", "final_state"))
        oa = a(Hcm, y, sigma2)
        r, k1 = oa["train_rows"].clone(), oa["final_state"].clone()
        b = Detector(B, nt, nr, M, n_chains, T1 + k, seed, precision, outputs=("final_state",))
        k2 = b(Hcm, y, sigma2)["final_state"].long()            # (B, C, 2 Nt), same chains k steps on
        moved = (k2 != k1.long()).any(-1)                        # (B, C)
        t = torch.stack([k2[..., 0::2], k2[..., 1::2]], -1).to(torch.int32)   # (B, C, Nt, 2)
        rows.append(r[moved].reshape(-1, TRAIN_ROW))
        tgts.append(t[moved].reshape(-1, 2).contiguous())
    return torch.cat(rows), torch.cat(tgts)


def train(weights, rows, targets, steps, batch=65536, lr=2e-3, seed=0, lr_final=None, log_every=0):
    """Adam steps on uniformly drawn mini-batches; returns the per-step mean losses (host floats)."""
    import torch
    R = rows.shape[0]
    g = torch.Generator(device=rows.device)
    g.manual_seed(int(seed))
    tr = MlpTrainer(weights, lr=lr)
    losses = []
    for s in range(steps):
        idx = torch.randint(0, R, (min(batch, R),), device=rows.device, generator=g)
        lr_s = lr if lr_final is None else lr * (lr_final / lr) ** (s / max(1, steps - 1))
        loss = tr.step(rows[idx].contiguous(), targets[idx].contiguous(), lr=lr_s)
        if log_every and (s % log_every == 0 or s == steps - 1):
            losses.append((s, float(loss.item())))
    return losses


def save(weights, path):
    np.save(path, weights.detach().cpu().numpy().astype(np.float32))


def load(path, device="cuda"):
    import torch
    w = np.load(path, allow_pickle=False).astype(np.float32).reshape(-1)
    if w.size != MLP_PARAMS:
        raise ValueError("expected %d parameters" % MLP_PARAMS)
    return torch.from_numpy(w).to(device)
