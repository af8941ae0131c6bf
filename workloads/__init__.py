"""Seeded synthetic MIMO inputs shared by the tests, the benchmark and the oracle's callers.

This module holds input generation only (channels, transmitted symbols, noise,
SNR -> noise variance); it contains none of the detector's arithmetic and imports
neither the oracle nor the HIP library.

System model (Section II-A, eq. sys_model): complex y = H x + n with Nr receive and
Nt transmit antennas, x drawn uniformly from unit-average-energy square M-QAM,
n ~ CN(0, sigma^2) (sigma^2/2 per real element).  SNR = E||Hx||^2 / E||n||^2
(footnote to the convergence experiment in Section III-B), which with
E|h_ij|^2 = v_h and unit symbol energy gives sigma^2 = Nt * Nr * v_h / (Nr * SNR).

Channels: i.i.d. Rayleigh CN(0, v_h) (Section IV-A uses unit variance; the
benchmark configurations use v_h = 1/Nr), or the Kronecker model
H = R_r^{1/2} G R_t^{1/2} with exponential correlation R_ij = rho^|i-j|
(Section IV-D).
"""
from dataclasses import dataclass, field
import numpy as np


def qam_points(M):
    """Unit-average-energy square M-QAM points, index k_I * Q + k_Q, ascending levels."""
    Q = int(round(np.sqrt(M)))
    if Q * Q != M or Q < 2:
        raise ValueError("square QAM only")
    s = np.sqrt(3.0 / (2.0 * (M - 1)))
    lv = s * (2.0 * np.arange(Q) - Q + 1)
    return (lv[:, None] + 1j * lv[None, :]).reshape(-1)


def sigma2_from_snr_db(snr_db, nt, nr, var_h):
    snr = 10.0 ** (np.asarray(snr_db, dtype=np.float64) / 10.0)
    return nt * nr * var_h / (nr * snr)


def exp_corr(n, rho):
    i = np.arange(n)
    return rho ** np.abs(i[:, None] - i[None, :])


def psd_sqrt(R):
    w, V = np.linalg.eigh(R)
    return (V * np.sqrt(np.clip(w, 0.0, None))) @ V.T


@dataclass
class Batch:
    """A batch of independent detection problems (one per channel realisation)."""
    H: np.ndarray          # (B, Nr, Nt) complex128
    y: np.ndarray          # (B, Nr) complex128
    sigma2: np.ndarray     # (B,) float64
    x_idx: np.ndarray      # (B, Nt) int64, transmitted point indices
    M: int
    meta: dict = field(default_factory=dict)

    @property
    def nt(self):
        return self.H.shape[2]

    @property
    def nr(self):
        return self.H.shape[1]

    def as_precision(self, dtype):
        """Round H, y and sigma^2 to the precision the detector receives.

        Returns a new Batch whose float64/complex128 arrays hold exactly the
        rounded values, so that every consumer sees identical inputs.
        """
        if dtype == np.float64:
            return self
        H = self.H.astype(np.complex64).astype(np.complex128)
        y = self.y.astype(np.complex64).astype(np.complex128)
        s2 = self.sigma2.astype(np.float32).astype(np.float64)
        return Batch(H, y, s2, self.x_idx, self.M, dict(self.meta))


def make_batch(nt, nr, M, snr_db, n_inst, seed, var_h=None, rho=0.0, cfg_id=0):
    """Seeded batch: x uniform over the constellation, then H, then noise.

    snr_db: scalar or per-instance array.  var_h defaults to 1/Nr.
    rho > 0 selects the Kronecker exponential-correlation channel (both ends).
    """
    if var_h is None:
        var_h = 1.0 / nr
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(seed)]))
    pts = qam_points(M)
    snr_db = np.broadcast_to(np.asarray(snr_db, dtype=np.float64), (n_inst,)).copy()
    x_idx = rng.integers(0, M, size=(n_inst, nt))
    G = (rng.standard_normal((n_inst, nr, nt)) + 1j * rng.standard_normal((n_inst, nr, nt))) * np.sqrt(var_h / 2.0)
    if rho > 0.0:
        Rr = psd_sqrt(exp_corr(nr, rho))
        Rt = psd_sqrt(exp_corr(nt, rho))
        G = Rr[None] @ G @ Rt[None]
    sigma2 = sigma2_from_snr_db(snr_db, nt, nr, var_h)
    n = (rng.standard_normal((n_inst, nr)) + 1j * rng.standard_normal((n_inst, nr))) * np.sqrt(sigma2[:, None] / 2.0)
    x = pts[x_idx]
    y = np.einsum("bij,bj->bi", G, x) + n
    return Batch(G, y, sigma2, x_idx, M, dict(nt=nt, nr=nr, snr_db=snr_db, rho=rho, var_h=var_h))


# Named workloads with the shapes of the paper's experiments and the benchmark
# configurations.  Each returns a list of Batch objects (one per uniform shape).

def c1_small(n_inst=200, seed=1):
    """4x4 16-QAM i.i.d. Rayleigh CN(0,1/Nr) at 10 dB (small exhaustive-check case)."""
    return make_batch(4, 4, 16, 10.0, n_inst, seed, cfg_id=1)


def c2_snr_sweep(n_per_snr=1024, seed=2, snrs=(16, 18, 20, 22, 24, 26, 28)):
    """32x32 64-QAM i.i.d. Rayleigh CN(0,1/Nr), SNR 16..28 dB, n_per_snr per point."""
    snr = np.repeat(np.asarray(snrs, dtype=np.float64), n_per_snr)
    return make_batch(32, 32, 64, snr, len(snr), seed, cfg_id=2)


def c4_correlated(n_inst=256, seed=4):
    """128x128 256-QAM Kronecker rho=0.5 both ends at 30 dB."""
    return make_batch(128, 128, 256, 30.0, n_inst, seed, rho=0.5, cfg_id=4)


def c5_learned_eval(n_per_snr=2048, seed=5, snrs=(20, 22, 24, 26)):
    """64x64 64-QAM i.i.d. Rayleigh, SNR 20..26 dB."""
    snr = np.repeat(np.asarray(snrs, dtype=np.float64), n_per_snr)
    return make_batch(64, 64, 64, snr, len(snr), seed, cfg_id=5)


def c3_uneven(n_inst=4096, seed=3):
    """Uneven batch: Nt in {16,32,64,128}, Nr in {Nt,2Nt}, M in {4,16,64}, SNR U(10,30) dB.

    Returns a dict of per-instance lists in batch order: shapes (Nt, Nr, M), H
    (Nr, Nt), y, sigma2, x_idx, snr_db.  Each instance draws x, H, n from its own
    seeded stream (i.i.d. Rayleigh CN(0, 1/Nr)).
    """
    rng = np.random.default_rng(np.random.SeedSequence([3, int(seed)]))
    nts = rng.choice([16, 32, 64, 128], size=n_inst)
    nrs = nts * rng.choice([1, 2], size=n_inst)
    Ms = rng.choice([4, 16, 64], size=n_inst)
    snrs = rng.uniform(10.0, 30.0, size=n_inst)
    out = dict(shapes=[], H=[], y=[], sigma2=[], x_idx=[], snr_db=snrs)
    for i in range(n_inst):
        b = make_batch(int(nts[i]), int(nrs[i]), int(Ms[i]), snrs[i], 1, seed * 100000 + i, cfg_id=3)
        out["shapes"].append((int(nts[i]), int(nrs[i]), int(Ms[i])))
        out["H"].append(b.H[0])
        out["y"].append(b.y[0])
        out["sigma2"].append(b.sigma2[0])
        out["x_idx"].append(b.x_idx[0])
    out["sigma2"] = np.array(out["sigma2"])
    return out


def imperfect_csi(batch, nmse_db, seed=0):
    """The same problems seen through an estimated channel H_hat = H + E (Section IV-F).

    E has i.i.d. CN(0, sigma_e^2) entries with sigma_e^2 = NMSE * E|h_ij|^2, so that
    E||E||_F^2 / E||H||_F^2 = NMSE.  y, sigma^2 and the transmitted symbols are
    unchanged (y was generated with the true H, kept in meta["H_true"]).
    """
    var_h = batch.meta.get("var_h", 1.0 / batch.nr)
    s2e = 10.0 ** (nmse_db / 10.0) * var_h
    rng = np.random.default_rng(np.random.SeedSequence([6, int(seed), int(round((nmse_db + 200.0) * 100))]))
    E = (rng.standard_normal(batch.H.shape) + 1j * rng.standard_normal(batch.H.shape)) * np.sqrt(s2e / 2.0)
    meta = dict(batch.meta, H_true=batch.H, nmse_db=nmse_db)
    return Batch(batch.H + E, batch.y, batch.sigma2, batch.x_idx, batch.M, meta)
