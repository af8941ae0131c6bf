"""Learned proposal on the GPU against the oracle (needs an MI355X).

* the network in the sampler's bf16 precision (dmala_mlp_forward, the same
  device code as inside the chain) against the oracle's rounded network;
* the training step (loss, gradient, Adam update) against the oracle's
  float64 training loss, backward and Adam;
* training rows exported by the sampler against the oracle's features;
* the device's learned kernel is reversible with respect to pi_a;
* chains of the plain/learned mixture follow the oracle's mixture chain
  (exactly with a zero output layer, and apart from near-ties otherwise).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from oracle import exact
from oracle import learned as ol
from tests.helpers import gpu_available, compare_chains

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _params(seed, scale=1.0, zero_last=False):
    P = ol.init_params(seed, zero_last=zero_last)
    if not zero_last:
        rng = np.random.default_rng(seed + 1)
        P["W3"] = rng.standard_normal(P["W3"].shape) * 0.3 * scale
        P["b3"] = rng.standard_normal(4) * 0.2 * scale
        P["b1"] = rng.standard_normal(ol.HID) * 0.1
        P["b2"] = rng.standard_normal(ol.HID) * 0.1
    return {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}


def _dev(P):
    import torch
    return torch.from_numpy(ol.flatten(P).astype(np.float32)).cuda()


def _feature_rows(R, seed):
    rng = np.random.default_rng(seed)
    X = np.empty((R, ol.N_FEAT))
    X[:, 0:4] = rng.uniform(-1.3, 1.3, (R, 4))
    X[:, 4] = rng.uniform(-1.2, 0.2, R)
    X[:, 5] = rng.uniform(-1.2, 0.2, R)
    X[:, 6] = rng.choice([0.25, 0.5, 0.75, 1.0], R)
    return X.astype(np.float32).astype(np.float64)


def test_network_forward_matches_the_oracle():
    import torch
    import paper_2407_06042_amd as dm
    P = _params(3, scale=2.0)
    for R in (1, 63, 64, 1000):          # partial and full wave groups
        X = _feature_rows(R, R)
        out = dm.mlp_forward(_dev(P), torch.from_numpy(X.astype(np.float32)).cuda()).cpu().numpy()
        ref, _ = ol.mlp_forward(P, X, rounded=True)
        err = np.abs(out - ref)
        print("mlp forward R=%d max err %.3g median %.3g" % (R, err.max(), np.median(err)), flush=True)
        # fp32 sums; an activation whose rounding flips moves an output by about one bf16 step
        assert np.median(err) < 1e-5
        assert err.max() < 5e-3
        # the unrounded network is further away: the rounding is really in the device code
        if R == 1000:
            ex, _ = ol.mlp_forward(P, X, rounded=False)
            assert np.abs(ex - ref).max() > 10 * np.median(err)


def _train_set(R, seed):
    rng = np.random.default_rng(seed)
    X = _feature_rows(R, seed)
    Q = rng.choice([4, 8], R)
    mu = rng.uniform(-1, Q[:, None], (R, 2))
    kap = np.full(R, 2.0)
    tgt = np.stack([rng.integers(0, Q), rng.integers(0, Q)], axis=-1)
    rows = np.zeros((R, 12))
    rows[:, :7] = X
    rows[:, 7:9] = mu
    rows[:, 9] = kap
    rows[:, 10] = Q
    rows = rows.astype(np.float32).astype(np.float64)
    return rows, tgt


def test_training_step_matches_the_oracle():
    import torch
    import paper_2407_06042_amd as dm
    P = _params(5, scale=3.0)
    rows, tgt = _train_set(1500, 9)     # 6 partial-sum chunks of 256 rows, the last one ragged
    w = _dev(P)
    tr = dm.MlpTrainer(w, lr=2e-3)
    rows_d = torch.from_numpy(rows.astype(np.float32)).cuda()
    tgt_d = torch.from_numpy(tgt.astype(np.int32)).cuda()
    Po = {k: v.copy() for k, v in P.items()}
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    for step in range(1, 4):
        loss = float(tr.step(rows_d, tgt_d).cpu().numpy()[0])
        g = tr.grad.cpu().numpy().astype(np.float64)
        Lo, Go = ol.training_loss(Po, rows[:, :7], rows[:, 7:9], rows[:, 9], rows[:, 10].astype(int), tgt, grad=True)
        go = ol.flatten(Go)
        print("train step %d loss gpu %.6f oracle %.6f grad err %.3g (|g| %.3g)" %
              (step, loss, Lo, np.abs(g - go).max(), np.abs(go).max()), flush=True)
        assert abs(loss - Lo) < 1e-4 * max(1.0, abs(Lo))
        assert np.abs(g - go).max() < 1e-3 * np.abs(go).max()
        ol.adam_step(Po, Go, m, v, step, 2e-3)
        wn = w.cpu().numpy().astype(np.float64)
        d = np.abs(wn - ol.flatten(Po))
        # Adam divides by |g|: components whose gradient is at rounding level may move differently
        firm = np.abs(go) > 1e-4 * np.abs(go).max()
        assert d[firm].max() < 1e-5
        assert d.max() <= 2 * 2e-3 * step


def test_training_rows_match_the_oracle_features():
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(6, 8, 64, 18.0, 5, seed=31).as_precision(np.float32)
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
    C = 20
    det = dm.Detector(5, 6, 8, 64, C, 7, 123, outputs=("final_state", "train_rows"))
    out = det(Hcm, y, s2)
    torch.cuda.synchronize()
    k = out["final_state"].cpu().numpy().astype(np.int64)
    rows = out["train_rows"].cpu().numpy()
    for i in range(5):
        prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], 64)
        mu, kap = ol.plain_index_params(prob, k[i])
        f = ol.features(prob, k[i], mu)                              # (C, Nt, 7)
        np.testing.assert_allclose(rows[i, :, :, :7], f, atol=5e-5)
        np.testing.assert_allclose(rows[i, :, :, 7], mu[:, 0::2], atol=2e-4)
        np.testing.assert_allclose(rows[i, :, :, 8], mu[:, 1::2], atol=2e-4)
        np.testing.assert_allclose(rows[i, :, :, 9], kap, rtol=1e-6)
        assert np.all(rows[i, :, :, 10] == 8) and np.all(rows[i, :, :, 11] == 0)


@pytest.mark.parametrize("nt,M", [(2, 4), (1, 16), (2, 16)])
def test_device_learned_kernel_is_reversible(nt, M):
    import torch
    import paper_2407_06042_amd as dm
    P = _params(M + nt, scale=3.0)
    b = W.make_batch(nt, 2, M, 8.0, 1, seed=17 + nt + M).as_precision(np.float32)
    prob = odm.Problem(b.H[0], b.y[0], b.sigma2[0], M)
    K = exact.all_states(prob.N, prob.Q)
    S = len(K)
    xf = np.repeat(K, S, axis=0)
    xt = np.tile(K, (S, 1))
    per = min(1024, S * S)
    rep = (S * S) // per
    Hcm, y, s2 = dm.device_inputs(np.repeat(b.H, rep, 0), np.repeat(b.y, rep, 0), np.repeat(b.sigma2, rep, 0))
    out = dm.debug_eval(Hcm, y, s2, M, torch.from_numpy(xf.reshape(rep, per, -1)).cuda(),
                        torch.from_numpy(xt.reshape(rep, per, -1)).cuda(), proposal="learned",
                        mlp_weights=_dev(P)).cpu().numpy().reshape(S * S, 4)
    LQ = out[:, 0].reshape(S, S)
    DF = out[:, 2].reshape(S, S)
    R = out[:, 3].reshape(S, S)
    Pm = np.exp(LQ + np.minimum(0.0, R))
    np.fill_diagonal(Pm, 0.0)
    Pm[np.arange(S), np.arange(S)] = 1.0 - Pm.sum(1)
    assert np.all(np.isfinite(LQ)) and np.all(np.isfinite(R))
    # fp32 log-probabilities of peaked proposals carry ~1e-6 absolute error: rows sum to 1 within that
    assert np.diag(Pm).min() > -1e-5
    lt = DF[0] - DF[0].max()
    pt = np.exp(lt) / np.exp(lt).sum()
    F = pt[:, None] * Pm
    assert np.abs(F - F.T).max() < 2e-5 * max(1.0, F.max())
    # detailed balance in the log domain, also where the flows underflow (peaked learned proposals)
    A = lt[:, None] + LQ + np.minimum(0.0, R)
    off = ~np.eye(S, dtype=bool)
    assert np.all((np.abs(A - A.T) <= 1e-5 * np.maximum(1.0, np.abs(A)))[off])
    # the device's learned proposal is the oracle's (bf16 network) up to fp32 sums and rounding flips
    _, LQo = ol.kernel_matrix(prob, K, odm.log_softmax(ol.learned_logits(prob, K, P)))
    _, LQp = ol.kernel_matrix(prob, K, odm.log_softmax(ol.plain_logits(prob, K)))
    err = np.abs(LQ - LQo)
    print("learned log q err max %.3g median %.3g; plain vs learned %.3g" %
          (err.max(), np.median(err), np.abs(LQp - LQo).max()), flush=True)
    assert np.median(err) < 1e-4
    assert err.max() < 0.05 * max(1.0, np.abs(LQo).max())
    assert np.abs(LQp - LQo).max() > 20 * np.median(err)


def _mixture_run(b, P, eps, C, T, seed, precision="fp32", tile_config=0):
    import torch
    import paper_2407_06042_amd as dm
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    det = dm.Detector(len(b.sigma2), b.nt, b.nr, b.M, C, T, seed, precision, "learned",
                      outputs=("final_state", "accept_count"), trace=True, mlp_weights=_dev(P), mix_eps=eps,
                      tile_config=tile_config)
    out = det(Hcm, y, s2)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["trace_hash"] = res["trace_hash"].view(np.uint32)
    return res


@pytest.mark.parametrize("nt,M,eps", [(4, 16, 0.5), (8, 64, 0.0), (16, 4, 0.3)])
def test_zero_output_layer_mixture_is_the_plain_chain(nt, M, eps):
    """With W3 = b3 = 0 both kernels of the mixture are the plain preconditioned kernel."""
    P = _params(1, zero_last=True)
    b = W.make_batch(nt, nt, M, 16.0, 3, seed=40 + nt).as_precision(np.float32)
    C, T, seed = 16, 25, 77
    g = _mixture_run(b, P, eps, C, T, seed)
    n_id = n_tot = 0
    for i in range(3):
        o = odm.detect(b.H[i], b.y[i], b.sigma2[i], M, C, T, seed, instance=i, trace=True, estimators=False)
        ni, nf, bad = compare_chains(g["trace_hash"][i], o, 2e-5, 2e-3)
        assert not bad, bad
        n_id += ni
        n_tot += C
    assert n_id >= 0.8 * n_tot


@pytest.mark.parametrize("nt,M,eps,tile", [(2, 16, 0.3, 0), (4, 64, 0.2, 0), (8, 16, 0.5, 0), (16, 64, 0.1, 0),
                                           (24, 16, 0.2, 0), (24, 64, 0.3, 2), (40, 64, 0.2, 0), (40, 16, 0.2, 4),
                                           (100, 64, 0.2, 0)])
def test_mixture_chains_follow_the_oracle(nt, M, eps, tile):
    """Default layouts 0, 5 (64 dims), 6 (128 dims), 4 (256 dims) and the explicit
    four-tile layouts 1 (64 dims) and 3 (128 dims, matrices from L2)."""
    P = _params(7 + nt, scale=2.0)
    b = W.make_batch(nt, nt + 2, M, 15.0, 3, seed=50 + nt).as_precision(np.float32)
    C, T, seed = 16, 20, 4242
    g = _mixture_run(b, P, eps, C, T, seed, tile_config=tile)
    n_ok = n_id = n_tot = 0
    used = 0.0
    for i in range(3):
        o = ol.mixture_sample(odm.Problem(b.H[i], b.y[i], b.sigma2[i], M), P, eps, seed, i, C, T, trace=True)
        ni, nf, bad = compare_chains(g["trace_hash"][i], o, 1e-4, 1e-2)
        n_id += ni
        n_ok += ni + nf
        n_tot += C
        used += o["trace"]["use_learned"].mean()
        clean = ~np.any((o["trace"]["cat_margin"] < 1e-4) | (o["trace"]["mh_margin"] < 1e-2), axis=0)
        same = np.all(g["final_state"][i] == o["k"], axis=1)
        np.testing.assert_array_equal(g["accept_count"][i][same], o["n_acc"][same])
    print("mixture nt=%d M=%d: %d identical, %d ok of %d; learned share %.2f" % (nt, M, n_id, n_ok, n_tot, used / 3),
          flush=True)
    # bf16 rounding flips inside the network can move a draw that is not a near-tie of the
    # float64 oracle; they are rare
    assert n_ok >= 0.9 * n_tot
    assert n_id >= 0.5 * n_tot


def test_trained_network_gains_over_the_plain_kernel():
    """Train on the method's own 32x32 64-QAM and 128x128 256-QAM chains, evaluate on 64x64 64-QAM at 20..26 dB:
    the mixture with the trained network reaches a lower symbol error rate than the plain
    kernel at the same number of transitions, and at 25 transitions a lower one than the
    plain kernel at 50."""
    import torch
    import paper_2407_06042_amd as dm
    from paper_2407_06042_amd import learned as L
    b = W.c2_snr_sweep(n_per_snr=128, seed=202).as_precision(np.float32)
    H, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
    rows, tg = L.collect(H, y, s2, 32, 32, 64, 32, [0, 5, 10, 20, 40, 80], 20, 11)
    b4 = W.c4_correlated(n_inst=48, seed=204).as_precision(np.float32)
    H4, y4, s4 = dm.device_inputs(b4.H, b4.y, b4.sigma2)
    r4, t4 = L.collect(H4, y4, s4, 128, 128, 256, 32, [0, 10, 40], 20, 12)
    rows, tg = torch.cat([rows, r4]), torch.cat([tg, t4])
    w = L.init_weights(1)
    hist = L.train(w, rows, tg, 400, batch=65536, lr=3e-3, lr_final=2e-4, log_every=50)
    print("training rows", tuple(rows.shape), "loss", hist, flush=True)
    assert hist[-1][1] < 0.5 * hist[0][1]
    ev = W.c5_learned_eval(n_per_snr=128, seed=205).as_precision(np.float32)
    He, ye, se = dm.device_inputs(ev.H, ev.y, ev.sigma2)
    B = len(ev.sigma2)

    def ser(T, prop):
        kw = dict(mlp_weights=w, mix_eps=0.1) if prop == "learned" else {}
        det = dm.Detector(B, 64, 64, 64, 32, T, 5, "bf16", prop, outputs=("symbols",), **kw)
        sym = det(He, ye, se)["symbols"].cpu().numpy()
        return float(np.mean(sym != ev.x_idx))

    p25, p50, l25 = ser(25, "precond"), ser(50, "precond"), ser(25, "learned")
    print("SER plain T=25 %.4f, plain T=50 %.4f, learned T=25 %.4f" % (p25, p50, l25), flush=True)
    assert l25 < p25 - 0.015
    assert l25 < p50
