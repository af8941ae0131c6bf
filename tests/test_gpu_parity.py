"""Parity of the HIP detector with the float64 oracle (needs an MI355X).

Chains are compared trajectory by trajectory on the shared counter-based random
numbers: a chain must follow the oracle exactly until its first near-tie draw
(a categorical or MH decision whose oracle margin is below the stated
threshold).  Estimators are compared on identical sample lists.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dmala as odm
from oracle import exact
from tests.helpers import gpu_available, run_gpu, run_oracle, compare_chains, EPS64, EPS32 as _EPS32, eps32_mh

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# fp32 near-tie rule (thresholds derived in tests/test_gpu_near_ties.py): categorical margin, and an MH
# margin that scales with the tempered energies of the transition
EPS32 = (_EPS32[0], eps32_mh)


def _print(tag, **kv):
    print(tag, " ".join("%s=%s" % (k, v) for k, v in kv.items()), flush=True)


@pytest.mark.parametrize("proposal", ["precond", "naive"])
def test_fp64_chain_identity_small(proposal):
    """4x4 16-QAM at 10 dB, 16 chains x 50 transitions, float64: every chain identical."""
    batch = W.c1_small(n_inst=12)
    seed = 0x1234
    b, g = run_gpu(batch, 16, 50, seed, "fp64", proposal)
    for i in range(12):
        o = run_oracle(b, i, 16, 50, seed, proposal, estimators=False)
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS64)
        _print("fp64", inst=i, identical=n_id, flagged=n_fd, bad=bad[:3])
        assert not bad
        assert n_id >= 15
        same = [c for c in range(16) if np.array_equal(g["trace_hash"][i, c], o["trace"]["hash"][:, c])]
        np.testing.assert_array_equal(g["final_state"][i][same], o["k"][same])
        np.testing.assert_array_equal(g["accept_count"][i][same], o["n_acc"][same])


def test_fp64_outputs_match_oracle():
    """Hard decision, LLRs and marginals of the float64 path vs the oracle on the same chains."""
    batch = W.c1_small(n_inst=8)
    seed = 99
    b, g = run_gpu(batch, 16, 50, seed, "fp64")
    compared = 0
    for i in range(8):
        o = run_oracle(b, i, 16, 50, seed)
        if not np.array_equal(g["final_state"][i], o["k"]):
            continue
        compared += 1
        np.testing.assert_array_equal(g["symbols"][i], o["symbols"])
        np.testing.assert_allclose(g["best_energy"][i], o["best_energy"], rtol=1e-5)
        np.testing.assert_allclose(g["marginals"][i], o["marginals"], atol=1e-6)
        np.testing.assert_allclose(g["llrs"][i], o["llr"], atol=1e-4, rtol=1e-5)
        np.testing.assert_allclose(g["marginals_mc"][i], o["marginals_mc"], atol=1e-7)
    _print("fp64 outputs", compared=compared)
    assert compared >= 6


@pytest.mark.parametrize("snr", [16.0, 22.0, 28.0])
@pytest.mark.parametrize("precision,proposal", [("fp32", "precond"), ("fp32", "naive")])
def test_fp32_chain_identity_32x32(snr, precision, proposal):
    """32x32 64-QAM, 32 chains x 100 transitions: chains follow the oracle up to flagged near-ties."""
    batch = W.make_batch(32, 32, 64, snr, 4, seed=int(snr), cfg_id=2)
    seed = 0x2407060420 + int(snr)
    b, g = run_gpu(batch, 32, 100, seed, precision, proposal)
    tot_id = tot = 0
    for i in range(4):
        o = run_oracle(b, i, 32, 100, seed, proposal, estimators=False)
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS32)
        _print("fp32", snr=snr, prop=proposal, inst=i, identical=n_id, flagged=n_fd, bad=bad[:3])
        assert not bad
        tot_id += n_id
        tot += 32
    assert tot_id >= 0.75 * tot


def test_fp32_estimators_on_gpu_samples():
    """Estimator parity given identical sample lists (GPU final states fed to the oracle)."""
    batch = W.make_batch(32, 32, 64, 20.0, 3, seed=5, cfg_id=2)
    b, g = run_gpu(batch, 32, 100, 7, "fp32")
    for i in range(3):
        prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], b.M)
        k = g["final_state"][i].astype(np.int64)
        m_or = odm.marginals_is(prob, k)
        l_or = odm.llr_is(prob, k)
        np.testing.assert_allclose(g["marginals"][i], m_or, atol=1e-4)
        np.testing.assert_allclose(g["llrs"][i], l_or, atol=2e-3 * np.maximum(1.0, np.abs(l_or)).max())
        np.testing.assert_allclose(g["marginals_mc"][i], odm.marginals_mc(prob.Q, prob.Nt, k), atol=1e-6)
        # the reported hard decision is one of the chains' states and its energy is reported correctly
        sym = g["symbols"][i]
        x = np.zeros(prob.N, dtype=np.int64)
        x[0::2], x[1::2] = sym // prob.Q, sym % prob.Q
        np.testing.assert_allclose(g["best_energy"][i], prob.energy(prob.x_of(x)), rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("nt,nr,M,C,T", [(3, 5, 16, 20, 30), (1, 2, 4, 16, 40), (5, 5, 256, 16, 20), (8, 16, 64, 33, 25)])
def test_edge_shapes_fp32(nt, nr, M, C, T):
    """Odd antenna counts, Nr != Nt, QPSK and 256-QAM, chain counts off the 16-chain tile."""
    batch = W.make_batch(nt, nr, M, 15.0, 3, seed=nt * 100 + M)
    b, g = run_gpu(batch, C, T, 31337, "fp32")
    for i in range(3):
        o = run_oracle(b, i, C, T, 31337, estimators=False)
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS32)
        _print("edge", nt=nt, nr=nr, M=M, C=C, inst=i, identical=n_id, flagged=n_fd, bad=bad[:3])
        assert not bad


@pytest.mark.parametrize("alpha_mult", [0.05, 0.2, 3.0])
def test_step_size_multiplier_fp32(alpha_mult):
    """Step size alpha = alpha_mult sigma^2 (Section IV-A scales it with the noise): the index-unit
    precision is kL = 2 log2(e) / alpha_mult, so 0.2 runs the 3-level window (kL = 14.4), 0.05 a
    kernel too peaked for the window's fp32 factorisation (kL = 57.7, all levels weighted directly)
    and 3.0 a flat kernel (kL = 0.96).  Chains follow the oracle run with the same alpha."""
    batch = W.make_batch(8, 8, 64, 20.0, 3, seed=41)
    b, g = run_gpu(batch, 16, 40, 4242, "fp32", alpha_mult=alpha_mult)
    assert np.all(np.isfinite(g["best_energy"]))
    for i in range(3):
        o = run_oracle(b, i, 16, 40, 4242, estimators=False, alpha=alpha_mult * float(b.sigma2[i]))
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS32)
        _print("alpha", mult=alpha_mult, inst=i, identical=n_id, flagged=n_fd, bad=bad[:3])
        assert not bad
        assert n_id >= 12


def test_zero_iterations_gives_initial_states():
    batch = W.make_batch(6, 6, 16, 12.0, 2, seed=3)
    b, g = run_gpu(batch, 16, 0, 555, "fp32", trace=False)
    for i in range(2):
        o = run_oracle(b, i, 16, 0, 555, trace=False, estimators=False)
        np.testing.assert_array_equal(g["final_state"][i], o["k"])
        np.testing.assert_array_equal(g["accept_count"][i], 0)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "fp64"])
@pytest.mark.parametrize("nt,M", [(2, 4), (1, 16), (2, 16)])
def test_device_kernel_detailed_balance(precision, nt, M):
    """Transition matrix from the device's own q and acceptance: stochastic and reversible w.r.t. pi_a.

    The proposal values agree with the oracle to the precision of the mode.
    """
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(nt, 2, M, 8.0, 1, seed=17 + nt + M)
    b = b.as_precision(np.float64 if precision == "fp64" else np.float32)
    prob = odm.Problem(b.H[0], b.y[0], b.sigma2[0], M)
    K = exact.all_states(prob.N, prob.Q)
    S = len(K)
    xf = np.repeat(K, S, axis=0)
    xt = np.tile(K, (S, 1))
    # at most 1024 pairs per instance: replicate the problem over instances
    per = min(1024, S * S)
    rep = (S * S) // per
    Hcm, y, s2 = dm.device_inputs(np.repeat(b.H, rep, 0), np.repeat(b.y, rep, 0), np.repeat(b.sigma2, rep, 0), precision)
    out = dm.debug_eval(Hcm, y, s2, M, torch.from_numpy(xf.reshape(rep, per, -1)).cuda(),
                        torch.from_numpy(xt.reshape(rep, per, -1)).cuda(), precision=precision).cpu().numpy()
    out = out.reshape(S * S, 4)
    LQ = out[:, 0].reshape(S, S)          # log q(x_j | x_i)
    DF = out[:, 2].reshape(S, S)          # f(x_j)/tau - f(x_i)/tau as the device computes it
    R = out[:, 3].reshape(S, S)           # log acceptance ratio of i -> j
    P = np.exp(LQ + np.minimum(0.0, R))
    np.fill_diagonal(P, 0.0)
    P[np.arange(S), np.arange(S)] = 1.0 - P.sum(1)
    assert np.abs(P.sum(1) - 1).max() < 1e-9
    assert P[~np.eye(S, dtype=bool)].min() > 0 and np.diag(P).min() > 0
    # reversible with respect to the device's own tempered target exp(DF[0, j])
    lt = DF[0] - DF[0].max()
    pt = np.exp(lt) / np.exp(lt).sum()
    F = pt[:, None] * P
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert np.abs(F - F.T).max() < tol * max(1.0, F.max())
    # ... which is pi_a up to the arithmetic of the energy term, and the proposal agrees with the oracle
    pi = np.exp(exact.log_target(prob, K))
    assert exact.tv(pt, pi) < (1e-10 if precision == "fp64" else 1e-4)
    _, LQo, LAo = exact.transition_matrix(prob, K)
    qtol = {"fp64": 1e-9, "fp32": 1e-4, "bf16": 0.3, "fp16": 0.05}[precision]
    assert np.abs(LQ - LQo).max() < qtol * max(1.0, np.abs(LQo).max())
    fo = prob.f(prob.x_of(K)) / prob.tau
    ftol = 1e-9 if precision == "fp64" else 1e-4
    np.testing.assert_allclose(DF, fo[None, :] - fo[:, None], atol=ftol * max(1.0, np.abs(fo).max()))


def _proposal_centres(prob, K):
    """Continuous centres (index units) of the oracle's quadratic proposal logits, per state and dimension."""
    lg = prob.proposal_logits(prob.x_of(K))
    a = (lg[:, :, 2] - 2 * lg[:, :, 1] + lg[:, :, 0]) / 2
    return -(lg[:, :, 1] - lg[:, :, 0] - a) / (2 * a)


@pytest.mark.parametrize("M,snr,shift", [(64, 6.0, 0.0), (64, 30.0, 0.0), (64, 30.0, 8.0), (64, 30.0, -8.0),
                                         (256, 30.0, 8.0)])
def test_windowed_proposal_matches_oracle(M, snr, shift):
    """The 3-level window of the fp32 proposal (Q >= 8) with its per-mode coefficient table: log q(x'|x)
    for every state pair of a 1x2 system equals the oracle's exact discretised Gaussian.  With y moved
    along h by shift (1 + j) (a received vector far outside the constellation) the proposal centres lie
    many levels outside [0, Q): edge modes with |mode - centre| > 1/2, where the bound on the window's
    exponentials applies; a negative shift puts them below the lowest level."""
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(1, 2, M, snr, 1, seed=90 + M + int(snr)).as_precision(np.float32)
    b.y[0] = (b.y[0] + b.H[0][:, 0] * shift * (1 + 1j)).astype(b.y.dtype)
    prob = odm.Problem(b.H[0], b.y[0], b.sigma2[0], M)
    K = exact.all_states(prob.N, prob.Q)
    S = len(K)
    mu = _proposal_centres(prob, K)
    outside = float(np.mean((mu < -0.5) | (mu > prob.Q - 0.5)))
    if shift > 0:
        # most centres outside, some beyond the bound max(1/2, 12.5 / kL) = 4.33 levels (kL = 2 log2 e)
        assert outside > 0.5 and mu.max() > prob.Q - 1 + 12.5 / (2 * np.log2(np.e))
    if shift < 0:
        assert outside > 0.5 and mu.min() < -12.5 / (2 * np.log2(np.e))
    per = 1024
    rep = (S * S) // per
    xf = np.repeat(K, S, axis=0).reshape(rep, per, -1)
    xt = np.tile(K, (S, 1)).reshape(rep, per, -1)
    Hcm, y, s2 = dm.device_inputs(np.repeat(b.H, rep, 0), np.repeat(b.y, rep, 0), np.repeat(b.sigma2, rep, 0))
    out = dm.debug_eval(Hcm, y, s2, M, torch.from_numpy(xf).cuda(), torch.from_numpy(xt).cuda()).cpu().numpy()
    LQ = out.reshape(S * S, 4)[:, 0].reshape(S, S)
    _, LQo, _ = exact.transition_matrix(prob, K)
    _print("window", M=M, snr=snr, shift=shift, outside=outside, err=float(np.abs(LQ - LQo).max()),
           scale=float(np.abs(LQo).max()))
    np.testing.assert_allclose(LQ, LQo, rtol=1e-4, atol=1e-4 * max(1.0, np.abs(LQo).max()))


@pytest.mark.parametrize("nt,M,rho,snr,C,T,tile", [
    (48, 64, 0.0, 20.0, 32, 30, 0),      # 96 dims padded to 128, automatic layout
    (64, 64, 0.0, 22.0, 32, 30, 3),      # one wave per 16 chains, matrices in LDS
    (64, 64, 0.0, 22.0, 32, 30, 4),      # two waves per 16 chains, matrices from L2
    (64, 64, 0.0, 22.0, 48, 30, 8),      # the same with complex-plane matrices, three chain blocks
    (50, 16, 0.0, 18.0, 32, 30, 8),      # complex planes, 50 antennas (padding rows and K columns)
    (128, 256, 0.5, 30.0, 32, 20, 0),    # Kronecker-correlated 128x128 256-QAM, four waves per 16 chains
    (128, 256, 0.5, 30.0, 48, 20, 9),    # complex planes, four waves per 16 chains, 512-thread workgroups
    (100, 64, 0.0, 24.0, 32, 20, 9),     # complex planes, 100 antennas
    (41, 16, 0.0, 18.0, 32, 30, 0),      # 512-thread setup: 41 antennas, one single pivot, ragged register slots
    (32, 64, 0.0, 22.0, 32, 30, 10),     # complex planes in LDS, one wave per 16 chains
    (32, 64, 0.0, 22.0, 32, 30, 2),      # real-equivalent matrices in LDS, one wave per 16 chains
    (20, 16, 0.0, 18.0, 48, 30, 10),     # the same, 20 antennas (padding rows and K columns), three chain blocks
    (70, 64, 0.0, 22.0, 32, 20, 0),      # working matrix in the workspace, 70 rows over 8 threads per row
    (128, 4, 0.0, 8.0, 32, 20, 0),       # QPSK: 256 marginal rows, H read from global memory (1024 threads)
])
def test_large_shapes_fp32(nt, M, rho, snr, C, T, tile):
    """Chain identity on the large layouts; estimators on a few antennas (oracle one by one)."""
    batch = W.make_batch(nt, nt, M, snr, 2, seed=nt + M, rho=rho)
    b, g = run_gpu(batch, C, T, 4242 + tile, "fp32", tile_config=tile)
    for i in range(2):
        o = run_oracle(b, i, C, T, 4242 + tile, estimators=False)
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS32)
        _print("large", nt=nt, M=M, tile=tile, inst=i, identical=n_id, flagged=n_fd, bad=bad[:3])
        assert not bad
        assert n_id >= C // 2
        prob = odm.Problem(b.H[i], b.y[i], b.sigma2[i], M)
        k = g["final_state"][i].astype(np.int64)
        ants = [0, nt // 2, nt - 1]
        m_or = odm.marginals_is(prob, k, antennas=ants)
        l_or = odm.llr_is(prob, k, antennas=ants)
        np.testing.assert_allclose(g["marginals"][i][ants], m_or[ants], atol=1e-3)
        np.testing.assert_allclose(g["llrs"][i][ants], l_or[ants], atol=5e-3 * np.maximum(1.0, np.abs(l_or[ants])).max())


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("nt,M,tile", [(32, 64, 0), (64, 64, 0), (128, 256, 0), (64, 64, 8), (128, 256, 9), (32, 64, 10)])
def test_reduced_precision_kernel_is_reversible(precision, nt, M, tile):
    """Reduced-precision proposals keep the exact target: device log-ratios are antisymmetric
    and the energy term matches the float64 metric on random state pairs (tile 8, 9: complex-plane
    matrices)."""
    import torch
    import paper_2407_06042_amd as dm
    b = W.make_batch(nt, nt, M, 25.0, 1, seed=nt).as_precision(np.float32)
    prob = odm.Problem(b.H[0], b.y[0], b.sigma2[0], M)
    rng = np.random.default_rng(nt)
    P = 256
    xf = rng.integers(0, prob.Q, size=(1, P, prob.N))
    xt = np.where(rng.random((1, P, prob.N)) < 0.1, rng.integers(0, prob.Q, size=(1, P, prob.N)), xf)
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    fwd = dm.debug_eval(Hcm, y, s2, M, torch.from_numpy(xf).cuda(), torch.from_numpy(xt).cuda(), precision=precision,
                        tile_config=tile).cpu().numpy()[0]
    rev = dm.debug_eval(Hcm, y, s2, M, torch.from_numpy(xt).cuda(), torch.from_numpy(xf).cuda(), precision=precision,
                        tile_config=tile).cpu().numpy()[0]
    # log q(x'|x) forward == log q(x'|x) seen as the reverse term of the swapped pair
    np.testing.assert_allclose(fwd[:, 0], rev[:, 1], rtol=1e-6, atol=1e-5)
    np.testing.assert_allclose(fwd[:, 3], -rev[:, 3], rtol=1e-5, atol=1e-4)
    fo = prob.f(prob.x_of(xt[0])) / prob.tau - prob.f(prob.x_of(xf[0])) / prob.tau
    np.testing.assert_allclose(fwd[:, 2], fo, atol=2e-4 * max(1.0, np.abs(fo).max()))


def _decision_gap(o, Q):
    """Relative energy gap between the oracle's hard decision and the best visited state that differs from it
    (a near-tie of the minimum-residual choice when small)."""
    tr = o["trace"]
    E = np.concatenate([tr["init_E"][None], tr["E"]], 0)
    Hh = np.concatenate([tr["init_hash"][None], tr["hash"]], 0)
    sym = o["symbols"]
    k = np.zeros(2 * len(sym), np.int64)
    k[0::2], k[1::2] = sym // Q, sym % Q
    other = E[Hh != odm.state_hash(k)]
    return (other.min() - o["best_energy"]) / o["best_energy"] if other.size else np.inf


@pytest.mark.parametrize("snr", [16.0, 22.0, 28.0])
def test_fp32_hard_decision_matches_oracle_32x32(snr):
    """Minimum-residual hard decision (text after Algorithm 1) of the fp32 path: on every instance whose
    chains all follow the oracle, the symbols and the best energy are the oracle's (unless two distinct
    visited states are within 1e-5 relative energy)."""
    batch = W.make_batch(32, 32, 64, snr, 8, seed=100 + int(snr), cfg_id=2)
    seed = 0x4D4150 + int(snr)
    b, g = run_gpu(batch, 32, 100, seed, "fp32")
    compared = skipped_tie = 0
    for i in range(8):
        o = run_oracle(b, i, 32, 100, seed, estimators=False)
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS32)
        assert not bad
        if n_id < 32:
            continue
        if _decision_gap(o, 8) < 1e-5:
            skipped_tie += 1
            continue
        compared += 1
        np.testing.assert_array_equal(g["symbols"][i], o["symbols"])
        np.testing.assert_allclose(g["best_energy"][i], o["best_energy"], rtol=2e-5)
    _print("hard decision", snr=snr, compared=compared, near_tie=skipped_tie)
    assert compared >= 2


def test_c4_shape_chains_and_hard_decision():
    """128x128 256-QAM, Kronecker rho = 0.5 at both ends, 30 dB, 64 chains x 200 transitions (the large
    correlated workload's chain count and length) on two problems: every chain follows the oracle up to its
    first near-tie; the hard decision is the oracle's when all chains agree."""
    batch = W.c4_correlated(n_inst=2, seed=44)
    seed = 0x2407060424
    b, g = run_gpu(batch, 64, 200, seed, "fp32")
    for i in range(2):
        o = run_oracle(b, i, 64, 200, seed, estimators=False)
        n_id, n_fd, bad = compare_chains(g["trace_hash"][i], o, *EPS32)
        _print("c4 shape", inst=i, identical=n_id, flagged=n_fd, bad=bad[:3])
        assert not bad
        assert n_id >= 16
        same = [c for c in range(64) if np.array_equal(g["trace_hash"][i, c], o["trace"]["hash"][:, c])]
        np.testing.assert_array_equal(g["final_state"][i][same], o["k"][same])
        np.testing.assert_array_equal(g["accept_count"][i][same], o["n_acc"][same])
        if n_id == 64 and _decision_gap(o, 16) >= 1e-5:
            np.testing.assert_array_equal(g["symbols"][i], o["symbols"])
            np.testing.assert_allclose(g["best_energy"][i], o["best_energy"], rtol=2e-5)
