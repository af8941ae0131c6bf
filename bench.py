#!/usr/bin/env python
"""Throughput of the DMALA detector on one MI355X, at matched symbol error rate.

Headline workload (the learned-proposal evaluation configuration, where the metric's
plain / BF16 / learned comparison is defined): 64x64 MIMO, 64-QAM (unit energy), i.i.d.
Rayleigh CN(0, 1/Nr), SNR 20, 22, 24, 26 dB with 2048 realisations each (8192 detection
problems), 32 chains per problem, preconditioned DMALA, tau = 2.  `value` is the plain
fp32-class form at 100 MH transitions: one step = one dmala_detect call over the whole
batch (setup, sampler and estimator kernels), inputs resident in HBM, chain-iterations/s.

The same JSON line carries:
* matched SER: every form (fp32, BF16 gradient, BF16 + learned proposal) swept over the
  number of transitions; for each form the fastest setting whose SER is not worse than the
  fp32 form at 100 transitions within a paired 95 % confidence interval, with its detected
  vectors/s and its speed-up; the learned network is first trained on the GPU (own kernels)
  on 32x32 64-QAM and 128x128 256-QAM chains;
* the same comparison on 8x8 64-QAM at 22-26 dB, where the detector beats linear MMSE
  (the SER of an MMSE detector on the same inputs is reported beside both workloads);
* timed extra workloads: the 32x32 64-QAM SNR sweep (7168 problems, 32 x 100), the
  4096-problem uneven batch in one plan launch (32 x 100), the 128x128 256-QAM Kronecker
  system (256 problems, 64 x 200); per form: ms, stage times, chain-iterations/s, vectors/s, SER;
* roofline of the dominant kernel (the sampler of the headline step) against the VALU
  lane-operation peak, and the G.X stage alone (dmala_gx_loop) against the bf16 MFMA peak at
  the 32x32, 64x64 and 128x128 shapes;
* the float64 oracle timed on the host cores (16 worker processes, the GPU machine's CPU share,
  and one core) on a bounded sample of the headline workload.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "chain-iterations/s and detected vectors/s at matched SER (plain vs BF16/learned)"
SEED = 0x240706042005
C5_NT, C5_M, C5_C, C5_T = 64, 64, 32, 100
C5_SNRS = (20, 22, 24, 26)

# MI355X published peaks
PEAK_FP32_VECTOR = 157.3e12          # packed fp32 FMA, 256 flop/clk/CU
PEAK_BF16_MFMA = 2.5e15              # dense bf16 / fp16 matrix
# VALU lane-operation roof of the chain kernel: one non-packed lane operation per lane per clock,
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the build disables packed fp32; the chain's operations
# are mostly compares, selects, exponentials and integer multiplies, not FMAs)
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9
CPU_WORKERS = 16                     # the GPU machine's host-CPU share for one GPU


def progress(msg):
    """Phase marker on stderr (the JSON line is the only stdout output)."""
    print("[bench %.1fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def valu_ops_per_chain_iter(nt, M):
    """Algorithmic VALU lane operations of one chain-transition (per-unit work, N = 2 Nt, Q = sqrt M):
    logits and CDF 6 N Q, two exponentials per dimension (the quadratic-logit recurrence), one
    logarithm (the product of the normaliser sums), Philox ceil((N+2)/4) blocks x 10 rounds x 6,
    energy difference and MH sums 2 N.  The G.x contraction (8 Nt^2 flops) runs on MFMA."""
    N, Q = 2 * nt, int(round(np.sqrt(M)))
    return 6 * N * Q + 2 * N + 1 + 60 * ((N + 2 + 3) // 4) + 2 * N


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2407_06042_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SAMPLER_SOURCES = ("common.hpp", "sampler_impl.hpp", "mlp_device.hpp", "sampler_f16x2.hip")


# ---------------------------------------------------------------- CPU baseline (the oracle)

def _oracle_worker(args):
    import threadpoolctl
    threadpoolctl.threadpool_limits(1)
    from oracle import dmala as odm
    H, y, s2, inst = args
    t = time.perf_counter()
    odm.detect(H, y, s2, C5_M, C5_C, C5_T, SEED, instance=inst)
    return time.perf_counter() - t


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, per_snr, one_core):
    """The float64 oracle (sampling + estimators) on a bounded sample of the headline workload."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(avail, CPU_WORKERS))
    n_snr = len(C5_SNRS)
    per = len(batch.sigma2) // n_snr
    idx = np.concatenate([np.arange(k * per, k * per + per_snr) for k in range(n_snr)])
    work = [(batch.H[i], batch.y[i], batch.sigma2[i], int(i)) for i in idx]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_worker, work[:workers], chunksize=1)          # warm the workers (imports)
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, work, chunksize=1)
        wall = time.perf_counter() - t0
    cpu = float(sum(res))
    t1 = time.perf_counter()
    for w in work[:one_core]:
        _oracle_worker(w)
    wall1 = time.perf_counter() - t1
    n = len(idx)
    return dict(value=n * C5_C * C5_T / wall, unit="chain-iterations/s", cores=workers, kind="oracle",
                sample="%d of the 8192 headline problems (%d per SNR), %d chains x %d transitions + estimators, "
                       "float64 numpy oracle, one process per core; %.1f s CPU in %.1f s wall"
                       % (n, per_snr, C5_C, C5_T, cpu, wall),
                vectors_per_s=n / wall, nproc=os.cpu_count(), cpu_model=cpu_model(),
                one_core=dict(value=one_core * C5_C * C5_T / wall1, unit="chain-iterations/s",
                              sample="%d problems sequentially, %.1f s" % (one_core, wall1)))


# ---------------------------------------------------------------- timing helpers

class HipEvents:
    def __init__(self, n):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.ev = []
        for _ in range(n):
            e = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(e.value)

    def record(self, i):
        import torch
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        if self.hip.hipEventRecord(ctypes.c_void_p(self.ev[i]), s) != 0:
            raise RuntimeError("hipEventRecord failed")

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.ev[a]), ctypes.c_void_p(self.ev[b])) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value


# the estimator's outputs written in every timed step: the hard decision, the bit LLRs and the
# symbol marginals (all of them are computed whichever are requested; requesting them all makes
# the timed step store them too)
EST_OUTPUTS = ("symbols", "llrs", "marginals")


def time_detector(det, args_, steps, warmup):
    """Mean step and stage times (HIP events on the launch stream) of a Detector over `steps` calls."""
    import torch
    ev = HipEvents(4 * steps)
    for _ in range(warmup):
        det(*args_)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = det(*args_, events=ev.ev[4 * k: 4 * k + 4])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    st = lambda a, b: float(np.mean([ev.elapsed_ms(4 * k + a, 4 * k + b) for k in range(steps)]))  # noqa: E731
    return out, dict(step_ms=st(0, 3), setup_ms=st(0, 1), sampler_ms=st(1, 2), estimator_ms=st(2, 3), wall_ms=wall)


def mmse_ser(b):
    """Symbol error rate of a linear MMSE detector on the same inputs (numpy reference, not timed)."""
    pts = W.qam_points(b.M)
    H = b.H
    Hh = np.conj(np.transpose(H, (0, 2, 1)))
    A = Hh @ H + b.sigma2[:, None, None] * np.eye(b.nt)[None]
    x = np.linalg.solve(A, (Hh @ b.y[..., None]))[..., 0]
    d = np.argmin(np.abs(x[..., None] - pts[None, None, :]), axis=-1)
    return float(np.mean(d != b.x_idx))


# ---------------------------------------------------------------- the learned proposal

def train_network(dm, torch, sources, data, keep_rows=False):
    """Train the per-antenna network on the method's own chains: sources = [(batch, C, feature_iters, seed)],
    targets = the same chain 20 transitions later (learned.collect)."""
    from paper_2407_06042_amd import learned as L
    ev = HipEvents(2)
    ev.record(0)
    rows, tg = [], []
    for b, C, its, sd in sources:
        b = b.as_precision(np.float32)
        H, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
        r, t = L.collect(H, y, s2, b.nt, b.nr, b.M, C, its, 20, sd)
        rows.append(r)
        tg.append(t)
    rows, tg = torch.cat(rows), torch.cat(tg)
    w = L.init_weights(1)
    hist = L.train(w, rows, tg, 400, batch=65536, lr=3e-3, lr_final=2e-4, log_every=399)
    ev.record(1)
    torch.cuda.synchronize()
    info = dict(ms=ev.elapsed_ms(0, 1), rows=int(rows.shape[0]), steps=400, final_loss=hist[-1][1], data=data)
    if keep_rows:
        return w, info, rows, tg
    return w, info


def head_comparison(torch, rows, tg, steps=400, batch=65536, seed=5):
    """Held-out cross-entropy (nats per antenna) of three proposals on the same rows (one constellation):
    the plain preconditioned one; the learned family (4 outputs: per-axis centre offset and log2 precision
    factor, clamped to [-4, 4]); and a head with one logit per QAM point added to the plain proposal's
    (M outputs).  Same 7 -> 64 -> 64 ReLU trunk, zero-initialised output layer, Adam with the library's
    schedule (3e-3 -> 2e-4), fp32 -- a torch model of both heads, used only for this comparison."""
    g = torch.Generator(device=rows.device)
    g.manual_seed(seed)
    Q = int(rows[0, 10].item())
    perm = torch.randperm(rows.shape[0], device=rows.device, generator=g)
    n_ho = rows.shape[0] // 5
    ho, trn = perm[:n_ho], perm[n_ho:]
    j = torch.arange(Q, device=rows.device, dtype=torch.float32)

    def axis_lq(mu, kap):
        return torch.log_softmax(-kap[:, None] * (j[None, :] - mu[:, None]) ** 2, dim=-1)

    def ce(kind, net, idx):
        X, mu, kap, t = rows[idx, :7], rows[idx, 7:9], rows[idx, 9], tg[idx].long()
        if kind == "plain":
            return -(axis_lq(mu[:, 0], kap).gather(1, t[:, :1]) + axis_lq(mu[:, 1], kap).gather(1, t[:, 1:2])).mean()
        out = net(X)
        if kind == "family":
            b = out[:, 2:4].clamp(-4.0, 4.0)
            l0 = axis_lq(mu[:, 0] + out[:, 0], kap * torch.exp2(b[:, 0])).gather(1, t[:, :1])
            l1 = axis_lq(mu[:, 1] + out[:, 1], kap * torch.exp2(b[:, 1])).gather(1, t[:, 1:2])
            return -(l0 + l1).mean()
        base = (-kap[:, None] * (j[None, :] - mu[:, :1]) ** 2)[:, :, None] + \
               (-kap[:, None] * (j[None, :] - mu[:, 1:2]) ** 2)[:, None, :]
        lq = torch.log_softmax(base.reshape(-1, Q * Q) + out, dim=-1)
        return -lq.gather(1, (t[:, 0] * Q + t[:, 1])[:, None]).mean()

    res = dict(rows_train=int(trn.numel()), rows_held_out=int(n_ho), Q=Q, steps=steps, batch=batch)
    with torch.no_grad():
        res["plain_xent"] = float(ce("plain", None, ho))
    for kind, n_out in (("family", 4), ("m_logits", Q * Q)):
        torch.manual_seed(seed)
        net = torch.nn.Sequential(torch.nn.Linear(7, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64), torch.nn.ReLU(),
                                  torch.nn.Linear(64, n_out)).to(rows.device)
        torch.nn.init.zeros_(net[4].weight)
        torch.nn.init.zeros_(net[4].bias)
        opt = torch.optim.Adam(net.parameters(), lr=3e-3)
        for s_ in range(steps):
            for pg in opt.param_groups:
                pg["lr"] = 3e-3 * (2e-4 / 3e-3) ** (s_ / max(1, steps - 1))
            idx = trn[torch.randint(0, trn.numel(), (batch,), device=rows.device, generator=g)]
            loss = ce(kind, net, idx)
            opt.zero_grad()
            loss.backward()
            opt.step()
        with torch.no_grad():
            res[kind + "_xent"] = float(ce(kind, net, ho))
    res["network_macs_per_antenna"] = dict(family=7 * 64 + 64 * 64 + 64 * 4, m_logits=7 * 64 + 64 * 64 + 64 * Q * Q)
    res["draw_exponentials_per_antenna"] = dict(family=4, m_logits=Q * Q)
    return res


def matched_ser_sweep(dm, torch, b, w, sweep, ref_T, reps):
    """Time and SER of every (form, T); the matched setting per form under the paired 95 % CI rule."""
    Hc, yc, sc = dm.device_inputs(b.H, b.y, b.sigma2)
    B, nt, M = len(b.sigma2), b.nt, b.M
    runs, errs = [], {}
    for form, Ts in sweep:
        prec, prop = ("bf16", "learned") if form == "bf16+learned" else (form, "precond")
        for T in Ts:
            kw = dict(mlp_weights=w, mix_eps=0.1) if prop == "learned" else {}
            det = dm.Detector(B, nt, nt, M, C5_C, T, SEED, prec, prop, outputs=EST_OUTPUTS + ("accept_count",), **kw)
            out, tm = time_detector(det, (Hc, yc, sc), reps, 1)
            sym = out["symbols"].cpu().numpy()
            errs[(form, T)] = (sym != b.x_idx).reshape(-1).astype(np.float64)
            runs.append(dict(form=form, T=T, ms=tm["step_ms"], sampler_ms=tm["sampler_ms"],
                             ser=float(errs[(form, T)].mean()),
                             accept=float(out["accept_count"].float().mean().item()) / T,
                             chain_iters_per_s=B * C5_C * T / (tm["step_ms"] * 1e-3),
                             vectors_per_s=B / (tm["step_ms"] * 1e-3)))
    ref_err = errs[("fp32", ref_T)]
    ref = next(r for r in runs if r["form"] == "fp32" and r["T"] == ref_T)
    matched = {}
    for form, _ in sweep:
        ok = []
        for r in runs:
            if r["form"] != form:
                continue
            d = errs[(form, r["T"])] - ref_err
            hw = 1.96 * d.std(ddof=1) / np.sqrt(d.size)
            r["ser_diff_vs_ref"] = float(d.mean())
            r["ser_diff_ci95"] = float(hw)
            if d.mean() <= hw:                      # not worse than the reference within the paired CI
                ok.append(r)
        if ok:
            best = min(ok, key=lambda r: r["ms"])
            matched[form] = dict(T=best["T"], ms=best["ms"], ser=best["ser"], vectors_per_s=best["vectors_per_s"],
                                 chain_iters_per_s=best["chain_iters_per_s"], speedup_vs_fp32_ref=ref["ms"] / best["ms"])
        else:
            matched[form] = None
    return runs, matched, ref


# ---------------------------------------------------------------- extra workloads

def extra_uniform(dm, torch, b, C, T, forms, steps, warmup, snr_split=None, tile=0):
    Hc, yc, sc = dm.device_inputs(b.H, b.y, b.sigma2)
    B = len(b.sigma2)
    res = {}
    for f in forms:
        det = dm.Detector(B, b.nt, b.nr, b.M, C, T, SEED, f, "precond", outputs=EST_OUTPUTS, tile_config=tile)
        out, tm = time_detector(det, (Hc, yc, sc), steps, warmup)
        err = out["symbols"].cpu().numpy() != b.x_idx
        r = dict(tm, chain_iters_per_s=B * C * T / (tm["step_ms"] * 1e-3), vectors_per_s=B / (tm["step_ms"] * 1e-3),
                 ser=float(err.mean()))
        if snr_split:
            n = B // len(snr_split)
            r["ser_per_snr"] = {str(s): float(err[k * n:(k + 1) * n].mean()) for k, s in enumerate(snr_split)}
        res[f] = r
    return res


def extra_uneven(dm, torch, forms, steps, warmup, autotune=None):
    d = W.c3_uneven()
    shapes = d["shapes"]
    H, y, sig = dm.pack_uneven(d["H"], d["y"], d["sigma2"])
    C, T = 32, 100
    truth = np.concatenate(d["x_idx"])
    res = {}
    for f in forms:
        plan = dm.Plan(shapes, C, T, SEED, precision=f, outputs=EST_OUTPUTS)
        if autotune:
            plan.autotune(H, y, sig, autotune)
        ev = HipEvents(2 * steps)
        for _ in range(warmup):
            plan(H, y, sig)
        torch.cuda.synchronize()
        for k in range(steps):
            out = plan(H, y, sig, events=[ev.ev[2 * k], None, None, ev.ev[2 * k + 1]])
        torch.cuda.synchronize()
        ms = float(np.mean([ev.elapsed_ms(2 * k, 2 * k + 1) for k in range(steps)]))
        res[f] = dict(step_ms=ms, chain_iters_per_s=len(shapes) * C * T / (ms * 1e-3),
                      vectors_per_s=len(shapes) / (ms * 1e-3),
                      ser=float(np.mean(out["symbols"].cpu().numpy() != truth)), classes=len(plan.classes()))
    return res


def gx_stage(dm, torch, loops):
    """The G.X stage alone (dmala_gx_loop, bf16) at the 32x32, 64x64 and 128x128 shapes: fraction of the
    dense bf16 MFMA peak, counting 8 Nt^2 flops per chain and loop."""
    out = {}
    for name, b, C in (("32x32 64-QAM, 7168 problems x 32 chains", W.c2_snr_sweep(n_per_snr=1024), 32),
                       ("64x64 64-QAM, 8192 problems x 32 chains", W.c5_learned_eval(), 32),
                       ("128x128 256-QAM, 256 problems x 64 chains", W.c4_correlated(), 64)):
        b = b.as_precision(np.float32)
        Hc, yc, sc = dm.device_inputs(b.H, b.y, b.sigma2)
        B = len(b.sigma2)
        g = dm.GxLoop(B, b.nt, b.nr, b.M, C, "bf16")
        g(Hc, yc, sc, 1, run_setup=True)
        n_loops = loops
        ev = HipEvents(2)
        g(Hc, yc, sc, n_loops)
        torch.cuda.synchronize()
        ev.record(0)
        g(Hc, yc, sc, n_loops)
        ev.record(1)
        torch.cuda.synchronize()
        ms = ev.elapsed_ms(0, 1)
        flops = 8.0 * b.nt * b.nt * C * n_loops * B
        out[name] = dict(ms=ms, loops=n_loops, tflops=flops / (ms * 1e-3) / 1e12,
                         frac=flops / (ms * 1e-3) / PEAK_BF16_MFMA)
        del g
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-per-snr", type=int, default=24)
    ap.add_argument("--cpu-one-core", type=int, default=12)
    ap.add_argument("--no-extras", action="store_true", help="skip the 32x32, uneven and 128x128 workloads")
    ap.add_argument("--no-sweep", action="store_true", help="skip the matched-SER sweeps (headline form only)")
    ap.add_argument("--gx-loops", type=int, default=400)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--only", default=None, choices=("c5", "c2", "c4", "uneven", "gx"),
                    help="profiling: run one workload's timed steps only and print its timing")
    ap.add_argument("--autotune", default=None, help="uneven workload: autotune cache path (JSON)")
    ap.add_argument("--tile", type=int, default=0, help="profiling (--only): sampler layout (tile_config) to use")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: problems shard across GPUs with no communication, and this "
              "build times one GPU's share only; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=1 << 30, reps=3)))
        return

    progress("inputs")
    c5 = W.c5_learned_eval().as_precision(np.float32)
    cpu = None
    if not args.no_cpu_baseline and args.only is None:
        progress("cpu baseline")
        cpu = cpu_baseline(c5, args.cpu_per_snr, args.cpu_one_core)   # before any GPU work in this process

    import torch
    import paper_2407_06042_amd as dm
    dm.lib()  # raises if the HIP library is not built

    if args.only:
        if args.only == "c5":
            r = extra_uniform(dm, torch, c5, C5_C, C5_T, ["fp32", "bf16"], args.steps, args.warmup, tile=args.tile)
        elif args.only == "c2":
            r = extra_uniform(dm, torch, W.c2_snr_sweep().as_precision(np.float32), 32, 100, ["fp32", "bf16"],
                              args.steps, args.warmup, tile=args.tile)
        elif args.only == "c4":
            r = extra_uniform(dm, torch, W.c4_correlated().as_precision(np.float32), 64, 200,
                              ["fp32", "bf16", "fp16"], args.steps, args.warmup, tile=args.tile)
        elif args.only == "uneven":
            r = extra_uneven(dm, torch, ["bf16"], args.steps, args.warmup, args.autotune)
        else:
            r = gx_stage(dm, torch, args.gx_loops)
        print(json.dumps({"only": args.only, "result": r}))
        return

    progress("headline")
    # headline: plain fp32 form at 100 transitions
    B = len(c5.sigma2)
    Hc, yc, sc = dm.device_inputs(c5.H, c5.y, c5.sigma2)
    det = dm.Detector(B, C5_NT, C5_NT, C5_M, C5_C, C5_T, SEED, "fp32", "precond", outputs=EST_OUTPUTS)
    out, tm = time_detector(det, (Hc, yc, sc), args.steps, args.warmup)
    err = out["symbols"].cpu().numpy() != c5.x_idx
    ci = B * C5_C * C5_T
    value = ci / (tm["step_ms"] * 1e-3)
    del det

    # matched SER: the learned network, then the sweeps
    progress("training")
    w, training = train_network(
        dm, torch, [(W.c2_snr_sweep(n_per_snr=128, seed=102), 32, [0, 5, 10, 20, 40, 80], 11),
                    (W.c4_correlated(n_inst=48, seed=104), 32, [0, 10, 40], 12)],
        "32x32 64-QAM (896 problems) and 128x128 256-QAM rho=0.5 (48 problems) chains, "
        "targets = the same chain 20 transitions later")
    c5_sweep = [("fp32", (25, 50, 100, 200)), ("bf16", (25, 50, 100, 200)), ("bf16+learned", (10, 25, 50, 100))]
    matched = dict(workload="64x64 64-QAM headline batch", reference="fp32 plain, 100 transitions",
                   rule="fastest setting with SER - SER_ref <= paired 95 % half-width", mmse_ser=mmse_ser(c5))
    if not args.no_sweep:
        progress("matched-SER sweep 64x64")
        runs, m, _ = matched_ser_sweep(dm, torch, c5, w, c5_sweep, 100, 3)
        matched.update(runs=runs, matched=m)
        progress("matched-SER sweep 8x8")
        b8 = W.make_batch(8, 8, 64, np.repeat([22.0, 24.0, 26.0], 4096), 3 * 4096, seed=8, cfg_id=8).as_precision(np.float32)
        # a network trained on this size's own chains (other realisations), beside the one trained on
        # the large systems
        w8, training8, rows8, tg8 = train_network(
            dm, torch, [(W.make_batch(8, 8, 64, np.repeat([22.0, 24.0, 26.0], 1024), 3 * 1024, seed=88, cfg_id=8),
                         32, [0, 5, 10, 20, 40, 80], 13)],
            "8x8 64-QAM at 22/24/26 dB (3072 other problems) chains, targets = the same chain 20 transitions later",
            keep_rows=True)
        progress("head comparison")
        heads = head_comparison(torch, rows8, tg8)
        del rows8, tg8
        runs8, m8, ref8 = matched_ser_sweep(dm, torch, b8, w8, [("fp32", (25, 50, 100, 200)), ("bf16", (25, 50, 100)),
                                                                ("bf16+learned", (10, 25, 50, 100))], 100, 3)
        runs8x, m8x, _ = matched_ser_sweep(dm, torch, b8, w, [("fp32", (100,)), ("bf16+learned", (25, 50, 100))],
                                           100, 3)
        works = dict(workload="8x8 64-QAM i.i.d. Rayleigh CN(0,1/Nr), SNR 22/24/26 dB x 4096 (12288 problems), "
                              "32 chains", reference="fp32 plain, 100 transitions", mmse_ser=mmse_ser(b8),
                     training=training8, runs=runs8, matched=m8, head_comparison=heads,
                     large_system_network=dict(runs=[r for r in runs8x if r["form"] != "fp32"], matched=m8x))
    else:
        works = None

    extras = None
    if not args.no_extras:
        progress("extra workloads")
        extras = dict(
            c2=dict(workload="32x32 64-QAM i.i.d. Rayleigh, SNR 16:2:28 dB x 1024 (7168 problems), 32 chains x 100",
                    forms=extra_uniform(dm, torch, W.c2_snr_sweep().as_precision(np.float32), 32, 100,
                                        ["fp32", "bf16"], args.steps, args.warmup, (16, 18, 20, 22, 24, 26, 28))),
            c3_uneven=dict(workload="4096 uneven problems: Nt in {16,32,64,128}, Nr in {Nt,2Nt}, M in {4,16,64}, "
                                    "SNR U(10,30) dB, 32 chains x 100, one plan (graph) launch",
                           forms=extra_uneven(dm, torch, ["bf16", "fp32"], args.steps, args.warmup, args.autotune)),
            c4=dict(workload="128x128 256-QAM Kronecker rho=0.5 both ends, 30 dB, 256 problems, 64 chains x 200",
                    forms=extra_uniform(dm, torch, W.c4_correlated().as_precision(np.float32), 64, 200,
                                        ["fp32", "bf16", "fp16"], max(3, args.steps // 2), args.warmup)))
    progress("gradient stage")
    gx = gx_stage(dm, torch, args.gx_loops)

    ops = valu_ops_per_chain_iter(C5_NT, C5_M)
    achieved = ops * ci / (tm["sampler_ms"] * 1e-3)
    traffic = None
    tf = os.path.join(ROOT, "profiles", "sampler_64x64_64qam_fp32_traffic.json")
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("source_hash") == source_hash(SAMPLER_SOURCES):
            traffic = t.get("bytes_per_launch")
    gx5 = gx["64x64 64-QAM, 8192 problems x 32 chains"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "chain-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tm["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "64x64 64-QAM i.i.d. Rayleigh CN(0,1/Nr), SNR 20:2:26 dB x 2048 realisations "
                               "(8192 problems), 32 chains x 100 transitions, preconditioned DMALA, tau=2, "
                               "fp32-class (fp16-split MFMA); each step writes hard decisions, IS bit LLRs and "
                               "symbol marginals", "instances": B, "chains": C5_C, "iters": C5_T},
        "vectors_per_s": B / (tm["step_ms"] * 1e-3),
        "ser": {str(s): float(err[k * 2048:(k + 1) * 2048].mean()) for k, s in enumerate(C5_SNRS)},
        "stage_ms": tm,
        "matched_ser": dict(matched, training=training),
        "detector_works": works,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12,
                     "unit": "T lane-ops/s", "frac": achieved / PEAK_VALU_OPS, "traffic": traffic,
                     "peak_definition": "non-packed VALU lane operations: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz",
                     "frac_of_packed_fp32_flop_peak": achieved / PEAK_FP32_VECTOR,
                     "kernel": "sampler_kernel_w2<float, 4, 2, true, 8, PM_F16X2, false, 3, 0, true, false, "
                               "true> (two waves per 16 chains, two chain blocks per workgroup, complex-plane "
                               "matrices from L2, 3-level window, no padding dimensions)",
                     "ops_per_chain_iter": ops,
                     "gx_frac": gx5["frac"], "gx_tflops": gx5["tflops"],
                     "gx_kernel": "gx_loop_kernel<8, 1, 1, true> (dmala_gx_loop, bf16)"},
        "gx_stage": gx,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
