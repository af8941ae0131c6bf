#!/usr/bin/env python
"""Throughput of the DMALA detector on one MI355X.

Workload (default): 32x32 MIMO, 64-QAM (unit energy), i.i.d. Rayleigh CN(0, 1/Nr),
SNR 16..28 dB in 2 dB steps with 1024 realisations per SNR (7168 detection
problems), 32 chains x 100 MH transitions each, float32-class arithmetic,
preconditioned proposal, tau = 2.  One step = one dmala_detect call over the
whole batch (setup, sampler and estimator kernels), inputs resident in HBM.

Prints one JSON line: chain-iterations/s (value), detected vectors/s, SER per
SNR, the BF16-gradient form's throughput and SER, the sampler kernel's
roofline figures measured with HIP events around that kernel, and the float64
oracle timed on the host cores on a bounded sample of the same workload.
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
NT = NR = 32
M = 64
CHAINS, ITERS = 32, 100
SNRS = (16, 18, 20, 22, 24, 26, 28)
SEED = 0x240706042002

# MI355X published peaks
PEAK_FP32_VECTOR = 157.3e12          # published: packed fp32 FMA, 256 flop/clk/CU
# ALU roofline of the sampler: one VALU lane operation per lane per clock, non-packed
# (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz); the build disables packed fp32 and most of the
# chain's operations are not FMAs (compares, selects, exponentials, integer multiplies).
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9
PEAK_BF16_MFMA = 2.5e15


def algorithmic_ops_per_chain_iter(nt, nr, M):
    """VALU work of one chain-iteration that the method must do (per-unit figure).

    Counts: logits + CDF 6 N Q, exponentials N Q, logarithms N, Philox
    ceil((N+2)/4) blocks of 10 rounds x 6 ops, energy and MH terms 4 Nr + 2 N
    (N = 2 Nt real dimensions, Q = sqrt(M)).  The G.x contraction (8 Nt^2
    flops) runs on MFMA and is reported separately.
    """
    N, Q = 2 * nt, int(round(np.sqrt(M)))
    return 6 * N * Q + N * Q + N + 60 * ((N + 2 + 3) // 4) + 4 * nr + 2 * N


def gx_flops_per_chain_iter(nt):
    return 8 * nt * nt


def source_hash():
    h = hashlib.sha256()
    for f in ("common.hpp", "sampler_impl.hpp", "sampler_f16x2.hip"):
        with open(os.path.join(ROOT, "paper_2407_06042_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _oracle_worker(args):
    import threadpoolctl
    threadpoolctl.threadpool_limits(1)
    from oracle import dmala as odm
    H, y, s2, inst = args
    t = time.perf_counter()
    r = odm.detect(H, y, s2, M, CHAINS, ITERS, SEED, instance=inst)
    return time.perf_counter() - t, r["symbols"]


def cpu_baseline(batch, per_snr):
    """Time the float64 oracle (sampling + estimators) on a bounded sample, all host cores."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    idx = np.concatenate([np.arange(k * 1024, k * 1024 + per_snr) for k in range(len(SNRS))])
    work = [(batch.H[i], batch.y[i], batch.sigma2[i], int(i)) for i in idx]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, work, chunksize=1)
    wall = time.perf_counter() - t0
    cpu = sum(r[0] for r in res)
    n = len(idx)
    return dict(value=n * CHAINS * ITERS / wall, unit="chain-iterations/s", cores=cores, kind="oracle",
                sample="%d of the 7168 problems (%d per SNR), %d chains x %d transitions + estimators, "
                       "float64 numpy oracle, one process per core; %.1f s CPU in %.1f s wall"
                       % (n, per_snr, CHAINS, ITERS, cpu, wall),
                vectors_per_s=n / wall)


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
        if self.hip.hipEventRecord(ctypes.c_void_p(self.ev[i]), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.ev[a]), ctypes.c_void_p(self.ev[b])) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value


def run_form(dm, torch, b, precision, steps, warmup):
    Hcm, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2, precision)
    B = len(b.sigma2)
    det = dm.Detector(B, NT, NR, M, CHAINS, ITERS, SEED, precision, "precond")
    ev = HipEvents(4 * steps)
    for _ in range(warmup):
        det(Hcm, y, s2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = det(Hcm, y, s2, events=ev.ev[4 * k: 4 * k + 4])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev.elapsed_ms(4 * k, 4 * k + 3) for k in range(steps)]
    samp_ms = [ev.elapsed_ms(4 * k + 1, 4 * k + 2) for k in range(steps)]
    setup_ms = [ev.elapsed_ms(4 * k, 4 * k + 1) for k in range(steps)]
    est_ms = [ev.elapsed_ms(4 * k + 2, 4 * k + 3) for k in range(steps)]
    sym = out["symbols"].cpu().numpy()
    err = (sym != b.x_idx)
    ser = {str(s): float(err[k * 1024:(k + 1) * 1024].mean()) for k, s in enumerate(SNRS)}
    return dict(wall_ms=wall * 1e3 / steps, step_ms=float(np.mean(step_ms)), sampler_ms=float(np.mean(samp_ms)),
                setup_ms=float(np.mean(setup_ms)), estimator_ms=float(np.mean(est_ms)), ser=ser)


def learned_comparison(dm, torch, reps=3):
    """64x64 64-QAM at 20..26 dB (2048 problems per SNR), 32 chains: symbol error rate and time of
    the plain fp32 form, the BF16 form and the BF16 form with the learned proposal (mixture, eps 0.1)
    over a sweep of transitions; the network is first trained on the GPU on the method's own
    32x32 64-QAM and 128x128 256-QAM chains (training time reported separately)."""
    from paper_2407_06042_amd import learned as L
    ev0 = HipEvents(2)
    hip_t0 = time.perf_counter()
    ev0.record(0)
    b = W.c2_snr_sweep(n_per_snr=128, seed=102).as_precision(np.float32)
    H, y, s2 = dm.device_inputs(b.H, b.y, b.sigma2)
    rows, tg = L.collect(H, y, s2, 32, 32, 64, 32, [0, 5, 10, 20, 40, 80], 20, 11)
    b4 = W.c4_correlated(n_inst=48, seed=104).as_precision(np.float32)
    H4, y4, s4 = dm.device_inputs(b4.H, b4.y, b4.sigma2)
    r4, t4 = L.collect(H4, y4, s4, 128, 128, 256, 32, [0, 10, 40], 20, 12)
    rows, tg = torch.cat([rows, r4]), torch.cat([tg, t4])
    w = L.init_weights(1)
    hist = L.train(w, rows, tg, 400, batch=65536, lr=3e-3, lr_final=2e-4, log_every=399)
    ev0.record(1)
    torch.cuda.synchronize()
    train_ms = ev0.elapsed_ms(0, 1)
    ev = W.c5_learned_eval().as_precision(np.float32)
    He, ye, se = dm.device_inputs(ev.H, ev.y, ev.sigma2)
    B = len(ev.sigma2)
    runs = []
    sweep = [("fp32", "precond", (25, 50, 100, 200)), ("bf16", "precond", (25, 50, 100, 200)),
             ("bf16", "learned", (10, 25, 50, 100))]
    for prec, prop, Ts in sweep:
        for T in Ts:
            kw = dict(mlp_weights=w, mix_eps=0.1) if prop == "learned" else {}
            det = dm.Detector(B, 64, 64, 64, 32, T, SEED, prec, prop, outputs=("symbols", "accept_count"), **kw)
            det(He, ye, se)
            e = HipEvents(4 * reps)
            for k in range(reps):
                out = det(He, ye, se, events=e.ev[4 * k: 4 * k + 4])
            torch.cuda.synchronize()
            ms = float(np.mean([e.elapsed_ms(4 * k, 4 * k + 3) for k in range(reps)]))
            sym = out["symbols"].cpu().numpy()
            runs.append(dict(form=prec + ("+learned" if prop == "learned" else ""), T=T, ms=ms,
                             ser=float(np.mean(sym != ev.x_idx)),
                             accept=float(out["accept_count"].float().mean().item()) / T,
                             chain_iters_per_s=B * 32 * T / (ms * 1e-3)))
    ref = next(r for r in runs if r["form"] == "fp32" and r["T"] == 100)
    matched = {}
    for form in ("fp32", "bf16", "bf16+learned"):
        ok = [r for r in runs if r["form"] == form and r["ser"] <= ref["ser"]]
        if ok:
            best = min(ok, key=lambda r: r["ms"])
            matched[form] = dict(T=best["T"], ms=best["ms"], ser=best["ser"], speedup_vs_fp32_T100=ref["ms"] / best["ms"])
        else:
            matched[form] = None
    return dict(workload="64x64 64-QAM i.i.d. Rayleigh CN(0,1/Nr), SNR 20:2:26 dB x 2048 (8192 problems), "
                         "32 chains, swept transitions; learned = BF16 with the trained network, plain kernel "
                         "with probability 0.1 per transition",
                training=dict(ms=train_ms, rows=int(rows.shape[0]), steps=400, final_loss=hist[-1][1],
                              data="32x32 64-QAM (896 problems) and 128x128 256-QAM rho=0.5 (48 problems) "
                                   "chains, targets = the same chain 20 transitions later"),
                runs=runs, reference="fp32 plain, 100 transitions", matched_ser=matched)


def bench_uneven(args):
    """4096 uneven problems: Nt in {16,32,64,128}, Nr in {Nt,2Nt}, M in {4,16,64}, SNR U(10,30) dB,
    32 chains x 100 transitions, BF16 gradient with fp32 acceptance, one plan (graph) launch per step."""
    import torch
    import paper_2407_06042_amd as dm
    d = W.c3_uneven()
    shapes = d["shapes"]
    H, y, sig = dm.pack_uneven(d["H"], d["y"], d["sigma2"])
    C, T = 32, 100
    forms = [f for f in args.forms.split(",") if f] if args.forms != "fp32,bf16" else ["bf16", "fp32"]
    truth = np.concatenate(d["x_idx"])
    res = {}
    for f in forms:
        plan = dm.Plan(shapes, C, T, SEED, precision=f, outputs=("symbols",))
        if args.autotune:
            plan.autotune(H, y, sig, args.autotune)
        ev = HipEvents(4 * args.steps)
        for _ in range(args.warmup):
            plan(H, y, sig)
        torch.cuda.synchronize()
        for k in range(args.steps):
            out = plan(H, y, sig, events=[ev.ev[4 * k], None, None, ev.ev[4 * k + 3]])
        torch.cuda.synchronize()
        ms = float(np.mean([ev.elapsed_ms(4 * k, 4 * k + 3) for k in range(args.steps)]))
        ser = float(np.mean(out["symbols"].cpu().numpy() != truth))
        res[f] = dict(ms_per_step=ms, chain_iters_per_s=len(shapes) * C * T / (ms * 1e-3), ser=ser,
                      classes=plan.classes())
    r = res[forms[0]]
    line = {"metric": METRIC, "value": r["chain_iters_per_s"], "unit": "chain-iterations/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": forms[0], "data": "synthetic",
            "config": {"workload": "4096 uneven problems: Nt in {16,32,64,128}, Nr in {Nt,2Nt}, M in {4,16,64}, "
                                   "SNR U(10,30) dB, 32 chains x 100 transitions, one graph launch",
                       "instances": len(shapes)},
            "vectors_per_s": len(shapes) / (r["ms_per_step"] * 1e-3), "ser": r["ser"],
            "forms": {f: {k: v for k, v in res[f].items() if k != "classes"} for f in forms},
            "classes": r["classes"]}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-per-snr", type=int, default=24)
    ap.add_argument("--forms", default="fp32,bf16", help="comma list; the first is the reported value")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--workload", default="c2", choices=("c2", "uneven"),
                    help="c2: the default 32x32 64-QAM sweep; uneven: 4096 mixed-shape problems in one plan")
    ap.add_argument("--autotune", default=None, help="uneven workload: autotune cache path (JSON)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the 64x64 64-QAM plain / BF16 / learned-proposal comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the detector has no multi-GPU path to time "
              "(instances shard across GPUs with no communication); run with --gpus 1", file=sys.stderr)
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

    if args.workload == "uneven":
        return bench_uneven(args)

    batch = W.c2_snr_sweep(n_per_snr=1024).as_precision(np.float32)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, args.cpu_per_snr)   # before any GPU work in this process

    import torch
    import paper_2407_06042_amd as dm
    dm.lib()  # raises if the HIP library is not built
    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for f in forms:
        res[f] = run_form(dm, torch, batch, f, args.steps, args.warmup)

    learned = None if args.no_learned else learned_comparison(dm, torch)

    main_form = forms[0]
    r = res[main_form]
    B = len(batch.sigma2)
    ci = B * CHAINS * ITERS
    value = ci / (r["step_ms"] * 1e-3)
    ops = algorithmic_ops_per_chain_iter(NT, NR, M) * ci
    achieved = ops / (r["sampler_ms"] * 1e-3)
    traffic = None
    tf = os.path.join(ROOT, "profiles", "sampler_32x32_64qam_fp32_traffic.json")
    if os.path.exists(tf):
        t = json.load(open(tf))
        if t.get("source_hash") == source_hash():
            traffic = t.get("bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "chain-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "32x32 64-QAM i.i.d. Rayleigh CN(0,1/Nr), SNR 16:2:28 dB x 1024 realisations "
                               "(7168 problems), 32 chains x 100 transitions, preconditioned DMALA, tau=2, "
                               "fp32-class (fp16-split MFMA)", "instances": B, "chains": CHAINS, "iters": ITERS},
        "vectors_per_s": B / (r["step_ms"] * 1e-3),
        "ser": r["ser"],
        "stage_ms": {k: r[k] for k in ("setup_ms", "sampler_ms", "estimator_ms", "wall_ms")},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_OPS, "traffic": traffic,
                     "peak_definition": "non-packed VALU lane operations: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz",
                     "frac_of_packed_fp32_flop_peak": achieved / PEAK_FP32_VECTOR,
                     "kernel": "sampler_kernel<float,4,8,PM_F16X2>",
                     "gx_mfma_tflops": gx_flops_per_chain_iter(NT) * ci / (r["sampler_ms"] * 1e-3) / 1e12,
                     "ops_per_chain_iter": algorithmic_ops_per_chain_iter(NT, NR, M)},
        "cpu_baseline": cpu,
        "learned_c5": learned,
        "forms": {f: {"chain_iters_per_s": ci / (res[f]["step_ms"] * 1e-3), "ms_per_step": res[f]["step_ms"],
                      "sampler_ms": res[f]["sampler_ms"], "ser": res[f]["ser"]} for f in forms},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
