"""Benchmark: particle-forces/s of one full FMM force evaluation on one GPU.

Workload (default): Plummer sphere, N = 10^6 equal masses (total 1, G = 1,
scale radius 1, seeded, untruncated), FP64, criterion a (relative force error)
with the accuracy parameter chosen so that the measured rms relative force
error stays at or below 1e-7.  One step = one fmm_forces call: tree build,
low-order estimate, upward pass, walk, M2L, P2P, downward pass, output -
inputs resident in HBM before the timed region.

Prints ONE JSON line (rank 0): metric, value, ... plus
  errors        rms / percentiles of |a_fmm - a_true| / |a_true| on sampled
                sinks against the CPU oracle (exact FP64 direct sum), and
                against the GPU FP64 direct sum on all sinks
  direct        the GPU FP64 direct-summation kernel on the same input
  roofline      for the dominant kernel (algorithmic FLOP per launch / the
                launch's HIP-event duration on the library's stream)
  cpu_baseline  the CPU oracle (direct sum) on a bounded sample of sinks
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 vector peak


def m2l_flops(p: int) -> float:
    """Algorithmic FLOPs of one direct M2L (eq:M2L) in the m >= 0 half:
    (n+1)(p-n+1)^2 complex multiply-adds per output degree n, 8 FLOP each."""
    return 8.0 * sum((n + 1) * (p - n + 1) ** 2 for n in range(p + 1))


P2P_FLOPS = 20.0   # per ordered particle pair: 3 sub, 5 for r^2, rsqrt, 3 mul, 3 fma, 1 add (+ rsqrt)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--eps", type=float, default=None,
                    help="accuracy parameter epsilon (default: calibrated for rms 1e-7)")
    ap.add_argument("--p", type=int, default=-1)
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--p2p-factor", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--check-sinks", type=int, default=16384,
                    help="sinks checked against the CPU oracle (also the CPU-baseline sample)")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="omit the CPU baseline field")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2

    import torch
    import oracle
    from paper_1405_2255_amd import fmm, workloads

    target_rms = 1e-7
    eps = args.eps if args.eps is not None else 5e-8
    n = args.n
    pos_np, m_np = workloads.cluster("plummer", n, args.seed)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    mass = torch.from_numpy(m_np).to(dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    ctx = fmm.Context(device=0, leaf_size=args.leaf, p2p_factor=args.p2p_factor, timing=True)

    for _ in range(args.warmup):
        ctx.forces(pos, mass, 1.0, args.p, eps, pot, acc)
        print(f"warmup step done: {ctx.stats()['t_total']:.2f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    kstats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.forces(pos, mass, 1.0, args.p, eps, pot, acc)
        kstats.append(ctx.stats())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    st = kstats[-1]
    print(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    # accuracy of the last result: the CPU oracle on a sample of sinks (timed:
    # this is also the CPU baseline), all sinks against the GPU direct sum
    acc_np = acc.cpu().numpy()
    rng = np.random.default_rng(12345)
    sinks = np.sort(rng.choice(n, min(n, args.check_sinks), replace=False))
    cores = len(os.sched_getaffinity(0))
    t1 = time.perf_counter()
    _, a_true, _ = oracle.direct(pos_np, m_np, sinks=sinks, threads=cores)
    t_cpu = time.perf_counter() - t1
    rel = np.linalg.norm(acc_np[sinks] - a_true, axis=1) / np.linalg.norm(a_true, axis=1)
    err_oracle = oracle.error_summary(rel)
    print(f"errors vs oracle ({len(sinks)} sinks): {err_oracle}", file=sys.stderr, flush=True)

    direct = None
    err_direct = None
    if not args.no_direct:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, acc_d = ctx.direct(pos, mass, 1.0)
        torch.cuda.synchronize()
        t_direct = time.perf_counter() - t2
        ad = acc_d.cpu().numpy()
        rel_d = np.linalg.norm(acc_np - ad, axis=1) / np.linalg.norm(ad, axis=1)
        err_direct = oracle.error_summary(rel_d)
        chk = np.linalg.norm(ad[sinks] - a_true, axis=1) / np.linalg.norm(a_true, axis=1)
        direct = {"value": n / t_direct, "unit": "particle-forces/s", "ms": 1e3 * t_direct,
                  "pair_interactions_per_s": float(n) * (n - 1) / t_direct,
                  "max_rel_vs_oracle": float(chk.max())}
        print(f"gpu direct: {t_direct:.3f} s", file=sys.stderr, flush=True)

    # roofline of the dominant kernel, from the HIP events around its launch
    p = st["p"]
    m2l_ms = float(np.mean([s["t_m2l_kernel"] for s in kstats]))
    p2p_ms = float(np.mean([s["t_p2p_kernel"] for s in kstats]))
    m2l_f = st["n_m2l"] * m2l_flops(p)
    p2p_f = st["n_p2p_pairs"] * P2P_FLOPS
    if m2l_ms >= p2p_ms:
        kname, kms, kflop = "k_m2l", m2l_ms, m2l_f
    else:
        kname, kms, kflop = "k_p2p", p2p_ms, p2p_f
    achieved = kflop / (kms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": kname, "achieved": achieved,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                "launch_ms": kms, "algorithmic_flop_per_launch": kflop,
                "other": {"k_m2l": {"ms": m2l_ms, "tflops": m2l_f / (m2l_ms * 1e-3) / 1e12},
                          "k_p2p": {"ms": p2p_ms, "tflops": p2p_f / (p2p_ms * 1e-3) / 1e12}}}

    cpu = None
    if not args.no_cpu:
        cpu = {"value": len(sinks) / t_cpu, "unit": "particle-forces/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{len(sinks)} seeded random sinks of the N={n} Plummer workload "
                         f"against all {n} sources (FP64 Neumaier-compensated direct sum)",
               "seconds": t_cpu}

    phases = {k: st[k] for k in ("t_tree", "t_estimate", "t_up", "t_walk", "t_m2l", "t_down",
                                 "t_p2p", "t_total")}
    out = {
        "metric": "particle-forces/s at rms rel. force err 1e-7 vs plain FMM & direct sum; p99 lat",
        "value": n / (ms_per_step * 1e-3),
        "unit": "particle-forces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Plummer sphere N={n}, equal masses, G=1, untruncated, seed "
                               f"{args.seed}; FP64 FMM, criterion a (eq:mac:better:a), "
                               f"eps={eps:g}, p={p}",
                   "n": n, "p": p, "eps": eps, "leaf_size": args.leaf or 32,
                   "parallelism": "single GPU"},
        "errors": {"vs_oracle_sampled": err_oracle, "vs_gpu_direct_all": err_direct,
                   "target_rms": target_rms,
                   "meets_target": bool((err_direct or err_oracle)["rms"] <= target_rms)},
        "direct": direct,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases_ms": phases,
        "counts": {k: st[k] for k in ("n_cells", "n_leaves", "depth", "n_m2l", "n_p2p_lists",
                                      "n_p2p_pairs", "n_est_m2l", "n_est_p2p_pairs",
                                      "walk_iterations")},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
