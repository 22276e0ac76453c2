"""Autotuner for the free parameters of the method: leaf size n_L, direct-sum
threshold factor (T = factor (p+1)^3), expansion order p and the accuracy
parameter eps for a requested rms relative force error.

The paper leaves n_L and T unstated and fixes p by experiment (Sec. 6.2); the
best values depend on the machine (here the cost of M2L against the direct
sums) and on the particle distribution.  `tune` measures them on the caller's
own particles.  The rms relative force error is dominated by a few outliers
(the largest errors are 10^2-10^3 times the median), so a few thousand sample
sinks underestimate it; every candidate is therefore compared over ALL
particles with a reference evaluation: the FP64 FMM at eps = target/100 and an
order above the library's rule for that eps.  The reference itself is checked
against the exact FP64 direct sum (`fmm_direct_sinks`) on seeded sample sinks
and must be within a tenth of the target there.  For each candidate the tuner
times the full force evaluation on the GPU, keeps those whose rms over all
particles is within `margin` of the target and returns the fastest.

`BandTuner` caches one result per (N band, target, precision) so that a
serving loop or a batch of clusters of similar size reuses it.  Running the
module on the GPU tunes the benchmark workloads (on samples with seeds other
than the measured inputs') and writes the committed table tuned.json.
"""
from __future__ import annotations

import dataclasses
import math
import os
import time

import numpy as np


@dataclasses.dataclass(frozen=True)
class Candidate:
    leaf_size: int
    p2p_factor: float
    eps: float
    p: int
    centre: str = "auto"    # expansion-centre rule: "auto", "midpoint" or "enclosing"


@dataclasses.dataclass
class Result:
    best: Candidate | None
    ms: float
    rms: float
    table: list            # (Candidate, ms, rms over all particles) per candidate
    ref_rms: float = 0.0   # sampled rms of the reference against the direct sum


def candidates(target: float, leaf_sizes=(32, 40, 48, 56, 64, 72, 80, 88, 96, 128, 192),
               p2p_factors=(1.0, 1.5, 2.0, 2.5, 3.0),
               kappas=(0.6, 0.75, 0.9), order_offsets=(0, 1),
               centres=("midpoint", "enclosing")) -> list[Candidate]:
    """The search grid: eps = kappa * target, p = the library's order for eps
    plus an offset, and both expansion-centre rules (the enclosing-sphere
    centre accepts more interactions at the same eps, which changes the error
    of the worst particles as well as the cost, so the rule is tuned with the
    rest)."""
    from . import fmm
    out = []
    for centre in centres:
        for leaf in leaf_sizes:
            for pf in p2p_factors:
                for k in kappas:
                    eps = k * target
                    p0 = fmm.order_for_error(eps)
                    for d in order_offsets:
                        p = min(fmm.P_MAX, max(fmm.P_MIN, p0 + d))
                        out.append(Candidate(int(leaf), float(pf), float(eps), int(p), centre))
    return list(dict.fromkeys(out))


def select(table, target: float, margin: float):
    """Fastest candidate whose rms <= margin * target (None if none)."""
    ok = [row for row in table if row[2] <= margin * target]
    if not ok:
        return None
    return min(ok, key=lambda row: row[1])


def _sample(offsets, n: int, sinks: int, clusters: int, rng):
    """Sample sinks: (list of (lo, hi, local sink indices))."""
    if offsets is None:
        k = min(n, sinks)
        return [(0, n, np.sort(rng.choice(n, k, replace=False)))]
    off = np.asarray(offsets, dtype=np.int64)
    nonempty = [i for i in range(len(off) - 1) if off[i + 1] - off[i] >= 2]
    pick = rng.choice(len(nonempty), min(clusters, len(nonempty)), replace=False)
    per = max(1, sinks // max(1, len(pick)))
    out = []
    for j in sorted(pick):
        i = nonempty[j]
        lo, hi = int(off[i]), int(off[i + 1])
        k = min(hi - lo, per)
        out.append((lo, hi, np.sort(rng.choice(hi - lo, k, replace=False))))
    return out


def _time(run, ctx, cand, repeats: int) -> float:
    """Best wall-clock time (ms) of `repeats` synchronised calls."""
    import torch
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(repeats):
        t0 = time.perf_counter()
        run(ctx, cand.p, cand.eps)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return 1e3 * best


def _rel(a, b):
    import torch
    d = torch.linalg.norm(a - b, dim=1)
    nb = torch.linalg.norm(b, dim=1)
    keep = nb > 0          # a lone particle (a cluster of one) has no force
    return d[keep] / nb[keep]


def _run(ctx, pos, mass, offsets, p, eps):
    if offsets is None:
        return ctx.forces(pos, mass, 1.0, p, eps)[1]
    return ctx.forces_batched(offsets, pos, mass, 1.0, p, eps)[1]


def _reference(pos, mass, offsets, target, ref_factor, sinks, clusters, rng, device):
    """A tight FMM evaluation (eps = target * ref_factor, one order above the
    rule) checked against the exact GPU direct sum on sampled sinks: returns
    (accelerations, sampled rms of the reference)."""
    import torch
    from . import fmm
    ref = fmm.Context(device=device)
    eps_ref = target * ref_factor
    p_ref = min(fmm.P_MAX, fmm.order_for_error(eps_ref) + 1)
    a_ref = _run(ref, pos, mass, offsets, p_ref, eps_ref)
    errs = []
    for lo, hi, s in _sample(offsets, pos.shape[0], sinks, clusters, rng):
        idx = torch.from_numpy(s).to(pos.device)
        _, a = ref.direct_sinks(pos[lo:hi].contiguous(), mass[lo:hi].contiguous(), idx, 1.0)
        errs.append(_rel(a_ref[lo + idx], a))
    ref.close()
    e = torch.cat(errs)
    ref_rms = float(torch.sqrt(torch.mean(e * e))) if e.numel() else 0.0
    if ref_rms > 0.1 * target:
        raise RuntimeError(f"reference evaluation (p={p_ref}, eps={eps_ref:g}) has sampled rms "
                           f"{ref_rms:g}, not below target/10; the target is out of reach")
    return a_ref, ref_rms


def tune(pos, mass, target: float, *, offsets=None, precision: str = "fp64",
         grid: list[Candidate] | None = None, sinks: int = 4096, clusters: int = 16,
         repeats: int = 3, finalists: int = 4, margin: float = 0.9, ref_factor: float = 0.01,
         seed: int = 0, device: int = 0, validate=()) -> Result:
    """Measure every candidate of `grid` (default `candidates(target)`) on the
    particles (torch float64 CUDA tensors; `offsets` for a batch of clusters)
    and return the fastest one that meets the target over all particles.
    validate: further samples (pos, mass, offsets) of the same workload; the
    pick must then meet the target with the rms pooled over all particles of
    the first sample and these (the rms of one sample is carried by a few halo
    outliers and varies between samples; the pooled value is the rms of the
    workload's population)."""
    import torch
    from . import fmm
    rng = np.random.default_rng(seed)

    def run(ctx, p, eps):
        return _run(ctx, pos, mass, offsets, p, eps)

    rel = _rel
    a_ref, ref_rms = _reference(pos, mass, offsets, target, ref_factor, sinks, clusters, rng,
                                device)
    vrefs = [(v, _reference(*v, target, ref_factor, sinks, clusters, rng, device)[0])
             for v in validate]
    # pass 1: one timed call per candidate (after a call that sizes the
    # workspace and gives the error); pass 2: the `finalists` fastest that
    # qualify are timed `repeats` more times each, the minimum is kept
    table = []
    for cand in (grid if grid is not None else candidates(target)):
        ctx = fmm.Context(device=device, leaf_size=cand.leaf_size, p2p_factor=cand.p2p_factor,
                          precision=precision, centre=cand.centre)
        acc = run(ctx, cand.p, cand.eps)
        d = rel(acc, a_ref)
        rms = float(torch.sqrt(torch.mean(d * d))) if d.numel() else 0.0
        del acc, d
        table.append([cand, _time(run, ctx, cand, 1), rms])
        ctx.close()
    ok = sorted((row for row in table if row[2] <= margin * target), key=lambda row: row[1])
    for row in ok[:finalists]:
        cand = row[0]
        ctx = fmm.Context(device=device, leaf_size=cand.leaf_size, p2p_factor=cand.p2p_factor,
                          precision=precision, centre=cand.centre)
        run(ctx, cand.p, cand.eps)
        row[1] = min(row[1], _time(run, ctx, cand, repeats))
        ctx.close()
    table = [tuple(row) for row in table]
    if vrefs:
        # the qualifying candidates in order of time, until one also meets the
        # target on every validation sample
        for row in sorted((r for r in table if r[2] <= margin * target), key=lambda r: r[1]):
            cand = row[0]
            ctx = fmm.Context(device=device, leaf_size=cand.leaf_size,
                              p2p_factor=cand.p2p_factor, precision=precision, centre=cand.centre)
            ss, cnt = row[2] ** 2 * pos.shape[0], pos.shape[0]
            for (vp, vm, voff), va in vrefs:
                d = rel(_run(ctx, vp, vm, voff, cand.p, cand.eps), va)
                ss += float(torch.sum(d * d))
                cnt += d.numel()
            ctx.close()
            pooled = math.sqrt(ss / cnt)
            if pooled <= margin * target:
                return Result(cand, row[1], pooled, table, ref_rms)
        return Result(None, math.inf, math.inf, table, ref_rms)
    row = select(table, target, margin)
    if row is None:
        return Result(None, math.inf, math.inf, table, ref_rms)
    return Result(row[0], row[1], row[2], table, ref_rms)


class BandTuner:
    """One tuned candidate per (log2 N band, target, precision), measured on
    the first workload of that band and reused afterwards."""

    def __init__(self, precision: str = "fp64", **tune_kw):
        self.precision = precision
        self.kw = tune_kw
        self.cache: dict = {}

    @staticmethod
    def band(n: int) -> int:
        return int(math.floor(math.log2(max(n, 1))))

    def get(self, pos, mass, target: float, offsets=None) -> Candidate | None:
        n = pos.shape[0] if offsets is None else int(
            np.median(np.diff(np.asarray(offsets, dtype=np.int64))))
        key = (self.band(n), float(target), self.precision)
        if key not in self.cache:
            self.cache[key] = tune(pos, mass, target, offsets=offsets,
                                   precision=self.precision, **self.kw).best
        return self.cache[key]


# ---- committed table -----------------------------------------------------
# Results of `tune` for named workloads, written by running this module on the
# GPU (python -m paper_1405_2255_amd.autotune --write), read back by callers
# that want the tuned parameters without spending the tuning time.
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def table_lookup(key: str, precision: str, path: str = TABLE_PATH):
    """(Candidate, record) stored for a workload key and precision, or None."""
    import json
    try:
        rec = json.load(open(path))[key][precision]
    except (OSError, KeyError, ValueError):
        return None
    c = rec["picked"]
    return Candidate(int(c["leaf_size"]), float(c["p2p_factor"]), float(c["eps"]), int(c["p"]),
                     str(c.get("centre", "auto"))), rec


def _bench_workloads():
    """The tuning samples of the benchmark legs: the same distributions as the
    measured inputs, other seeds."""
    from . import workloads as W
    out = {}

    def plummer_1e6():
        pos, m = W.cluster("plummer", 10 ** 6, 1001)
        return pos, m, None
    plummer_1e6.validate = [1002, 1003]     # further seeds the pick must also pass
    out["plummer_1e6"] = plummer_1e6

    def batched_sample():
        sizes = W.log_uniform_sizes(512, 78, 1e3, 1e5)[::8]
        pos = np.vstack([W.cluster("plummer", int(n), 5100 + i)[0] for i, n in enumerate(sizes)])
        m = np.concatenate([np.full(int(n), 1.0 / n) for n in sizes])
        return pos, m, np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out["batched_512_plummer_1e3_1e5"] = batched_sample
    return out


def main(argv=None) -> int:
    import argparse
    import json
    import torch
    from . import workloads as W
    ap = argparse.ArgumentParser(description="tune the benchmark workloads and write the table")
    ap.add_argument("--write", default=TABLE_PATH)
    ap.add_argument("--target", type=float, default=1e-7)
    args = ap.parse_args(argv)
    table = {}
    for key, make in _bench_workloads().items():
        pos, m, off = make()
        P = torch.from_numpy(pos).cuda()
        M = torch.from_numpy(m).cuda()
        vseeds = getattr(make, "validate", [])
        val = []
        for sd in vseeds:
            vp, vm = W.cluster("plummer", len(m), sd)
            val.append((torch.from_numpy(vp).cuda(), torch.from_numpy(vm).cuda(), None))
        for prec in ("fp64", "mixed"):
            t0 = time.perf_counter()
            res = tune(P, M, args.target, offsets=off, precision=prec, validate=val)
            rec = {"picked": None if res.best is None else dataclasses.asdict(res.best),
                   "target_rms": args.target, "rms_on_sample": res.rms, "ms_on_sample": res.ms,
                   "reference_rms_vs_direct": res.ref_rms, "candidates": len(res.table),
                   "tune_s": time.perf_counter() - t0,
                   "sample": f"{key}, n={len(m)}, seeds other than the measured input's"
                             + (f"; validated on seeds {vseeds}" if vseeds else "")}
            table.setdefault(key, {})[prec] = rec
            print(key, prec, json.dumps(rec), flush=True)
    with open(args.write, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
