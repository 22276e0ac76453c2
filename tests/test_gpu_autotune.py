"""The autotuner on the GPU: it measures every candidate, the one it returns
is the fastest that met the target against its reference evaluation, and that
choice also meets the target over every particle against the exact GPU
direct sum."""
import numpy as np
import pytest

from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rms(a, b):
    d = np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)
    return float(np.sqrt(np.mean(d ** 2)))


def test_tune_single_cluster(gpu_lib):
    import torch
    from paper_1405_2255_amd import autotune as A
    pos, m = W.cluster("plummer", 200_000, 11)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    target = 1e-6
    grid = A.candidates(target, leaf_sizes=(24, 48), p2p_factors=(1.0, 2.0), kappas=(0.8,),
                        order_offsets=(0, 1))
    print(f"tuning {len(grid)} candidates", flush=True)
    res = A.tune(P, M, target, grid=grid, sinks=2048, repeats=1)
    assert len(res.table) == len(grid)
    assert all(np.isfinite(ms) and ms > 0 and np.isfinite(r) for _, ms, r in res.table)
    assert res.best is not None and res.rms <= 0.9 * target
    assert res.ref_rms <= 0.1 * target
    ok = [row for row in res.table if row[2] <= 0.9 * target]
    assert res.ms == min(row[1] for row in ok)
    b = res.best
    ctx = gpu_lib.Context(leaf_size=b.leaf_size, p2p_factor=b.p2p_factor, centre=b.centre)
    _, acc = ctx.forces(P, M, 1.0, b.p, b.eps)
    _, ad = ctx.direct(P, M, 1.0)
    torch.cuda.synchronize()
    assert _rms(acc.cpu().numpy(), ad.cpu().numpy()) <= target


def test_tune_batched_and_band_cache(gpu_lib):
    import torch
    from paper_1405_2255_amd import autotune as A
    sizes = W.log_uniform_sizes(24, 5, 1e3, 3e4)
    pos = np.vstack([W.cluster("plummer", int(n), 40 + i)[0] for i, n in enumerate(sizes)])
    m = np.concatenate([np.full(int(n), 1.0 / n) for n in sizes])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    target = 1e-7
    grid = A.candidates(target, leaf_sizes=(32,), p2p_factors=(1.0, 2.0), kappas=(0.6, 0.8),
                        order_offsets=(0,))
    bt = A.BandTuner(precision="mixed", grid=grid, sinks=2048, clusters=8, repeats=1)
    print("tuning batched (mixed)", flush=True)
    best = bt.get(P, M, target, offsets=off)
    assert best is not None and len(bt.cache) == 1
    assert bt.get(P, M, target, offsets=off) is best
    ctx = gpu_lib.Context(leaf_size=best.leaf_size, p2p_factor=best.p2p_factor, precision="mixed")
    _, acc = ctx.forces_batched(off, P, M, 1.0, best.p, best.eps)
    torch.cuda.synchronize()
    acc = acc.cpu().numpy()
    got, want = [], []
    for i in range(0, 24, 4):
        a, b = int(off[i]), int(off[i + 1])
        _, ad = ctx.direct(P[a:b].contiguous(), M[a:b].contiguous(), 1.0)
        got.append(acc[a:b])
        want.append(ad.cpu().numpy())
    assert _rms(np.vstack(got), np.vstack(want)) <= target


def test_tune_reports_no_candidate_below_the_fp32_floor(gpu_lib):
    """Mixed precision cannot reach rms 1e-9 (its floor is a few 1e-8): no
    candidate qualifies although the FP64 reference does."""
    import torch
    from paper_1405_2255_amd import autotune as A
    pos, m = W.cluster("uniform", 20_000, 2)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    grid = [A.Candidate(32, 2.0, 1e-9, 16)]
    res = A.tune(P, M, 1e-9, grid=grid, precision="mixed", sinks=512, repeats=1)
    assert res.best is None and len(res.table) == 1 and res.table[0][2] > 1e-9
    assert res.ref_rms <= 1e-10


def test_tune_refuses_a_target_beyond_fp64(gpu_lib):
    import torch
    from paper_1405_2255_amd import autotune as A
    pos, m = W.cluster("plummer", 20_000, 3)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    with pytest.raises(RuntimeError, match="out of reach"):
        A.tune(P, M, 1e-16, grid=[A.Candidate(32, 2.0, 1e-16, 20)], sinks=256, repeats=1)
