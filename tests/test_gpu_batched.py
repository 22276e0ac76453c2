"""Batched evaluation of independent clusters in one call (one forest, every
stage one launch for all clusters) against the oracle, cluster by cluster,
and against single-cluster calls of the same library."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu


def _batch(sizes, seed):
    pos, mass = [], []
    for i, n in enumerate(sizes):
        kind = ["plummer", "dehnen1", "uniform"][i % 3]
        p, m = W.cluster(kind, int(n), seed + i)
        pos.append(p + 10.0 * i)          # clusters may overlap in space; they must not interact
        mass.append(m)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.vstack(pos), np.concatenate(mass), off


def test_batched_equals_single_calls_and_oracle(gpu_lib):
    import torch
    sizes = [0, 1, 2, 3, 700, 4096, 1, 2500, 0, 33, 12000, 65]
    pos, m, off = _batch(sizes, 100)
    # the direct M2L kernel sums each sink's list in chunks of its own, so a
    # batched call is bitwise equal to single calls (the rotation kernel's
    # windows cut across clusters: equal to rounding, tested separately)
    ctx = gpu_lib.Context(p2p_factor=0.5, m2l="direct")
    P = torch.from_numpy(pos).cuda()
    M = torch.from_numpy(m).cuda()
    pot, acc = ctx.forces_batched(off, P, M, G=1.0, p=8, target_err=1e-7)
    torch.cuda.synchronize()
    pot, acc = pot.cpu().numpy(), acc.cpu().numpy()
    single = gpu_lib.Context(p2p_factor=0.5, m2l="direct")
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        if b == a:
            continue
        print(f"cluster {k} n={b - a}", flush=True)
        ps, as_ = single.forces(P[a:b].contiguous(), M[a:b].contiguous(), G=1.0, p=8,
                                target_err=1e-7)
        torch.cuda.synchronize()
        # the same tree, lists and summation order: bitwise equal
        assert np.array_equal(ps.cpu().numpy(), pot[a:b])
        assert np.array_equal(as_.cpu().numpy(), acc[a:b])
        if b - a >= 2:
            ref = oracle.fmm(pos[a:b], m[a:b], p=8, eps=1e-7, leaf_size=32,
                             p2p_pairs=0.5 * 9 ** 3)
            d = np.linalg.norm(acc[a:b] - ref["acc"], axis=1) / np.linalg.norm(ref["acc"], axis=1)
            assert d.max() < 1e-10
        else:
            assert pot[a] == 0.0 and np.all(acc[a] == 0.0)


def test_batched_many_small_clusters_accuracy(gpu_lib):
    """512 clusters with N log-uniform in [10, 3000]: every cluster within the
    error bound against its own exact direct sum."""
    import torch
    sizes = W.log_uniform_sizes(512, 7, 10, 3000)
    pos, m, off = _batch(sizes, 500)
    ctx = gpu_lib.Context()
    P = torch.from_numpy(pos).cuda()
    M = torch.from_numpy(m).cuda()
    eps = 1e-7
    _, acc = ctx.forces_batched(off, P, M, G=1.0, p=-1, target_err=eps)
    torch.cuda.synchronize()
    acc = acc.cpu().numpy()
    errs = []
    for k in range(0, 512, 8):              # a subsample of clusters, all their sinks
        a, b = off[k], off[k + 1]
        _, a0, _ = oracle.direct(pos[a:b], m[a:b])
        errs.append(np.linalg.norm(acc[a:b] - a0, axis=1) / np.linalg.norm(a0, axis=1))
    e = oracle.error_summary(np.concatenate(errs))
    print("batched error", e, ctx.stats(), flush=True)
    assert e["rms"] < 2 * eps


def test_batched_bad_offsets(gpu_lib):
    import torch
    ctx = gpu_lib.Context()
    P = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    M = torch.ones(10, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.forces_batched([0, 4, 9], P, M)
    with pytest.raises(gpu_lib.FMMError) as e:
        ctx.forces_batched([0, 6, 4, 10], P, M)
    assert e.value.status == gpu_lib.E_INVAL


def test_batched_deep_and_shallow_clusters_equal_single_calls(gpu_lib):
    """Clusters that need the second key word (a far outlier squeezes them
    into a few level-21 cells) next to clusters that do not: each cluster's
    result is bitwise the single call's, and the deep ones match the oracle."""
    import torch
    parts, masses = [], []
    for i, (n, far) in enumerate([(3000, True), (2500, False), (4000, True), (700, False)]):
        p, m = W.cluster("plummer", n, 40 + i)
        if far:
            p = np.vstack([p, [[-1e7, 5.0, 1.0]]])
            m = np.append(m, m[0])
        parts.append(p)
        masses.append(m)
    sizes = [len(m) for m in masses]
    pos, m = np.vstack(parts), np.concatenate(masses)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P = torch.from_numpy(pos).cuda()
    M = torch.from_numpy(m).cuda()
    ctx = gpu_lib.Context(p2p_factor=0.5, m2l="direct")
    pot, acc = ctx.forces_batched(off, P, M, G=1.0, p=8, target_err=1e-7)
    torch.cuda.synchronize()
    assert ctx.stats()["depth"] > 21
    pot, acc = pot.cpu().numpy(), acc.cpu().numpy()
    single = gpu_lib.Context(p2p_factor=0.5, m2l="direct")
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        print(f"cluster {k} n={b - a}", flush=True)
        ps, as_ = single.forces(P[a:b].contiguous(), M[a:b].contiguous(), G=1.0, p=8,
                                target_err=1e-7)
        torch.cuda.synchronize()
        assert np.array_equal(ps.cpu().numpy(), pot[a:b])
        assert np.array_equal(as_.cpu().numpy(), acc[a:b])
        ref = oracle.fmm(pos[a:b], m[a:b], p=8, eps=1e-7, leaf_size=32, p2p_pairs=0.5 * 9 ** 3)
        assert ref["stats"]["depth"] == single.stats()["depth"]
        d = np.linalg.norm(acc[a:b] - ref["acc"], axis=1) / np.linalg.norm(ref["acc"], axis=1)
        assert d.max() < 1e-10
