"""The rotation-accelerated M2L kernel (App. A, eq:M2L:z) through the C ABI,
against the direct M2L kernel on the same interaction lists and against the
oracle's FMM (which uses the direct M2L of eq:M2L).

Tolerances: the two kernels evaluate the same expansion; they differ by
rounding only, amplified by the swap matrices (entries up to ~2e4 at degree
16): per-particle relative force difference <= 1e-12.  Against the oracle the
parity bound of the direct kernel applies (1e-10)."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

# Skipped: the first device run of this file ended in a GPU memory fault (or
# a hung queue) before any output came back, and no cause has been shown by
# reading the kernel (indices, piece bookkeeping, generated code at p = 1) or
# the order-dependent paths it exercised first (p = 1..3 had never run on the
# device before).  The library keeps the rotation kernel switched off
# (FMM_M2L_ROTATION gives FMM_E_UNSUPPORTED) until a cause is found and fixed.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="rotation M2L switched off: its first device run faulted "
                                      "and the cause is not yet found")]


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _run(ctx, pos, m, p, eps):
    import torch
    P = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    M = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    pot, acc = ctx.forces(P, M, G=1.0, p=p, target_err=eps)
    torch.cuda.synchronize()
    return pot.cpu().numpy(), acc.cpu().numpy()


@pytest.fixture(scope="module")
def ctxs(gpu_lib):
    return (gpu_lib.Context(m2l="rotation", p2p_factor=0.5),
            gpu_lib.Context(m2l="direct", p2p_factor=0.5))


@pytest.mark.parametrize("p", list(range(3, 17)))
def test_rotation_equals_direct(ctxs, p):
    """Every compiled order; a workload whose lists fill many 64-entry
    windows, with sinks whose lists span more than one window and a ragged
    last window."""
    rot, dirk = ctxs
    pos, m = W.cluster("dehnen1", 12000, 40 + p)
    print(f"p={p}", flush=True)
    pr, ar = _run(rot, pos, m, p, 1e-8)
    pd, ad = _run(dirk, pos, m, p, 1e-8)
    sr, sd = rot.stats(), dirk.stats()
    assert sr["m2l_rotation"] == 1 and sd["m2l_rotation"] == 0
    assert sr["n_m2l"] == sd["n_m2l"] and sr["n_m2l"] % 64 != 0 and sr["n_m2l"] > 64 * 50
    ids = rot.export_m2l()[:, 1]
    assert np.unique(ids, return_counts=True)[1].max() > 64      # a list over > 1 window
    assert _rel(ar, ad).max() < 1e-12
    assert (np.abs(pr - pd) / np.abs(pd)).max() < 1e-12


@pytest.mark.parametrize("p", [8, 13, 16])
def test_rotation_matches_oracle(ctxs, p):
    rot, _ = ctxs
    pos, m = W.cluster("plummer", 3000, 7 + p)
    _, acc = _run(rot, pos, m, p, 1e-7)
    ref = oracle.fmm(pos, m, p=p, eps=1e-7, leaf_size=32, p2p_pairs=0.5 * (p + 1) ** 3)
    assert rot.stats()["n_m2l"] == ref["stats"]["n_m2l"] > 0
    assert _rel(acc, ref["acc"]).max() < 1e-10


def test_rotation_tiny_inputs_and_empty_lists(ctxs):
    rot, _ = ctxs
    for n in (0, 1, 2, 3, 40):
        pos, m = W.cluster("uniform", n, 3)
        pot, acc = _run(rot, pos, m, 10, 1e-7)
        if n >= 2:
            _, ad, _ = oracle.direct(pos, m)
            assert _rel(acc, ad).max() < 1e-12     # all pairs summed directly
            assert rot.stats()["n_m2l"] == 0


def test_rotation_batched_matches_single_calls(gpu_lib):
    """Batched windows cut across cluster boundaries, so the partial sums are
    grouped differently from single calls: equal to rounding."""
    import torch
    sizes = [0, 1, 700, 4096, 2, 2500, 9000, 33]
    parts, masses = [], []
    for i, n in enumerate(sizes):
        p_, m_ = W.cluster(["plummer", "dehnen1", "uniform"][i % 3], n, 60 + i)
        parts.append(p_ + 10.0 * i)
        masses.append(m_)
    pos, m = np.vstack(parts), np.concatenate(masses)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    ctx = gpu_lib.Context(m2l="rotation", p2p_factor=0.5)
    pot, acc = ctx.forces_batched(off, P, M, G=1.0, p=12, target_err=1e-7)
    torch.cuda.synchronize()
    assert ctx.stats()["m2l_rotation"] == 1
    acc = acc.cpu().numpy()
    single = gpu_lib.Context(m2l="rotation", p2p_factor=0.5)
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        if b - a < 2:
            continue
        _, a1 = single.forces(P[a:b].contiguous(), M[a:b].contiguous(), G=1.0, p=12,
                              target_err=1e-7)
        torch.cuda.synchronize()
        assert _rel(acc[a:b], a1.cpu().numpy()).max() < 1e-13


def test_rotation_above_its_orders_is_unsupported(gpu_lib):
    import torch
    ctx = gpu_lib.Context(m2l="rotation")
    pos, m = W.cluster("plummer", 500, 1)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    with pytest.raises(gpu_lib.FMMError, match="FMM_E_UNSUPPORTED"):
        ctx.forces(P, M, G=1.0, p=17, target_err=1e-9)
