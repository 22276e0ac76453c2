"""Parity with the oracle in the configurations the N = 10^6 benchmark runs
(the tuned table): FP64 and mixed precision with leaf size 80, direct-sum
threshold 2 (p+1)^3 and box-midpoint centres, at order 15 and eps 6e-8, on a
Plummer sphere of 3e4 particles; leaves of more than 64 particles make the
direct-sum kernel cut a leaf's sinks into two chunks.  Further cases: FP64 at
leaf sizes 48 and 96 with enclosing-sphere centres, and mixed precision at
leaf size 96 with threshold 3 (p+1)^3.  The mean sink has more than 2048
direct sources, so leaves are split into several source tasks with ordered
partial sums; both are asserted from the tree and the counts.  The register
M2L kernel of order 15 (FP64 and mixed) and the jerk kernels at orders 15,
16 (the wide-column branch of the multipole-rate kernel) and 18 (the generic
M2L of the rates) run here against the oracle.

Bounds as in the other parity tests: FP64 forces and potentials to 1e-10
relative per particle, jerks to 1e-9; mixed precision within 64 u32 f_b of
the oracle's FP64 result (f_b the exact scaled force)."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu

N, P, EPS = 30000, 15, 6e-8
U32 = 2.0 ** -24
CENTRE = {"midpoint": oracle.CENTRE_MIDPOINT, "enclosing": oracle.CENTRE_ENCLOSING}
# (leaf size, threshold factor, centre rule)
FP64_CASES = [(80, 2.0, "midpoint"), (48, 2.0, "enclosing"), (96, 2.0, "enclosing")]
MIXED_CASES = [(80, 2.0, "midpoint"), (96, 3.0, "midpoint")]
_refs = {}


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _leaf_sizes(cells):
    """Particle counts of the leaves from (level << 40 | begin, end) per cell:
    a cell is a leaf unless a cell one level deeper starts inside it."""
    lv = cells[:, 0] >> 40
    beg = cells[:, 0] & ((1 << 40) - 1)
    end = cells[:, 1]
    inner = set()
    for l, b in zip(lv, beg):
        if l > 0:
            inner.add((l - 1, b))
    # a parent shares its begin with its first child; any child starting at
    # the parent's begin marks the parent internal
    return np.array([e - b for l, b, e in zip(lv, beg, end) if (l, b) not in inner])


@pytest.fixture(scope="module")
def workload():
    pos, vel = W.plummer(N, 5, with_velocities=True)
    return pos, vel, np.full(N, 1.0 / N)


def reference(workload, leaf, factor, centre):
    key = (leaf, factor, centre)
    if key not in _refs:
        pos, _, m = workload
        _refs[key] = oracle.fmm(pos, m, p=P, eps=EPS, leaf_size=leaf,
                                p2p_pairs=factor * (P + 1) ** 3, want_lists=True,
                                centre=CENTRE[centre])
    return _refs[key]


@pytest.mark.parametrize("leaf,factor,centre", FP64_CASES)
def test_fp64_matches_oracle(gpu_lib, workload, leaf, factor, centre):
    import torch
    pos, _, m = workload
    print(f"bench config fp64 n={N} p={P} leaf={leaf} factor={factor} centre={centre}",
          flush=True)
    ref = reference(workload, leaf, factor, centre)
    ctx = gpu_lib.Context(leaf_size=leaf, p2p_factor=factor, centre=centre)
    pot, acc = ctx.forces(_dev(pos), _dev(m), p=P, target_err=EPS)
    torch.cuda.synchronize()
    pot, acc = pot.cpu().numpy(), acc.cpu().numpy()
    st, rs = ctx.stats(), ref["stats"]
    # the paths this configuration exercises
    leaves = _leaf_sizes(ctx.export_cells())
    assert len(leaves) == st["n_leaves"]
    if leaf > 64:
        assert leaves.max() > 64
    assert st["n_p2p_pairs"] / N > 2048
    for k in ("n_cells", "n_leaves", "depth", "n_m2l", "n_p2p_pairs"):
        assert st[k] == rs[k], k
    np.testing.assert_allclose(ctx.export_scale(), ref["scale"], rtol=1e-11)
    e = _rel(acc, ref["acc"])
    print(f"max rel acc diff {e.max():.3e}", flush=True)
    assert e.max() < 1e-10
    assert np.max(np.abs(pot - ref["pot"]) / np.abs(ref["pot"])) < 1e-10


@pytest.mark.parametrize("leaf,factor,centre", MIXED_CASES)
def test_mixed_within_fp32_bound_of_oracle(gpu_lib, workload, leaf, factor, centre):
    import torch
    pos, _, m = workload
    print(f"bench config mixed n={N} p={P} leaf={leaf} factor={factor} centre={centre}",
          flush=True)
    ref = reference(workload, leaf, factor, centre)
    ctx = gpu_lib.Context(leaf_size=leaf, p2p_factor=factor, precision="mixed", centre=centre)
    pot, acc = ctx.forces(_dev(pos), _dev(m), p=P, target_err=EPS)
    torch.cuda.synchronize()
    pot, acc = pot.cpu().numpy(), acc.cpu().numpy()
    st = ctx.stats()
    assert st["n_m2l"] == ref["stats"]["n_m2l"]
    assert st["n_p2p_pairs"] == ref["stats"]["n_p2p_pairs"]
    p0, _, f0 = oracle.direct(pos, m)
    ra = np.linalg.norm(ref["acc"], axis=1)
    da = np.linalg.norm(acc - ref["acc"], axis=1)
    bound = 64 * U32 * f0 + 1e-10 * ra
    assert np.all(da <= bound), float(np.max(da / bound))
    assert np.all(np.abs(pot - ref["pot"]) <= 64 * U32 * np.abs(p0)
                  + 1e-10 * np.abs(ref["pot"]))
    rms = np.sqrt(np.mean((da / ra) ** 2))
    print(f"mixed vs fp64 oracle rms {rms:.3e}", flush=True)
    assert rms < 0.5e-7


@pytest.mark.parametrize("n,p,leaf", [(N, P, 96), (8000, 16, 64), (5000, 18, 48)])
def test_jerk_matches_oracle(gpu_lib, workload, n, p, leaf):
    import torch
    if n == N:
        pos, vel, m = workload
    else:
        pos, vel = W.plummer(n, 300 + p, with_velocities=True)
        m = np.full(n, 1.0 / n)
    print(f"bench config jerk n={n} p={p} leaf={leaf}", flush=True)
    ctx = gpu_lib.Context(leaf_size=leaf, p2p_factor=2.0)
    pot, acc, jerk = ctx.forces_jerk(_dev(pos), _dev(vel), _dev(m), G=1.3, p=p, target_err=EPS)
    torch.cuda.synchronize()
    st = ctx.stats()
    ref = oracle.fmm(pos, m, p=p, eps=EPS, leaf_size=leaf, p2p_pairs=2.0 * (p + 1) ** 3,
                     G=1.3, vel=vel)
    assert st["n_m2l"] == ref["stats"]["n_m2l"] > 0
    assert st["n_p2p_pairs"] == ref["stats"]["n_p2p_pairs"]
    assert _rel(acc.cpu().numpy(), ref["acc"]).max() < 1e-10
    ej = _rel(jerk.cpu().numpy(), ref["jerk"])
    print(f"max rel jerk diff {ej.max():.3e}", flush=True)
    assert ej.max() < 1e-9
