"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (FP64 everywhere):
  * direct sums: the GPU and the oracle add the same terms in different
    orders, so per-particle relative differences stay at a few ulp times
    sqrt(number of terms): bound 1e-12.
  * FMM vs the oracle's FMM with identical parameters: the tree, centres and
    radii are bitwise equal by construction, the interaction lists equal; the
    far-field sums differ only by rounding order.  Bound: relative force
    difference <= 1e-10 for every particle (the expansions are summed to
    about 1e-16 of terms that are at most ~1/eps larger than the result).
    An acceptance decision that flips on a last-bit difference of the
    multipole power or sink scale would change one particle by at most a few
    eps; the lists are compared, so such a flip would be reported.
  * FMM vs the exact direct sum: the paper's own statement for criterion a -
    rms of delta a / a about eps or below, 99.9th percentile within ~10x.
"""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu


def _to_dev(pos, m):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(pos)).cuda(),
            torch.from_numpy(np.ascontiguousarray(m)).cuda())


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context(timing=True)


def _gpu_fmm(ctx, pos, m, p, eps, G=1.0):
    import torch
    P, M = _to_dev(pos, m)
    pot, acc = ctx.forces(P, M, G=G, p=p, target_err=eps)
    torch.cuda.synchronize()
    return pot.cpu().numpy(), acc.cpu().numpy()


def _merged(entries):
    """(sink id, first, end) entries -> per-sink maximal particle ranges."""
    e = np.asarray(entries, dtype=np.int64).reshape(-1, 3)
    e = e[np.lexsort((e[:, 1], e[:, 0]))]
    out = []
    for sink, a, b in e:
        if out and out[-1][0] == sink and out[-1][2] == a:
            out[-1][2] = b
        else:
            out.append([sink, a, b])
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def _ids_sorted(a):
    a = np.asarray(a)
    if a.size == 0:
        return a.reshape(0, 2)
    return a[np.lexsort((a[:, 0], a[:, 1]))]


@pytest.mark.parametrize("n", [1000, 4096])
def test_direct_sum_matches_oracle(ctx, n):
    import torch
    pos, m = W.cluster("plummer", n, 3, masses="salpeter")
    P, M = _to_dev(pos, m)
    pot, acc = ctx.direct(P, M, G=1.7)
    torch.cuda.synchronize()
    p0, a0, _ = oracle.direct(pos, m, G=1.7)
    assert np.max(np.abs(pot.cpu().numpy() - p0) / np.abs(p0)) < 1e-12
    assert _rel(acc.cpu().numpy(), a0).max() < 1e-12


def _input(kind, n, masses, seed=5):
    """W.cluster, or with '+far': n - 1 particles of the profile and one more
    1e7 away, which squeezes the cluster into a few level-21 cells (the tree
    then refines them with the second key word)."""
    if kind.endswith("+far"):
        pos, m = W.cluster(kind[:-4], n - 1, seed, masses=masses)
        pos = np.vstack([pos, [[1e7, -3.0, 2.0]]])
        m = np.append(m, m.mean())
        return np.ascontiguousarray(pos), np.ascontiguousarray(m)
    return W.cluster(kind, n, seed, masses=masses)


CASES = [
    # (kind, n, masses, p, eps, leaf) - the small paper workload first
    ("plummer", 4096, "equal", 8, 1e-7, 32),
    ("plummer+far", 6001, "equal", 8, 1e-7, 32),
    ("dehnen1.5+far", 9001, "salpeter", 6, 1e-6, 16),
    ("plummer", 20011, "equal", 10, 1e-7, 32),
    ("dehnen1.5", 12345, "salpeter", 6, 1e-5, 16),
    ("uniform", 7777, "equal", 12, 1e-8, 24),
    ("dehnen0", 9000, "equal", 4, 1e-4, 8),
]


@pytest.mark.parametrize("kind,n,masses,p,eps,leaf", CASES)
def test_fmm_matches_oracle_fmm(gpu_lib, kind, n, masses, p, eps, leaf):
    print(f"case {kind} n={n} p={p} eps={eps} leaf={leaf}", flush=True)
    ctx = gpu_lib.Context(leaf_size=leaf, p2p_factor=0.5)
    pos, m = _input(kind, n, masses)
    pot, acc = _gpu_fmm(ctx, pos, m, p, eps)
    st = ctx.stats()
    ref = oracle.fmm(pos, m, p=p, eps=eps, leaf_size=leaf, p2p_pairs=0.5 * (p + 1) ** 3,
                     want_lists=True)
    # identical tree and identical interaction lists
    assert st["n_cells"] == ref["stats"]["n_cells"]
    assert st["n_leaves"] == ref["stats"]["n_leaves"]
    assert st["depth"] == ref["stats"]["depth"]
    np.testing.assert_array_equal(_ids_sorted(ctx.export_m2l()), _ids_sorted(ref["m2l"]))
    gp2p = ctx.export_p2p()
    end_of = dict(map(tuple, ctx.export_cells()))
    mask = (1 << 40) - 1
    want = np.array([(b, a & mask, end_of[a]) for a, b in ref["p2p"]], dtype=np.int64)
    # the same particle pairs summed directly onto each sink cell (the GPU walk
    # emits a whole source cell at once where the recursion would reach only
    # its leaves; merged ranges compare equal)
    np.testing.assert_array_equal(_merged(gp2p), _merged(want))
    assert st["n_p2p_pairs"] == ref["stats"]["n_p2p_pairs"]
    assert st["n_m2l"] == ref["stats"]["n_m2l"]
    # the sink scale of the estimate pass
    np.testing.assert_allclose(ctx.export_scale(), ref["scale"], rtol=1e-11)
    # forces and potentials
    assert _rel(acc, ref["acc"]).max() < 1e-10
    assert np.max(np.abs(pot - ref["pot"]) / np.abs(ref["pot"])) < 1e-10
    assert gp2p.shape[0] > 0


def test_fmm_accuracy_against_direct_sum(ctx):
    """rms delta a / a about eps (criterion a), 99.9% within ~10x (Sec. 6.3)."""
    n, eps = 50000, 1e-7
    pos, m = W.cluster("plummer", n, 8)
    pot, acc = _gpu_fmm(ctx, pos, m, -1, eps)
    sinks = np.random.default_rng(1).choice(n, 3000, replace=False)
    p0, a0, _ = oracle.direct(pos, m, sinks=sinks)
    e = oracle.error_summary(_rel(acc[sinks], a0))
    print("error", e, ctx.stats(), flush=True)
    assert e["rms"] < 2 * eps
    assert e["p99.9"] < 30 * eps
    assert np.max(np.abs(pot[sinks] - p0) / np.abs(p0)) < 1e-6


def test_high_order_generic_kernel_matches_oracle(gpu_lib):
    """Orders 13 and 16 (the largest register kernels) and 18 (above them: the
    LDS-staged kernel)."""
    ctx = gpu_lib.Context(leaf_size=16, p2p_factor=0.5)
    for p in (13, 16, 18):
        pos, m = W.cluster("plummer", 5000, 9)
        pot, acc = _gpu_fmm(ctx, pos, m, p, 1e-9)
        ref = oracle.fmm(pos, m, p=p, eps=1e-9, leaf_size=16, p2p_pairs=0.5 * (p + 1) ** 3)
        assert ctx.stats()["n_m2l"] == ref["stats"]["n_m2l"] > 0
        assert _rel(acc, ref["acc"]).max() < 1e-10


def test_criterion_f_and_theta_modes(gpu_lib):
    pos, m = W.cluster("plummer", 8000, 2)
    c_f = gpu_lib.Context(mac="f", p2p_factor=0.5)
    _, acc = _gpu_fmm(c_f, pos, m, 10, 10 ** -6.25)
    ref = oracle.fmm(pos, m, p=10, eps=10 ** -6.25, leaf_size=32, mac=oracle.MAC_F,
                     p2p_pairs=0.5 * 11 ** 3)
    assert c_f.stats()["n_m2l"] == ref["stats"]["n_m2l"]
    assert _rel(acc, ref["acc"]).max() < 1e-10
    c_t = gpu_lib.Context(mac="theta", theta_crit=0.4, p2p_factor=0.5)
    _, acc = _gpu_fmm(c_t, pos, m, 8, 0.0)
    ref = oracle.fmm(pos, m, p=8, eps=0.0, leaf_size=32, mac=oracle.MAC_THETA, theta_crit=0.4,
                     p2p_pairs=0.5 * 9 ** 3)
    assert c_t.stats()["n_m2l"] == ref["stats"]["n_m2l"]
    assert _rel(acc, ref["acc"]).max() < 1e-10


def test_deterministic(ctx):
    pos, m = W.cluster("dehnen1", 30000, 4)
    a = _gpu_fmm(ctx, pos, m, 9, 1e-7)
    b = _gpu_fmm(ctx, pos, m, 9, 1e-7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_tiny_and_degenerate_inputs(ctx, gpu_lib):
    import torch
    for n in (0, 1, 2, 3, 5):
        pos, m = W.cluster("uniform", n, 1)
        if n == 0:
            P = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
            M = torch.zeros(0, dtype=torch.float64, device="cuda")
            ctx.forces(P, M)
            continue
        pot, acc = _gpu_fmm(ctx, pos, m, 6, 1e-7)
        p0, a0, _ = oracle.direct(pos, m)
        np.testing.assert_allclose(pot, p0, rtol=1e-13, atol=0)
        np.testing.assert_allclose(acc, a0, rtol=1e-12, atol=1e-300)
    # particles closer than the 42-bit quantum: an overfull leaf at depth 42
    rng = np.random.default_rng(4)
    pos = np.vstack([1e-14 * rng.normal(size=(40, 3)) + 0.5, 100.0 * rng.normal(size=(60, 3))])
    m = np.full(100, 0.01)
    c4 = gpu_lib.Context(leaf_size=4)
    _, acc = _gpu_fmm(c4, pos, m, 8, 1e-10)
    assert c4.stats()["depth"] == 42
    _, a0, _ = oracle.direct(pos, m)
    assert _rel(acc, a0)[:40].max() < 1e-9


def test_error_paths(ctx, gpu_lib):
    import torch
    pos, m = W.cluster("plummer", 100, 1)
    P, M = _to_dev(pos, m)
    with pytest.raises(gpu_lib.FMMError) as e:
        ctx.forces(P, M, target_err=-1.0)
    assert e.value.status == gpu_lib.E_INVAL
    with pytest.raises(gpu_lib.FMMError) as e:
        ctx.forces(P, M, p=25, target_err=1e-7)
    assert e.value.status == gpu_lib.E_UNSUPPORTED
    with pytest.raises(TypeError):
        ctx.forces(P.float(), M)
    # orders below the supported range are refused before any launch: FP64
    # and jerk calls need p >= 3, mixed precision p >= 2
    for p in (1, 2):
        with pytest.raises(gpu_lib.FMMError) as e:
            ctx.forces(P, M, p=p, target_err=1e-6)
        assert e.value.status == gpu_lib.E_UNSUPPORTED
    mixed = gpu_lib.Context(precision="mixed")
    with pytest.raises(gpu_lib.FMMError) as e:
        mixed.forces(P, M, p=1, target_err=1e-6)
    assert e.value.status == gpu_lib.E_UNSUPPORTED
    with pytest.raises(gpu_lib.FMMError) as e:
        mixed.forces_jerk(P, torch.zeros_like(P), M, p=2, target_err=1e-6)
    assert e.value.status == gpu_lib.E_UNSUPPORTED
    # two distinct particles at one position: non-finite result is reported
    pos2 = pos.copy()
    pos2[7] = pos2[3]
    P2, _ = _to_dev(pos2, m)
    with pytest.raises(gpu_lib.FMMError) as e:
        ctx.forces(P2, M, p=6, target_err=1e-6)
    assert e.value.status == gpu_lib.E_NONFINITE
    # the context stays usable after an error
    pot, acc = ctx.forces(P, M, p=6, target_err=1e-6)
    torch.cuda.synchronize()
    assert torch.isfinite(acc).all()


def test_direct_sinks_matches_oracle(ctx, gpu_lib):
    """The exact sum for listed sinks (the reference used on large inputs)."""
    import torch
    pos, m = W.cluster("dehnen1", 6000, 3, masses="salpeter")
    P, M = _to_dev(pos, m)
    sinks = np.array([0, 5999, 17, 17, 3000, 1234], dtype=np.int64)
    pot, acc = ctx.direct_sinks(P, M, torch.from_numpy(sinks).cuda(), G=2.0)
    torch.cuda.synchronize()
    p0, a0, _ = oracle.direct(pos, m, G=2.0, sinks=sinks)
    np.testing.assert_allclose(pot.cpu().numpy(), p0, rtol=1e-12)
    assert _rel(acc.cpu().numpy(), a0).max() < 1e-12
    with pytest.raises(gpu_lib.FMMError) as e:
        ctx.direct_sinks(P, M, torch.tensor([3, 6000], dtype=torch.int64, device="cuda"))
    assert e.value.status == gpu_lib.E_INVAL
