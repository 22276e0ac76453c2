"""Forces for a listed subset of sinks (Sec. 7.1, active particles of block
time steps) through the C ABI.  The tree, expansions and sink scale are those
of the full call and the walk only drops pairs whose sink cell holds no listed
particle, so every listed particle's result must equal the full call's
bitwise; against the oracle's FMM the parity bound of the full path holds."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _subsets(n, pos, rng):
    r = np.linalg.norm(pos, axis=1)
    inner = np.argsort(r)[: max(1, n // 50)]                 # the innermost 2%
    return {
        "random 1%": rng.choice(n, n // 100, replace=False),
        "random 10%, unsorted": rng.permutation(rng.choice(n, n // 10, replace=False)),
        "half": rng.choice(n, n // 2, replace=False),
        "all": np.arange(n),
        "one": np.array([n // 3]),
        "repeats": np.array([5, 5, 0, n - 1, 5]),
        "innermost 2%": inner,
    }


@pytest.mark.parametrize("kind,masses,precision", [("plummer", "equal", "fp64"),
                                                   ("dehnen1", "salpeter", "fp64"),
                                                   ("plummer", "equal", "mixed")])
def test_listed_sinks_equal_the_full_call(gpu_lib, kind, masses, precision):
    import torch
    n = 20000
    pos, m = W.cluster(kind, n, 21, masses=masses)
    P, M = _dev(pos), _dev(m)
    ctx = gpu_lib.Context(precision=precision)
    pot, acc = ctx.forces(P, M, 1.0, 10, 1e-7)
    torch.cuda.synchronize()
    pot, acc = pot.cpu().numpy(), acc.cpu().numpy()
    full = ctx.stats()
    rng = np.random.default_rng(3)
    for name, idx in _subsets(n, pos, rng).items():
        print(f"{kind} {precision}: {name} ({len(idx)})", flush=True)
        pa, aa = ctx.forces_active(P, M, _dev(idx.astype(np.int64)), 1.0, 10, 1e-7)
        torch.cuda.synchronize()
        st = ctx.stats()
        assert np.array_equal(pa.cpu().numpy(), pot[idx])
        assert np.array_equal(aa.cpu().numpy(), acc[idx])
        assert st["n_m2l"] <= full["n_m2l"] and st["n_p2p_pairs"] <= full["n_p2p_pairs"]
        if name == "all":
            assert st["n_m2l"] == full["n_m2l"] and st["n_p2p_pairs"] == full["n_p2p_pairs"]
        if name in ("one", "innermost 2%"):
            assert st["n_p2p_pairs"] < full["n_p2p_pairs"] / 5


def test_listed_sinks_match_the_oracle(gpu_lib):
    import torch
    pos, m = W.cluster("plummer", 6000, 8)
    idx = np.random.default_rng(1).choice(6000, 700, replace=False)
    ctx = gpu_lib.Context(p2p_factor=0.5)
    _, acc = ctx.forces_active(_dev(pos), _dev(m), _dev(idx.astype(np.int64)), 1.0, 8, 1e-7)
    torch.cuda.synchronize()
    ref = oracle.fmm(pos, m, p=8, eps=1e-7, leaf_size=32, p2p_pairs=0.5 * 9 ** 3)
    d = np.linalg.norm(acc.cpu().numpy() - ref["acc"][idx], axis=1) / np.linalg.norm(
        ref["acc"][idx], axis=1)
    assert d.max() < 1e-10


def test_listed_sinks_with_a_recycled_tree(gpu_lib):
    import torch
    pos, vel = W.plummer(15000, 4, with_velocities=True)
    m = np.full(15000, 1.0 / 15000)
    P0, M = _dev(pos), _dev(m)
    P1 = _dev(pos + 1e-3 * vel)
    idx = np.random.default_rng(2).choice(15000, 1500, replace=False).astype(np.int64)
    a = gpu_lib.Context(scale_source="previous")
    b = gpu_lib.Context(scale_source="previous")
    a.forces(P0, M, 1.0, 9, 1e-7)
    b.forces(P0, M, 1.0, 9, 1e-7)
    pa, aa = a.forces_active(P1, M, _dev(idx), 1.0, 9, 1e-7, refit=True)
    pb, ab = b.forces(P1, M, 1.0, 9, 1e-7, refit=True)
    torch.cuda.synchronize()
    assert a.stats()["refitted"] == 1 and b.stats()["refitted"] == 1
    assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy()[idx])
    assert np.array_equal(aa.cpu().numpy(), ab.cpu().numpy()[idx])


def test_listed_sinks_edge_cases(gpu_lib):
    import torch
    pos, m = W.cluster("uniform", 3000, 5)
    P, M = _dev(pos), _dev(m)
    ctx = gpu_lib.Context()
    pa, aa = ctx.forces_active(P, M, _dev(np.zeros(0, np.int64)))
    assert pa.shape == (0,) and aa.shape == (0, 3)
    for bad in ([3000], [-1], [0, 2999, 3000]):
        with pytest.raises(gpu_lib.FMMError, match="FMM_E_INVAL"):
            ctx.forces_active(P, M, _dev(np.array(bad, np.int64)))
    one_p, one_m = _dev(pos[:1]), _dev(m[:1])
    pa, aa = ctx.forces_active(one_p, one_m, _dev(np.array([0, 0], np.int64)))
    torch.cuda.synchronize()
    assert np.all(pa.cpu().numpy() == 0.0) and np.all(aa.cpu().numpy() == 0.0)
    with pytest.raises(gpu_lib.FMMError, match="FMM_E_INVAL"):
        ctx.forces_active(one_p, one_m, _dev(np.array([1], np.int64)))
