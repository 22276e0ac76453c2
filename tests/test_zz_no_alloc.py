"""fmm_direct_sinks_noalloc (the entry point that allocates nothing) through
the C ABI, against fmm_direct_sinks and the oracle.

Both entry points run the same kernels with the same split of the sources,
so their results are equal bit for bit; against the oracle's compensated
direct sum the bound of the other direct-sum tests applies (relative 1e-12
per sink).  Two calls in a row, the second with a smaller input (the static
scratch array keeps the first call's contents), a call with one source chunk,
an index out of range and an empty list."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,nsinks,seed", [(100000, 2048, 1), (40000, 300, 2), (3000, 77, 3)])
def test_noalloc_equals_direct_sinks_and_oracle(gpu_lib, n, nsinks, seed):
    import torch
    print(f"noalloc n={n} nsinks={nsinks}", flush=True)
    pos, m = W.cluster("dehnen1", n, seed, masses="salpeter")
    P, M = _dev(pos), _dev(m)
    sinks = np.random.default_rng(seed).choice(n, nsinks, replace=False).astype(np.int64)
    sinks[:3] = [0, n - 1, 0]                                  # ends and a repeat
    S = _dev(sinks)
    ctx = gpu_lib.Context()
    pot0, acc0 = ctx.direct_sinks(P, M, S, G=1.3)
    pot = torch.empty(nsinks, dtype=torch.float64, device="cuda")
    acc = torch.empty((nsinks, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.direct_sinks(P, M, S, G=1.3, pot=pot, acc=acc, noalloc=True)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0              # nothing allocated
    assert torch.equal(pot, pot0) and torch.equal(acc, acc0)
    p_ref, a_ref, _ = oracle.direct(pos, m, G=1.3, sinks=sinks)
    np.testing.assert_allclose(pot.cpu().numpy(), p_ref, rtol=1e-12)
    assert _rel(acc.cpu().numpy(), a_ref).max() < 1e-12


def test_noalloc_two_calls_second_smaller(gpu_lib):
    """The second call reads less of the shared array than the first wrote:
    stale rows must not leak into its sums."""
    import torch
    ctx = gpu_lib.Context()
    out = []
    for n, ns, seed in ((120000, 4096, 11), (30000, 1000, 12)):
        pos, m = W.cluster("plummer", n, seed)
        sinks = np.random.default_rng(seed).choice(n, ns, replace=False).astype(np.int64)
        P, M, S = _dev(pos), _dev(m), _dev(sinks)
        pot, acc = ctx.direct_sinks(P, M, S, noalloc=True)
        pot0, acc0 = ctx.direct_sinks(P, M, S)
        torch.cuda.synchronize()
        assert torch.equal(pot, pot0) and torch.equal(acc, acc0)
        p_ref, a_ref, _ = oracle.direct(pos, m, sinks=sinks)
        np.testing.assert_allclose(pot.cpu().numpy(), p_ref, rtol=1e-12)
        assert _rel(acc.cpu().numpy(), a_ref).max() < 1e-12
        out.append(pot)
    assert out[0].shape[0] > out[1].shape[0]


def test_noalloc_errors_and_empty(gpu_lib):
    import torch
    ctx = gpu_lib.Context()
    pos, m = W.cluster("plummer", 5000, 4)
    P, M = _dev(pos), _dev(m)
    with pytest.raises(gpu_lib.FMMError) as e:
        ctx.direct_sinks(P, M, _dev(np.array([3, 5000], np.int64)), noalloc=True)
    assert e.value.status == gpu_lib.E_INVAL
    pot, acc = ctx.direct_sinks(P, M, _dev(np.zeros(0, np.int64)), noalloc=True)
    assert pot.shape == (0,)
    # the shared flag was cleared again: a valid call after the failed one succeeds
    sinks = np.array([1, 2, 4999], np.int64)
    pot, acc = ctx.direct_sinks(P, M, _dev(sinks), noalloc=True)
    torch.cuda.synchronize()
    _, a_ref, _ = oracle.direct(pos, m, sinks=sinks)
    assert _rel(acc.cpu().numpy(), a_ref).max() < 1e-12
