"""Host logic of the autotuner: the search grid, the selection rule, the
sampling of sinks and the per-band cache (no GPU, no kernel launched)."""
import numpy as np
import pytest

from paper_1405_2255_amd import autotune as A


def test_grid_spans_leaf_threshold_order_and_centre_rule():
    g = A.candidates(1e-7)
    assert len(g) == len(set(g)) == 11 * 5 * 3 * 2 * 2
    from paper_1405_2255_amd import fmm
    for c in g:
        assert fmm.P_MIN <= c.p <= fmm.P_MAX
        assert c.eps in (0.6e-7, 0.75e-7, 0.9e-7)
        assert c.p - fmm.order_for_error(c.eps) in (0, 1)
        assert c.centre in ("midpoint", "enclosing")
    # each point of the grid under both centre rules
    assert {(c.leaf_size, c.p2p_factor, c.eps, c.p) for c in g if c.centre == "midpoint"} == \
        {(c.leaf_size, c.p2p_factor, c.eps, c.p) for c in g if c.centre == "enclosing"}
    # the library's own defaults (n_L = 32, factor 2, p from eps) are in the grid
    assert any(c.leaf_size == 32 and c.p2p_factor == 2.0 and c.p == fmm.order_for_error(c.eps)
               for c in g)
    # orders clamp at the top of the compiled range
    assert all(c.p <= fmm.P_MAX for c in A.candidates(1e-14))


def test_select_takes_the_fastest_that_meets_the_target():
    c = [A.Candidate(32, 2.0, 1e-7, 10 + i) for i in range(4)]
    table = [(c[0], 5.0, 0.9e-7), (c[1], 7.0, 0.5e-7), (c[2], 6.0, 0.79e-7), (c[3], 9.0, 0.1e-7)]
    assert A.select(table, 1e-7, 0.8)[0] == c[2]
    assert A.select(table, 1e-7, 1.0)[0] == c[0]
    assert A.select(table, 1e-9, 0.8) is None
    assert A.select([], 1e-7, 0.8) is None


def test_sample_for_single_and_batched_workloads():
    rng = np.random.default_rng(3)
    (lo, hi, s), = A._sample(None, 1000, 4096, 16, rng)
    assert (lo, hi) == (0, 1000) and np.array_equal(s, np.arange(1000))
    (lo, hi, s), = A._sample(None, 10 ** 6, 4096, 16, rng)
    assert s.size == 4096 and np.all(np.diff(s) > 0) and s[-1] < 10 ** 6
    off = np.array([0, 0, 1, 5000, 5002, 9000, 9000, 20000])
    groups = A._sample(off, 20000, 300, 16, rng)
    spans = {(int(a), int(b)) for a, b in zip(off[:-1], off[1:]) if b - a >= 2}
    assert len(groups) == len(spans) == 4
    for lo, hi, s in groups:
        assert (lo, hi) in spans
        assert s.size == min(hi - lo, 300 // 4)
        assert np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < hi - lo


def test_band_cache_tunes_once_per_band(monkeypatch):
    calls = []

    def fake_tune(pos, mass, target, **kw):
        calls.append((pos.shape[0], target, kw["precision"]))
        return A.Result(A.Candidate(32, 2.0, target, 8), 1.0, target / 2, [])

    monkeypatch.setattr(A, "tune", fake_tune)
    bt = A.BandTuner(precision="mixed")
    assert A.BandTuner.band(1) == 0 and A.BandTuner.band(1024) == 10
    assert A.BandTuner.band(1023) == 9
    a = bt.get(np.zeros((1500, 3)), np.zeros(1500), 1e-7)
    b = bt.get(np.zeros((1900, 3)), np.zeros(1900), 1e-7)       # same band
    c = bt.get(np.zeros((2100, 3)), np.zeros(2100), 1e-7)       # next band
    d = bt.get(np.zeros((1500, 3)), np.zeros(1500), 1e-6)       # other target
    assert a is b and len(calls) == 3
    assert c.p == 8 and d.eps == 1e-6
    # batched: the band of the median cluster size
    off = np.array([0, 100, 4000, 4100])
    bt.get(np.zeros((4100, 3)), np.zeros(4100), 1e-7, offsets=off)
    assert len(calls) == 4 and bt.band(100) in {k[0] for k in bt.cache}
