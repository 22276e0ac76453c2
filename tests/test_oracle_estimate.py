"""Pins of the oracle's low-order estimate of the sink scale (Sec. 5.4.2)
against values computed by hand from the definition, with no GPU.

The estimate puts every cell's expansion centre at its centre of mass z_com,
accepts a cell pair when rho_com,A + rho_com,B < |z_B - z_A|, and sums the rest
exactly.  For criterion a it uses the order-1 expansion: about z_com the dipole
vanishes, so a source cell acts on a sink cell through the monopole field
M_A (z_A - z_B)/|z_A - z_B|^3, which is constant over the sink cell.  For
criterion f it uses the order-0 term of the 1/r^2 Green's function,
M_A/|z_B - z_A|^2.  Geometries with two and three cells fix which pairs are
accepted, so the expected scale of every particle is a short closed sum.
"""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W


def _own(pos, m, idx):
    """Exact acceleration and 1/r^2 sum of each particle of idx from the other
    particles of idx (plain loops, FP64)."""
    a = np.zeros((len(idx), 3))
    f = np.zeros(len(idx))
    for u, b in enumerate(idx):
        for c in idx:
            if c == b:
                continue
            d = pos[c] - pos[b]
            r2 = d @ d
            a[u] += m[c] * d / r2 ** 1.5
            f[u] += m[c] / r2
    return a, f


def _com(pos, m, idx):
    return (m[idx, None] * pos[idx]).sum(0) / m[idx].sum()


def _monopole(pos, m, src, snk_centre):
    """Field and 1/r^2 term of the cell src's monopole at snk_centre."""
    d = _com(pos, m, src) - snk_centre
    r2 = d @ d
    M = m[src].sum()
    return M * d / r2 ** 1.5, M / r2


def _scale(pos, m, mac, leaf_size):
    r = oracle.fmm(pos, m, p=4, eps=1e-6, leaf_size=leaf_size, mac=mac, want_lists=True)
    return r["scale"], r["stats"]


def _two_clusters(rng):
    """Cluster A in the lower octant of the root cube, B in the upper one; each
    fits one leaf and they are far apart compared with their sizes."""
    a = 0.05 + 0.2 * rng.random((20, 3))
    b = 0.75 + 0.2 * rng.random((30, 3))
    pos = np.vstack([a, b])
    m = rng.uniform(0.5, 2.0, 50)
    return pos, m, np.arange(20), np.arange(20, 50)


@pytest.mark.parametrize("mac", [oracle.MAC_A, oracle.MAC_F])
def test_two_far_clusters(mac):
    """Two far clusters: each particle's scale is the exact sum over its own
    cluster plus the other cluster's monopole at its own centre of mass -
    the field for criterion a, M_A/r^2 for criterion f."""
    rng = np.random.default_rng(7)
    pos, m, A, B = _two_clusters(rng)
    s, st = _scale(pos, m, mac, leaf_size=32)
    assert st["n_cells"] == 3 and st["n_leaves"] == 2
    assert st["n_est_m2l"] == 2          # A -> B and B -> A
    for snk, src in ((A, B), (B, A)):
        a, f = _own(pos, m, snk)
        ga, gf = _monopole(pos, m, src, _com(pos, m, snk))
        want = np.linalg.norm(a + ga, axis=1) if mac == oracle.MAC_A else f + gf
        np.testing.assert_allclose(s[snk], want, rtol=1e-13)
        # the far term is not negligible: dropping it or using 1/r in place of
        # 1/r^2 would move the result well outside the tolerance
        r = np.linalg.norm(_com(pos, m, src) - _com(pos, m, snk))
        other = np.linalg.norm(a, axis=1) if mac == oracle.MAC_A else f + gf * r
        assert np.abs(other / want - 1).min() > 1e-4


def _lopsided_pair():
    """Two rod-like clusters along x, each with a heavy particle at its inner
    end.  About the centre of mass each rod's radius is about its length D,
    about the midpoint of its bounding box about D/2; the centres of mass are
    ~1.5 D apart.  So the estimate's test rho_com,A + rho_com,B < r fails
    (sum ~2 D), while radii about the box midpoints (sum ~D) would pass."""
    rng = np.random.default_rng(3)
    D = 1.0
    xa = np.concatenate([rng.uniform(0.0, 0.9 * D, 9), [D]])
    xb = np.concatenate([rng.uniform(2.6 * D, 3.5 * D, 9), [2.5 * D]])
    x = np.concatenate([xa, xb])
    yz = 0.01 * rng.random((20, 2))
    pos = np.column_stack([x, yz])
    m = np.ones(20)
    m[9] = m[19] = 100.0
    return pos, m, np.arange(10), np.arange(10, 20)


@pytest.mark.parametrize("mac", [oracle.MAC_A, oracle.MAC_F])
def test_acceptance_uses_radius_about_centre_of_mass(mac):
    """The estimate's acceptance uses the radii about z_com (Sec. 5.4.2): for
    the lopsided rods it rejects the pair, so both leaves are summed directly
    and the scale is the exact a (or f) of every particle."""
    pos, m, A, B = _lopsided_pair()
    ca, cb = _com(pos, m, A), _com(pos, m, B)
    r = np.linalg.norm(cb - ca)
    rho_com = [np.linalg.norm(pos[I] - c, axis=1).max() for I, c in ((A, ca), (B, cb))]
    mid = [(pos[I].min(0) + pos[I].max(0)) / 2 for I in (A, B)]
    rho_box = [np.linalg.norm(pos[I] - c, axis=1).max() for I, c in zip((A, B), mid)]
    assert rho_com[0] + rho_com[1] >= r > rho_box[0] + rho_box[1]   # the geometry works
    s, st = _scale(pos, m, mac, leaf_size=16)
    assert st["n_cells"] == 3 and st["n_leaves"] == 2
    assert st["n_est_m2l"] == 0 and st["n_est_p2p_pairs"] == 20 * 19
    _, a0, f0 = oracle.direct(pos, m)
    want = np.linalg.norm(a0, axis=1) if mac == oracle.MAC_A else f0
    np.testing.assert_allclose(s, want, rtol=1e-13)
    # accepting the pair would give a markedly different scale
    for snk, src in ((A, B), (B, A)):
        a, f = _own(pos, m, snk)
        ga, gf = _monopole(pos, m, src, _com(pos, m, snk))
        alt = np.linalg.norm(a + ga, axis=1) if mac == oracle.MAC_A else f + gf
        assert np.abs(alt / want[snk] - 1).max() > 1e-3


def _three_cells():
    """A small cluster A near the lower corner; a parent cell B in the upper
    octant with two adjacent leaf children B1, B2 that are too close to pass
    the test against each other, while A and B pass."""
    rng = np.random.default_rng(11)
    a = 0.08 * rng.random((10, 3))
    a[0] = 0.0                                   # root cube [0, 1]^3: B in [0.5, 1]^3,
    b1 = np.column_stack([rng.uniform(0.55, 0.72, 12), rng.uniform(0.55, 0.72, (12, 2))])
    b2 = np.column_stack([rng.uniform(0.78, 1.0, 14), rng.uniform(0.55, 0.72, (14, 2))])
    b2[0, 0] = 1.0                               # split at x = 0.75 into B1 and B2
    pos = np.vstack([a, b1, b2])
    m = rng.uniform(0.5, 2.0, 36)
    return pos, m, np.arange(10), np.arange(10, 22), np.arange(22, 36)


@pytest.mark.parametrize("mac", [oracle.MAC_A, oracle.MAC_F])
def test_far_field_passes_down_from_the_accepting_cell(mac):
    """A is accepted against the parent B, so every particle of B1 and B2 gets
    A's monopole evaluated at B's centre of mass (passed down unchanged: at
    order 1 the field is constant, the f term is a constant), plus the exact sum
    over B1 and B2 together; A gets B's monopole at its own centre of mass."""
    pos, m, A, B1, B2 = _three_cells()
    B = np.concatenate([B1, B2])
    s, st = _scale(pos, m, mac, leaf_size=16)
    assert st["n_cells"] == 5 and st["n_leaves"] == 3
    assert st["n_est_m2l"] == 2                        # A -> B, B -> A
    assert st["n_est_p2p_pairs"] == 10 * 9 + 26 * 25   # A with A; B1, B2 among themselves
    for snk, src in ((A, B), (B, A)):
        a, f = _own(pos, m, snk)
        ga, gf = _monopole(pos, m, src, _com(pos, m, snk))
        want = np.linalg.norm(a + ga, axis=1) if mac == oracle.MAC_A else f + gf
        np.testing.assert_allclose(s[snk], want, rtol=1e-13)
    # the field at the children's own centres would differ
    for child in (B1, B2):
        a, f = _own(pos, m, B)
        ga, gf = _monopole(pos, m, A, _com(pos, m, child))
        alt = np.linalg.norm(a + ga, axis=1) if mac == oracle.MAC_A else f + gf
        k = np.searchsorted(B, child)
        assert np.abs(alt[k] / s[child] - 1).max() > 1e-6


@pytest.mark.parametrize("mac", [oracle.MAC_A, oracle.MAC_F])
def test_estimate_accuracy_on_plummer(mac):
    """Against the exact a_b (or f_b) of a Plummer sphere the estimate's rms
    relative error is of order 15% (Sec. 5.4.2), with no bias larger than a
    few percent."""
    pos, m = W.cluster("plummer", 8000, 13)
    _, acc0, f0 = oracle.direct(pos, m)
    s, st = _scale(pos, m, mac, leaf_size=16)
    ref = np.linalg.norm(acc0, axis=1) if mac == oracle.MAC_A else f0
    e = (s - ref) / ref
    assert st["n_est_m2l"] > 0
    assert 0.08 < np.sqrt(np.mean(e ** 2)) < 0.3
    assert abs(np.mean(e)) < 0.03
