"""Pins of the oracle's expansion centres (Sec. 5.1.1).

The enclosing rule approximates the centre of the smallest sphere enclosing
the spheres of a cell's grand-daughters (a leaf: its particles) by a few
Frank-Wolfe steps with line search, and keeps it only where the cell's radius
about it is below the radius about its bounding-box midpoint.  What fixes
the result independently of the oracle's code:

  * closed forms: the smallest enclosing sphere of an acute triangle is its
    circumcircle, of an obtuse one the sphere on its longest side, of a
    regular tetrahedron its circumsphere, of two points the sphere on them;
  * brute force: on sets of up to 9 points the smallest enclosing sphere is
    the smallest of the spheres through 1..4 of the points that contain all
    of them, so no centre can give a smaller radius, and the iteration must
    come close to it;
  * definitions: rho is the largest distance of the cell's own particles from
    its centre, never above the distance from the box midpoint, and equal to
    it under the midpoint rule, whose centre is the box midpoint;
  * accuracy: the acceptance test uses the actual radius, so either rule
    meets the same error level against the exact direct sum.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W


def _run(pos, leaf=16, centre=oracle.CENTRE_ENCLOSING, p=4, eps=1e-6):
    m = np.full(len(pos), 1.0 / len(pos))
    return oracle.fmm(pos, m, p=p, eps=eps, leaf_size=leaf, want_lists=True, centre=centre)


def _root(pos, **kw):
    """(centre, rho, rho about the midpoint) of the root cell."""
    g = _run(pos, **kw)["cell_geo"][0]
    return g[:3], g[3], g[4]


def _meb_radius(P):
    """Smallest enclosing sphere radius by enumerating the spheres through
    1..4 of the points (each the circumsphere in their affine hull)."""
    best = np.inf
    for k in range(1, 5):
        for S in itertools.combinations(range(len(P)), k):
            Q = P[list(S)]
            if k == 1:
                c = Q[0]
            else:
                A = Q[1:] - Q[0]
                G = A @ A.T
                if abs(np.linalg.det(G)) < 1e-14 * max(1.0, np.max(np.abs(G))) ** (k - 1):
                    continue
                c = Q[0] + np.linalg.solve(G, 0.5 * np.diag(G)) @ A
            best = min(best, np.max(np.linalg.norm(P - c, axis=1)))
    return best


def test_acute_triangle_gives_circumcentre():
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, np.sqrt(3) / 2, 0.0]])
    c, rho, rho_mid = _root(tri)
    np.testing.assert_allclose(c, [0.5, 0.5 / np.sqrt(3), 0.0], atol=1e-9)
    assert abs(rho - 1 / np.sqrt(3)) < 1e-9
    assert rho_mid == pytest.approx(np.sqrt(0.25 + 3 / 16))     # about (0.5, sqrt3/4, 0)


def test_obtuse_triangle_gives_longest_side_midpoint():
    ob = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [1.0, 0.3, 0.0]])
    c, rho, rho_mid = _root(ob)
    np.testing.assert_allclose(c, [1.0, 0.0, 0.0], atol=1e-9)
    assert abs(rho - 1.0) < 1e-9 and rho_mid > 1.01


def test_midpoint_kept_where_already_optimal():
    # regular tetrahedron and two points: the box midpoint is the optimal
    # centre, so the candidate cannot be strictly better and the midpoint stays
    tet = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) + [0.3, 0.1, -0.2]
    c, rho, rho_mid = _root(tet)
    np.testing.assert_array_equal(c, (tet.min(axis=0) + tet.max(axis=0)) / 2)
    assert rho == rho_mid == pytest.approx(np.sqrt(3))
    two = np.array([[0.1, 0.2, 0.3], [0.7, -0.4, 0.9]])
    c, rho, rho_mid = _root(two)
    np.testing.assert_array_equal(c, (two[0] + two[1]) / 2)
    assert rho == rho_mid


def test_leaf_radius_against_brute_force():
    rng = np.random.default_rng(11)
    ratios = []
    for _ in range(60):
        n = int(rng.integers(2, 10))
        P = rng.normal(size=(n, 3)) * rng.uniform(0.1, 2.0, size=3)
        _, rho, rho_mid = _root(P)
        opt = _meb_radius(P)
        assert rho >= opt * (1 - 1e-12)          # nothing beats the optimum
        assert rho <= rho_mid
        ratios.append(rho / opt)
    ratios = np.array(ratios)
    # 16 line-search steps: within a few per cent of the optimum, and on
    # average within 0.5 per cent
    assert ratios.max() < 1.05 and ratios.mean() < 1.005, (ratios.max(), ratios.mean())


def test_internal_cell_from_granddaughter_spheres():
    # three tight clumps at the corners of an acute triangle: the root is an
    # internal cell whose candidate comes from its grand-daughters' spheres;
    # its radius is the circumradius plus at most the clump size
    rng = np.random.default_rng(3)
    corners = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, np.sqrt(3) / 2, 0.0]])
    a = 1e-3
    pos = np.concatenate([c + a * rng.uniform(-1, 1, size=(200, 3)) for c in corners])
    r = _run(pos, leaf=16)
    ids = r["cells"][:, 0]
    assert ids[0] >> 40 == 0 and len(ids) > 20                    # root first, split
    c, rho, rho_mid = r["cell_geo"][0, :3], r["cell_geo"][0, 3], r["cell_geo"][0, 4]
    R = 1 / np.sqrt(3)
    assert R - 2 * a < rho < R + 2 * a * np.sqrt(3), rho
    assert rho_mid > 0.65
    np.testing.assert_allclose(c, [0.5, 0.5 / np.sqrt(3), 0.0], atol=5 * a)


@pytest.mark.parametrize("centre", [oracle.CENTRE_MIDPOINT, oracle.CENTRE_ENCLOSING])
def test_rho_is_the_radius_of_the_cells_particles(centre):
    n = 4000
    pos = W.plummer(n, 21)
    r = _run(pos, leaf=12, centre=centre)
    order, cells, geo = r["order"], r["cells"], r["cell_geo"]
    X = pos[order]                                   # Morton order
    smaller = 0
    for (cid, end), g in zip(cells, geo):
        beg = cid & ((1 << 40) - 1)
        P = X[beg:end]
        d2 = np.sum((P - g[:3]) ** 2, axis=1)
        assert np.sqrt(d2.max()) == pytest.approx(g[3], rel=1e-14, abs=1e-300)
        mid = (P.min(axis=0) + P.max(axis=0)) / 2
        rho_mid = np.sqrt(np.max(np.sum((P - mid) ** 2, axis=1)))
        assert g[4] == pytest.approx(rho_mid, rel=1e-14, abs=1e-300)
        assert g[3] <= g[4]
        if centre == oracle.CENTRE_MIDPOINT:
            np.testing.assert_array_equal(g[:3], mid)
            assert g[3] == g[4]
        elif end - beg >= 3 and g[3] < g[4]:
            smaller += 1
    if centre == oracle.CENTRE_ENCLOSING:
        multi = sum(1 for cid, end in cells if end - (cid & ((1 << 40) - 1)) >= 3)
        assert smaller > 0.8 * multi, (smaller, multi)


def test_accuracy_is_the_same_under_either_rule():
    n = 3000
    pos = W.plummer(n, 22)
    m = np.full(n, 1.0 / n)
    _, a0, _ = oracle.direct(pos, m)
    rms = {}
    for centre in (oracle.CENTRE_MIDPOINT, oracle.CENTRE_ENCLOSING):
        r = oracle.fmm(pos, m, p=6, eps=1e-6, leaf_size=16, centre=centre)
        e = np.linalg.norm(r["acc"] - a0, axis=1) / np.linalg.norm(a0, axis=1)
        rms[centre] = np.sqrt(np.mean(e ** 2))
        assert rms[centre] < 1e-5, rms
    assert rms[oracle.CENTRE_ENCLOSING] < 2 * rms[oracle.CENTRE_MIDPOINT]
