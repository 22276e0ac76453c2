"""Pins of the oracle's exact direct summation (eq:P2P, eq:f) against closed
forms, conservation laws and the analytic Plummer model (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W


def test_two_body():
    """a_1 = G m_2 (x_2 - x_1)/r^3, Phi_1 = -G m_2 / r, f_1 = G m_2 / r^2."""
    G = 2.5
    pos = np.array([[0.1, -0.3, 0.2], [1.3, 0.4, -0.5]])
    m = np.array([0.7, 1.9])
    pot, acc, f = oracle.direct(pos, m, G=G)
    d = pos[1] - pos[0]
    r = np.linalg.norm(d)
    assert pot[0] == pytest.approx(-G * m[1] / r, rel=1e-15)
    assert pot[1] == pytest.approx(-G * m[0] / r, rel=1e-15)
    np.testing.assert_allclose(acc[0], G * m[1] * d / r ** 3, rtol=1e-15)
    np.testing.assert_allclose(acc[1], -G * m[0] * d / r ** 3, rtol=1e-15)
    assert f[0] == pytest.approx(G * m[1] / r ** 2, rel=1e-15)


def test_three_body_equilateral():
    """Equal masses on an equilateral triangle of side l: |a_i| = sqrt(3) G m / l^2,
    pointing at the centroid."""
    l, m0 = 1.7, 0.4
    pos = np.array([[0, 0, 0], [l, 0, 0], [l / 2, l * math.sqrt(3) / 2, 0]], dtype=float)
    pos += np.array([0.3, -0.2, 0.9])
    _, acc, f = oracle.direct(pos, np.full(3, m0))
    cen = pos.mean(0)
    for i in range(3):
        assert np.linalg.norm(acc[i]) == pytest.approx(math.sqrt(3) * m0 / l ** 2, rel=1e-14)
        u = (cen - pos[i]) / np.linalg.norm(cen - pos[i])
        np.testing.assert_allclose(acc[i] / np.linalg.norm(acc[i]), u, atol=1e-14)
        assert f[i] == pytest.approx(2 * m0 / l ** 2, rel=1e-14)


def test_momentum_conservation_and_f_bound():
    """Newton III: sum_b mu_b a_b = 0 to rounding; f_b >= |a_b| (Sec. 3.1)."""
    pos, m = W.cluster("plummer", 3000, 11, masses="salpeter")
    _, acc, f = oracle.direct(pos, m)
    ptot = (m[:, None] * acc).sum(0)
    scale = (m * np.linalg.norm(acc, axis=1)).sum()
    assert np.linalg.norm(ptot) < 1e-14 * scale
    assert np.all(f >= np.linalg.norm(acc, axis=1) * (1 - 1e-14))


def test_thread_count_independence():
    pos, m = W.cluster("dehnen1", 1500, 4)
    a = oracle.direct(pos, m, threads=1)
    b = oracle.direct(pos, m, threads=7)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_sink_subset_matches_full():
    pos, m = W.cluster("uniform", 800, 5)
    full = oracle.direct(pos, m)
    sinks = np.array([0, 17, 799, 400])
    sub = oracle.direct(pos, m, sinks=sinks)
    for u, v in zip(full, sub):
        assert np.array_equal(u[sinks], v)


def test_plummer_potential_and_energy():
    """Sampled Plummer sphere: Phi_b / Phi(r_b) averages to 1 with
    Phi(r) = -G M / sqrt(r^2 + a^2), total W = (1/2) sum mu Phi -> -(3 pi/32) G M^2/a
    (textbook Plummer model); centrally f -> 2 G M / a^2 (Sec. 3.1)."""
    n = 20000
    pos, m = W.cluster("plummer", n, 3)
    pot, acc, f = oracle.direct(pos, m)
    r = np.linalg.norm(pos, axis=1)
    ratio = pot / (-1.0 / np.sqrt(r * r + 1.0))
    assert abs(np.mean(ratio) - 1.0) < 0.02
    W_tot = 0.5 * np.sum(m * pot)
    assert W_tot == pytest.approx(-3 * math.pi / 32, rel=0.05)
    central = f[r < 0.15]
    assert central.size > 30
    assert np.median(central) == pytest.approx(2.0, rel=0.15)


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.direct(np.zeros((2, 3)), np.ones(2), sinks=np.array([5]))
