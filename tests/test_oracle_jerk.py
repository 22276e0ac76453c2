"""Pins of the oracle's jerk (Sec. 7, jerk, eqs:fmm:dot; App. A.5 time
derivatives) against finite differences in time, closed forms and the direct
sum (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_1405_2255_amd import workloads as W


def _fd(f, h):
    return (f(h) - f(-h)) / (2 * h)


def test_upsilon_dot_is_time_derivative():
    """d/dt Upsilon_n^m(r + t v) at t = 0 by central differences, all n <= 8."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        r, v = rng.normal(size=3), rng.normal(size=3)
        an = oracle.upsilon_dot(r, v, 8)
        fd = _fd(lambda h: oracle.upsilon(r + h * v, 8), 1e-5)
        assert np.abs(fd - an).max() < 1e-9 * np.abs(an).max()


def test_upsilon_dot_closed_forms_and_pairing():
    """Upsilon_1^1 = (x+iy)/2 and Upsilon_1^0 = z, so their rates are
    (vx + i vy)/2 and vz; Upsilon_0^0 = 1 has rate 0.  The printed relation
    pairs xidot with Upsilon_{n-1}^{m+1}; that pairing gives the rate of
    Upsilon_1^1 as etadot = -(vx - i vy)/2, which is not it."""
    r, v = np.array([0.3, -0.7, 0.4]), np.array([0.9, 0.2, -0.5])
    ud = oracle.upsilon_dot(r, v, 3)
    assert ud[oracle.idx(0, 0)] == 0
    assert ud[oracle.idx(1, 1)] == pytest.approx(0.5 * (v[0] + 1j * v[1]), rel=1e-15)
    assert ud[oracle.idx(1, 0)] == pytest.approx(v[2], rel=1e-15)
    etad = -0.5 * (v[0] - 1j * v[1])
    assert abs(ud[oracle.idx(1, 1)] - etad) > 0.1


def test_p2m_dot_is_time_derivative():
    """eq:P2M:dot: the multipoles of particles moving with v, differentiated in
    time at a centre at rest."""
    rng = np.random.default_rng(2)
    x = rng.normal(size=(20, 3)) * 0.3
    v = rng.normal(size=(20, 3))
    m = rng.random(20)
    z = np.array([0.05, -0.02, 0.01])
    an = oracle.p2m_dot(x, v, m, z, 10)
    fd = _fd(lambda h: oracle.p2m(x + h * v, m, z, 10), 1e-5)
    assert np.abs(fd - an).max() < 1e-9 * np.abs(an).max()


def test_l2p_dot_is_time_derivative():
    """eq:L2P:dot: the field of a local expansion F(t) = F + t Fd at a particle
    moving with v (centre at rest) has time derivative -(Re Psidot_1^1,
    Im Psidot_1^1, Psidot_1^0)."""
    rng = np.random.default_rng(3)
    p = 9
    # expansions of a distant source cluster, so that F is a valid local field
    src = rng.normal(size=(30, 3)) * 0.2 + np.array([3.0, 1.0, -2.0])
    ms = rng.random(30)
    vs = rng.normal(size=(30, 3))
    zA = src.mean(0)
    sB = np.zeros(3)
    F = oracle.m2l(oracle.p2m(src, ms, zA, p), sB - zA, p)
    Fd = oracle.m2l(oracle.p2m_dot(src, vs, ms, zA, p), sB - zA, p)
    x, v = np.array([0.1, -0.15, 0.05]), np.array([0.4, -0.3, 0.8])
    an = oracle.l2p_dot(F, Fd, sB - x, v, p)
    fd = _fd(lambda h: oracle.l2p(F + h * Fd, sB - (x + h * v), p)[1], 1e-5)
    assert np.abs(fd - an).max() < 1e-8 * np.abs(an).max()


def test_direct_jerk_is_time_derivative():
    """The direct jerk is the time derivative of the direct acceleration."""
    pos, m = W.cluster("plummer", 400, 4)
    vel = np.random.default_rng(4).normal(size=(400, 3)) * 0.3
    j = oracle.direct_jerk(pos, vel, m, G=1.7)
    fd = _fd(lambda h: oracle.direct(pos + h * vel, m, G=1.7)[1], 1e-6)
    err = np.linalg.norm(fd - j, axis=1) / np.linalg.norm(j, axis=1)
    assert np.median(err) < 1e-7 and err.max() < 1e-4
    # sinks subset: the same values
    s = np.array([0, 17, 399])
    np.testing.assert_array_equal(oracle.direct_jerk(pos, vel, m, G=1.7, sinks=s), j[s])


def test_jerk_uniform_motion_and_rest():
    """Particles at rest have zero jerk; a common velocity leaves every
    separation fixed, so the direct jerk vanishes to rounding."""
    pos, m = W.cluster("plummer", 300, 6)
    assert np.all(oracle.direct_jerk(pos, np.zeros((300, 3)), m) == 0)
    j = oracle.direct_jerk(pos, np.tile([0.3, -0.2, 0.5], (300, 1)), m)
    assert np.abs(j).max() == 0


def _two_clusters(n_half=40, seed=9):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n_half, 3))
    x = 0.1 * x / np.linalg.norm(x, axis=1, keepdims=True) * rng.random((n_half, 1)) ** (1 / 3)
    pos = np.concatenate([x + 0.5, -x - 0.5])
    vel = rng.normal(size=(2 * n_half, 3)) * 0.5
    return pos, np.full(2 * n_half, 1.0 / (2 * n_half)), vel


def test_fmm_jerk_two_cells_is_derivative_of_its_expansion():
    """Two leaves, one M2L pair each way: the jerk of a sink particle is the
    direct jerk of its own leaf plus the time derivative of the far field
    L2P(M2L(P2M)) about the two cells' centres held at rest - the latter
    taken by central differences of the plain kernels."""
    pos, m, vel = _two_clusters()
    p = 10
    r = oracle.fmm(pos, m, p=p, eps=1e-4, leaf_size=64, vel=vel)
    assert r["stats"]["n_m2l"] == 2
    A, B = np.arange(40), np.arange(40, 80)
    zA = 0.5 * (pos[A].min(0) + pos[A].max(0))
    sB = 0.5 * (pos[B].min(0) + pos[B].max(0))

    def far_acc(h):
        xa, xb = pos[A] + h * vel[A], pos[B] + h * vel[B]
        F = oracle.m2l(oracle.p2m(xa, m[A], zA, p), sB - zA, p)
        return np.array([oracle.l2p(F, sB - x, p)[1] for x in xb])

    far_j = _fd(far_acc, 1e-6)
    near_j = oracle.direct_jerk(pos[B], vel[B], m[B])
    want = near_j + far_j
    err = np.linalg.norm(r["jerk"][B] - want, axis=1) / np.linalg.norm(want, axis=1)
    assert err.max() < 1e-7
    # and the expansion's jerk is close to the exact one
    exact = oracle.direct_jerk(pos, vel, m)[B]
    assert (np.linalg.norm(r["jerk"][B] - exact, axis=1) / np.linalg.norm(exact, axis=1)).max() < 1e-4


def test_fmm_jerk_single_leaf_is_direct():
    pos, m = W.cluster("dehnen1", 500, 7)
    vel = np.random.default_rng(7).normal(size=(500, 3))
    r = oracle.fmm(pos, m, p=4, eps=1e-6, leaf_size=1000, G=0.7, vel=vel)
    j = oracle.direct_jerk(pos, vel, m, G=0.7)
    assert (np.linalg.norm(r["jerk"] - j, axis=1) / np.linalg.norm(j, axis=1)).max() < 1e-12


def test_fmm_jerk_converges_with_accuracy():
    """Deep trees (M2M and L2L of the rates): the jerk error against the direct
    sum falls with eps and p, and its size follows the force error (the jerk
    adds one derivative, so its relative error is larger by about the order)."""
    n = 3000
    pos, m = W.cluster("plummer", n, 8)
    vel = np.random.default_rng(8).normal(size=(n, 3)) * 0.3
    j = oracle.direct_jerk(pos, vel, m)
    _, a, _ = oracle.direct(pos, m)
    rms = []
    for p, eps in ((6, 1e-4), (8, 1e-6), (12, 1e-8)):
        r = oracle.fmm(pos, m, p=p, eps=eps, leaf_size=16, vel=vel)
        ej = np.linalg.norm(r["jerk"] - j, axis=1) / np.linalg.norm(j, axis=1)
        ea = np.linalg.norm(r["acc"] - a, axis=1) / np.linalg.norm(a, axis=1)
        rj, ra = np.sqrt(np.mean(ej ** 2)), np.sqrt(np.mean(ea ** 2))
        assert rj < 4 * (p + 1) * ra
        rms.append(rj)
    assert rms[1] < rms[0] / 10 and rms[2] < rms[1] / 10
