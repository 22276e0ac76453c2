"""Pins of the oracle's FMM kernels (P2M, M2M, M2L, L2L, L2P, P_n, E_AB)
against exact identities and the paper's strict error bound (no GPU)."""
import math

import numpy as np
import pytest

import oracle


def _cloud(rng, n, centre, radius):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    d *= radius * rng.uniform(0, 1, n)[:, None] ** (1 / 3)
    return centre + d, rng.uniform(0.5, 1.5, n) / n


def _direct_field(src, m, x):
    d = src[None, :, :] - x[:, None, :]
    r = np.linalg.norm(d, axis=2)
    pot = np.sum(m / r, axis=1)
    acc = np.sum(m[None, :, None] * d / r[:, :, None] ** 3, axis=1)
    return pot, acc


def test_p2m_single_particle_power():
    """One particle at distance rho from the centre: P_n = mu rho^n (eq:def:PA,
    addition theorem at x-hat = r-hat)."""
    z = np.array([0.1, 0.2, -0.3])
    x = np.array([[0.5, -0.4, 0.2]])
    mu = np.array([0.7])
    p = 12
    P = oracle.power(oracle.p2m(x, mu, z, p), p)
    rho = np.linalg.norm(x[0] - z)
    for n in range(p + 1):
        assert P[n] == pytest.approx(mu[0] * rho ** n, rel=1e-13)


def test_power_bounds_and_rotation_invariance():
    """P_n <= M rho^n, |M_n^m| <= P_n / n!, invariant under rotation (Sec. 4.1.2)."""
    rng = np.random.default_rng(1)
    z = np.zeros(3)
    x, m = _cloud(rng, 50, z, 1.0)
    p = 10
    M = oracle.p2m(x, m, z, p)
    P = oracle.power(M, p)
    rho = np.max(np.linalg.norm(x - z, axis=1))
    for n in range(p + 1):
        assert P[n] <= m.sum() * rho ** n * (1 + 1e-12)
        for mm in range(-n, n + 1):
            assert abs(M[oracle.idx(n, mm)]) <= P[n] / math.factorial(n) * (1 + 1e-12)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    P2 = oracle.power(oracle.p2m(x @ q.T, m, z, p), p)
    np.testing.assert_allclose(P2, P, rtol=1e-12)
    assert M[0].real == pytest.approx(m.sum(), rel=1e-15)


def test_dipole_vanishes_at_centre_of_mass():
    rng = np.random.default_rng(2)
    x, m = _cloud(rng, 30, np.array([1.0, 2.0, 3.0]), 0.5)
    com = (m[:, None] * x).sum(0) / m.sum()
    M = oracle.p2m(x, m, com, 2)
    for mm in (-1, 0, 1):
        assert abs(M[oracle.idx(1, mm)]) < 1e-15


@pytest.mark.parametrize("p", [1, 4, 9])
def test_m2m_is_exact(p):
    """P2M about z then M2M to z' equals P2M about z' to rounding (eq:M2M)."""
    rng = np.random.default_rng(p)
    z = np.array([0.3, -0.2, 0.1])
    zp = np.array([-0.4, 0.5, 0.35])
    x, m = _cloud(rng, 40, z, 0.5)
    got = oracle.m2m(oracle.p2m(x, m, z, p), z - zp, p)
    want = oracle.p2m(x, m, zp, p)
    for n in range(p + 1):
        scale = m.sum() * np.max(np.linalg.norm(x - zp, axis=1)) ** n
        for mm in range(-n, n + 1):
            assert abs(got[oracle.idx(n, mm)] - want[oracle.idx(n, mm)]) <= 1e-13 * scale


@pytest.mark.parametrize("p", [2, 6, 10])
def test_l2l_is_exact(p):
    """Shifting the local expansion (eq:L2L) and evaluating it (eq:L2P) gives
    the value of the unshifted expansion at the same point."""
    rng = np.random.default_rng(10 + p)
    F = rng.normal(size=(p + 1) ** 2) + 1j * rng.normal(size=(p + 1) ** 2)
    for n in range(p + 1):           # make it the expansion of a real field
        F[oracle.idx(n, 0)] = F[oracle.idx(n, 0)].real
        for mm in range(1, n + 1):
            F[oracle.idx(n, -mm)] = (-1) ** mm * np.conj(F[oracle.idx(n, mm)])
    s = np.array([0.1, 0.2, 0.3])
    sp = np.array([0.25, 0.1, 0.45])
    x = np.array([0.2, 0.05, 0.5])
    Fp = oracle.l2l(F, s - sp, p)
    psi1, a1 = oracle.l2p(F, s - x, p)
    psi2, a2 = oracle.l2p(Fp, sp - x, p)
    assert psi2 == pytest.approx(psi1, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(a2, a1, rtol=1e-11, atol=1e-11)


def test_l2p_sign_single_unit_mass():
    """A unit mass at the origin seen through M2L + L2P: Psi = 1/|x| and
    a = -x/|x|^3 (eq:L2P: a = -(Re Psi_1^1, Im Psi_1^1, Psi_1^0))."""
    p = 14
    M = oracle.p2m(np.zeros((1, 3)), np.ones(1), np.zeros(3), p)
    s = np.array([3.0, -2.0, 4.0])
    F = oracle.m2l(M, s, p)
    x = s + np.array([0.05, 0.1, -0.08])
    psi, a = oracle.l2p(F, s - x, p)
    r = np.linalg.norm(x)
    assert psi == pytest.approx(1.0 / r, rel=1e-12)
    np.testing.assert_allclose(a, -x / r ** 3, rtol=1e-10)


def test_l2p_gradient_matches_finite_difference():
    rng = np.random.default_rng(3)
    src, m = _cloud(rng, 20, np.zeros(3), 0.5)
    p = 10
    M = oracle.p2m(src, m, np.zeros(3), p)
    s = np.array([2.5, 1.0, -1.5])
    F = oracle.m2l(M, s, p)
    x = s + np.array([0.1, -0.2, 0.15])
    _, a = oracle.l2p(F, s - x, p)
    h = 1e-5
    g = np.zeros(3)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        g[d] = (oracle.l2p(F, s - x - e, p)[0] - oracle.l2p(F, s - x + e, p)[0]) / (2 * h)
    np.testing.assert_allclose(a, g, rtol=1e-6)


def _pair(rng, theta, rho_a, rho_b, n_a=40):
    """Source cloud within rho_a of z_A and sink points within rho_b of s_B, at
    separation r = (rho_a + rho_b)/theta."""
    r = (rho_a + rho_b) / theta
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    zA = rng.normal(size=3)
    sB = zA + r * u
    src, m = _cloud(rng, n_a, zA, rho_a)
    snk, _ = _cloud(rng, 30, sB, rho_b)
    return zA, sB, src, m, snk, r


@pytest.mark.parametrize("p", [3, 6, 10])
def test_m2l_strict_error_bound(p):
    """Every M2L+L2P interaction with theta < 1 obeys the strict bound
    delta a <= (M_A / r^2) (p+1) theta^p / (1-theta)^2  (eq:err:bound);
    and the error falls as p grows."""
    rng = np.random.default_rng(100 + p)
    for trial in range(25):
        theta = rng.uniform(0.2, 0.8)
        rho_a, rho_b = rng.uniform(0.1, 1.0, 2)
        zA, sB, src, m, snk, r = _pair(rng, theta, rho_a, rho_b)
        # actual radii (the cloud lies inside the nominal ones)
        rho_a = np.max(np.linalg.norm(src - zA, axis=1))
        rho_b = np.max(np.linalg.norm(snk - sB, axis=1))
        th = (rho_a + rho_b) / r
        F = oracle.m2l(oracle.p2m(src, m, zA, p), sB - zA, p)
        _, acc_true = _direct_field(src, m, snk)
        bound = m.sum() / r ** 2 * (p + 1) * th ** p / (1 - th) ** 2
        for i, x in enumerate(snk):
            _, a = oracle.l2p(F, sB - x, p)
            assert np.linalg.norm(a - acc_true[i]) <= bound * (1 + 1e-9) + 1e-15


def test_m2l_converges_with_p():
    rng = np.random.default_rng(7)
    zA, sB, src, m, snk, r = _pair(rng, 0.5, 0.5, 0.5)
    _, acc_true = _direct_field(src, m, snk)
    errs = []
    for p in (2, 4, 8, 16):
        F = oracle.m2l(oracle.p2m(src, m, zA, p), sB - zA, p)
        errs.append(max(np.linalg.norm(oracle.l2p(F, sB - x, p)[1] - acc_true[i])
                        for i, x in enumerate(snk)))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-3 * errs[0]


def test_eab_equals_theta_power_for_point_source():
    """E_{A->B} <= theta^p with equality iff P_n = M rho^n (Sec. 4.1.2) - a
    single source particle at distance rho_A from the centre."""
    p = 9
    zA = np.zeros(3)
    rho_a, rho_b, r = 0.3, 0.5, 2.0
    x = np.array([[rho_a, 0.0, 0.0]])
    P = oracle.power(oracle.p2m(x, np.array([2.0]), zA, p), p)
    e = oracle.eab_times_mass(P, p, rho_b, r) / 2.0
    assert e == pytest.approx(((rho_a + rho_b) / r) ** p, rel=1e-13)
    rng = np.random.default_rng(9)
    src, m = _cloud(rng, 100, zA, rho_a)
    rho_act = np.max(np.linalg.norm(src, axis=1))
    P = oracle.power(oracle.p2m(src, m, zA, p), p)
    assert oracle.eab_times_mass(P, p, rho_b, r) / m.sum() <= ((rho_act + rho_b) / r) ** p


def test_eab_binomial_form():
    """E M_A = sum_k C(p,k) P_k rho_B^{p-k} / r^p (eq:def:EAB), checked on
    powers chosen so the sum has a closed form: P_k = c^k gives (c+rho_B)^p/r^p."""
    p, c, rb, r = 7, 0.4, 0.3, 1.9
    P = np.array([c ** k for k in range(p + 1)])
    assert oracle.eab_times_mass(P, p, rb, r) == pytest.approx((c + rb) ** p / r ** p, rel=1e-14)


def test_etilde_factor():
    """8 max(rho_A, rho_B)/(rho_A + rho_B) (eq:err:tilde): 4 for equal radii,
    8 when one radius vanishes (and when both do)."""
    assert oracle.etilde_factor(0.5, 0.5) == pytest.approx(4.0)
    assert oracle.etilde_factor(0.0, 0.5) == pytest.approx(8.0)
    assert oracle.etilde_factor(0.0, 0.0) == 8.0
    assert oracle.etilde_factor(1.0, 3.0) == pytest.approx(6.0)
