"""Pins of the oracle's solid harmonics against facts the paper and the
mathematics fix (no GPU)."""
import math

import numpy as np
import pytest

import oracle
from conftest import golden_path


def _load_table():
    rows = []
    with open(golden_path("tab_the.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, m, c, expr = line.split(None, 3)
            rows.append((int(n), int(m), int(c), expr))
    return rows


TABLE = _load_table()


def _real(X, n, m):
    v = X[oracle.idx(n, abs(m))]
    return v.real if m >= 0 else v.imag


def test_table_has_all_49_entries():
    assert len(TABLE) == 49
    assert {(n, m) for n, m, _, _ in TABLE} == {(n, m) for n in range(7) for m in range(-n, n + 1)}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_closed_forms_tab_the(seed):
    """(n-m)!(n+m)! U_n^m = r^{2n+1} T_n^m = the table's polynomial (tab:The)."""
    rng = np.random.default_rng(seed)
    x, y, z = rng.normal(size=3) * rng.uniform(0.3, 3.0)
    r = math.sqrt(x * x + y * y + z * z)
    U = oracle.upsilon([x, y, z], 6)
    T = oracle.theta([x, y, z], 6)
    for n, m, c, expr in TABLE:
        want = c * eval(expr, {}, {"x": x, "y": y, "z": z, "r": r})
        fac = math.factorial(n - m) * math.factorial(n + m)
        scale = r ** n * fac + 1e-300
        assert abs(fac * _real(U, n, m) - want) <= 1e-13 * scale, (n, m)
        assert abs(r ** (2 * n + 1) * _real(T, n, m) - want) <= 1e-13 * scale, (n, m)


def test_upsilon_on_z_axis():
    """Upsilon_n^m(z-hat) = delta_{m0} / n!  (App. A.6)."""
    p = 20
    U = oracle.upsilon([0.0, 0.0, 1.0], p)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            want = 1.0 / math.factorial(n) if m == 0 else 0.0
            assert abs(U[oracle.idx(n, m)] - want) <= 1e-15 * max(1.0, abs(want))


def test_theta_on_z_axis():
    """Theta_n^0(0,0,r) = n!/r^{n+1}, the factor of the z-axis M2L (eq:M2L:z);
    Theta_n^{m != 0} vanishes there."""
    p, r = 16, 1.7
    T = oracle.theta([0.0, 0.0, r], p)
    for n in range(p + 1):
        want = math.factorial(n) / r ** (n + 1)
        assert abs(T[oracle.idx(n, 0)] - want) <= 1e-13 * want
        for m in range(1, n + 1):
            assert abs(T[oracle.idx(n, m)]) <= 1e-14 * want


def test_homogeneity():
    """Theta_n^m(a r) = a^{-(n+1)} Theta_n^m(r), Upsilon_n^m(a r) = a^n Upsilon_n^m(r) (App. A.3)."""
    p, a = 12, 2.375
    r = np.array([0.3, -1.1, 0.7])
    T1, T2 = oracle.theta(r, p), oracle.theta(a * r, p)
    U1, U2 = oracle.upsilon(r, p), oracle.upsilon(a * r, p)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            k = oracle.idx(n, m)
            assert abs(T2[k] - a ** (-(n + 1)) * T1[k]) <= 1e-13 * abs(T1[k]) * a ** (-(n + 1)) + 1e-300
            assert abs(U2[k] - a ** n * U1[k]) <= 1e-13 * abs(U1[k]) * a ** n + 1e-300


def test_symmetry():
    """X_n^{-m} = (-1)^m conj(X_n^m) (eq:sym)."""
    p = 10
    r = [0.4, 0.9, -0.2]
    for X in (oracle.theta(r, p), oracle.upsilon(r, p)):
        for n in range(p + 1):
            for m in range(n + 1):
                assert X[oracle.idx(n, -m)] == pytest.approx((-1) ** m * np.conj(X[oracle.idx(n, m)]), rel=1e-15, abs=1e-300)


def test_addition_theorem():
    """1/|r - x| = sum_{n,m} Upsilon_n^m(x) conj(Theta_n^m(r)) for |x| < |r| (eq:Sph:r-x)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        r = rng.normal(size=3)
        r *= 2.0 / np.linalg.norm(r)
        x = rng.normal(size=3)
        x *= rng.uniform(0.05, 0.6) / np.linalg.norm(x)
        p = 40
        s = np.sum(oracle.upsilon(x, p) * np.conj(oracle.theta(r, p)))
        want = 1.0 / np.linalg.norm(r - x)
        assert abs(s.imag) < 1e-14
        assert abs(s.real - want) <= 1e-12 * want


def test_harmonic_laplacian_zero():
    """Theta and Upsilon are harmonic: a 7-point finite-difference Laplacian vanishes."""
    p, h = 8, 1e-3
    r0 = np.array([0.7, -0.4, 1.1])
    for fn in (oracle.theta, oracle.upsilon):
        centre = fn(r0, p)
        lap = -6.0 * centre
        for d in range(3):
            for s in (-1.0, 1.0):
                e = np.zeros(3)
                e[d] = s * h
                lap = lap + fn(r0 + e, p)
        lap /= h * h
        scale = np.abs(centre) / np.dot(r0, r0) + 1e-12
        assert np.all(np.abs(lap) <= 1e-4 * scale.max() * 50)


def test_theta_is_derivative_of_inverse_r():
    """Theta_1^m from the operator definition (eq:The:def): Theta_1^0 = z/r^3,
    Theta_1^1 = (x + i y)/r^3."""
    r = np.array([0.3, -0.5, 0.8])
    d = np.linalg.norm(r)
    T = oracle.theta(r, 1)
    assert T[oracle.idx(1, 0)] == pytest.approx(r[2] / d ** 3, rel=1e-15)
    assert T[oracle.idx(1, 1)] == pytest.approx((r[0] + 1j * r[1]) / d ** 3, rel=1e-15)
