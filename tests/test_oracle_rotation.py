"""Pins of the oracle's swap matrices and rotation-accelerated M2L (App. A,
fast rotations and a fast M2L kernel) against what the paper prints and what
the mathematics fixes (no GPU)."""
import numpy as np
import pytest

import oracle
from conftest import golden_path


def _fixture():
    blocks, cur = {}, None
    with open(golden_path("swap_b4.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line in ("complex", "real"):
                cur = blocks.setdefault(line, [])
                continue
            cur.append([int(v) for v in line.split()])
    return np.array(blocks["complex"]), np.array(blocks["real"])


def _swapped(r):
    return np.array([r[2], r[1], r[0]])


def _deg(X, n):
    return np.array([X[oracle.idx(n, m)] for m in range(-n, n + 1)])


def test_b4_matches_the_printed_complex_matrix():
    want, _ = _fixture()
    assert np.array_equal(oracle.swap_matrix(4) * 16, want)


def test_printed_real_matrix_is_the_swap_of_T4():
    """The paper's real-basis matrix maps T_4^m(x,y,z) to T_4^m(z,y,x): fitted
    from the harmonics at random points, independent of the recurrence."""
    _, want = _fixture()
    rng = np.random.default_rng(5)

    def t4(r):
        T = oracle.theta(r, 4)
        return np.array([T[oracle.idx(4, abs(m))].imag if m < 0 else T[oracle.idx(4, m)].real
                         for m in range(-4, 5)])

    pts = rng.normal(size=(40, 3))
    A = np.array([t4(r) for r in pts])
    Y = np.array([t4(_swapped(r)) for r in pts])
    R = np.linalg.lstsq(A, Y, rcond=None)[0].T
    assert np.allclose(R * 8, want, atol=1e-9)


@pytest.mark.parametrize("n", range(0, 13))
def test_swap_identities_theta_and_upsilon(n):
    """Theta_n(r~) = B_n Theta_n(r) (eq:Ylm:swap) and Upsilon_n(r~) = B_n^T
    Upsilon_n(r), r~ the point with x and z exchanged."""
    B = oracle.swap_matrix(n)
    rng = np.random.default_rng(n)
    for _ in range(4):
        r = rng.normal(size=3)
        t, ts = _deg(oracle.theta(r, n), n), _deg(oracle.theta(_swapped(r), n), n)
        u, us = _deg(oracle.upsilon(r, n), n), _deg(oracle.upsilon(_swapped(r), n), n)
        assert np.abs(B @ t - ts).max() <= 1e-13 * np.abs(ts).max()
        assert np.abs(B.T @ u - us).max() <= 1e-13 * np.abs(us).max()


def test_swap_is_an_involution_and_both_recurrences_agree():
    for n in range(0, 21):
        B = oracle.swap_matrix(n)
        assert np.abs(B @ B - np.eye(2 * n + 1)).max() < 1e-9 * max(1.0, np.abs(B).max())
        if n == 0:
            continue
        P = np.pad(oracle.swap_matrix(n - 1), 1)     # B_{n-1} on the index range of B_n
        # the second relation of the paper, used by the oracle only for the two
        # new rows, also holds for every interior row
        for m in range(-(n - 1), n):
            for s in (+1, -1):
                if abs(m + s) > n - 1:
                    continue
                for l in range(-n, n + 1):
                    lo = P[m + n, l - 1 + n] if l - 1 >= -n else 0.0
                    hi = P[m + n, l + 1 + n] if l + 1 <= n else 0.0
                    assert 2 * B[m + s + n, l + n] == pytest.approx(
                        lo + hi + 2 * s * P[m + n, l + n], abs=1e-9)


def _multipoles(rng, p, k=12):
    return oracle.p2m(rng.normal(size=(k, 3)) * 0.4, rng.uniform(0.1, 1.0, k), np.zeros(3), p)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 10, 12, 13, 15, 16, 18, 20])
def test_rotation_m2l_equals_direct_m2l(p):
    rng = np.random.default_rng(100 + p)
    dirs = [rng.normal(size=3) for _ in range(4)] + [
        np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, -1.0]), np.array([1.0, -2.0, 0.0]),
        np.array([1e-9, 0.0, 1.0]), np.array([0.0, 1.0, -1e-12])]
    for d in dirs:
        r = 3.0 * d / np.linalg.norm(d)
        M = _multipoles(rng, p)
        a = oracle.m2l(M, r, p)
        b = oracle.m2l_rot(M, r, p)
        # rounding: the swap matrices grow with n (entries up to ~3e5 at
        # n = 20), so at high order and along the z axis (where the two swaps
        # cancel exactly in theory) the difference reaches a few 1e-12
        assert np.abs(a - b).max() <= 2e-11 * np.abs(a).max()
        # the symmetry F^-m = (-1)^m conj(F^m) of a local expansion holds
        for n in range(p + 1):
            for m in range(1, n + 1):
                assert b[oracle.idx(n, -m)] == pytest.approx(
                    (-1) ** m * np.conj(b[oracle.idx(n, m)]), abs=2e-11 * np.abs(b).max())
