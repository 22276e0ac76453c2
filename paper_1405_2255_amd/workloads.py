"""Seeded synthetic inputs: star-cluster samples with the shapes of the paper's
workloads (Plummer spheres without outer truncation, Dehnen gamma-models,
uniform spheres, power-law mass functions).

This module holds no arithmetic of the multipole method.  It only draws
particle positions, velocities and masses, in float64 numpy arrays, from a
numpy PCG64 generator seeded by the caller.  Both the HIP path's tests and the
CPU oracle's tests take their inputs from here, so that the two sides see the
same numbers.

Units: G = 1, total mass M = 1, scale radius a = 1 unless stated.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "plummer",
    "dehnen",
    "uniform_sphere",
    "salpeter_masses",
    "cluster",
    "log_uniform_sizes",
    "drift_velocities",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _open_uniform(rng: np.random.Generator, n: int) -> np.ndarray:
    """U(0,1) excluding both end points."""
    u = rng.random(n)
    tiny = np.finfo(np.float64).tiny
    return np.clip(u, tiny, 1.0 - 2.0**-53)


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    n = r.shape[0]
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
    return np.stack([r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth], axis=1)


def plummer(n: int, seed: int, *, a: float = 1.0, with_velocities: bool = False):
    """Plummer (1911) sphere of total mass 1, untruncated.

    Radii from inverting the cumulative mass M(<r) = r^3 / (r^2 + a^2)^{3/2}:
    r = a (X^{-2/3} - 1)^{-1/2}, X uniform on (0,1).  Isotropic directions.
    Velocities (optional) by the rejection method of Aarseth, Henon & Wielen
    (1974): speed q * v_esc with q drawn from g(q) = q^2 (1-q^2)^{7/2}.
    Returns pos (n,3) [, vel (n,3)], float64.
    """
    rng = _rng(seed)
    x = _open_uniform(rng, n)
    r = a / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, r)
    if not with_velocities:
        return pos
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = rng.random(todo.size)
        x2 = rng.random(todo.size) * 0.1
        ok = x2 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (1.0 + (r / a) ** 2) ** -0.25 / np.sqrt(a)
    vel = _isotropic(rng, q * vesc)
    return pos, vel


def dehnen(n: int, seed: int, gamma: float, *, a: float = 1.0):
    """Dehnen (1993) gamma-model of total mass 1: M(<r) = (r/(r+a))^{3-gamma}.

    Inverting at X uniform on (0,1): with u = X^{1/(3-gamma)}, r = a u/(1-u).
    """
    rng = _rng(seed)
    x = _open_uniform(rng, n)
    u = x ** (1.0 / (3.0 - gamma))
    r = a * u / (1.0 - u)
    return _isotropic(rng, r)


def uniform_sphere(n: int, seed: int, *, radius: float = 1.0):
    """Homogeneous ball: r = R X^{1/3}."""
    rng = _rng(seed)
    x = _open_uniform(rng, n)
    return _isotropic(rng, radius * np.cbrt(x))


def salpeter_masses(n: int, seed: int, *, slope: float = 2.35,
                    m_lo: float = 0.1, m_hi: float = 100.0) -> np.ndarray:
    """Power-law mass function dN/dm ~ m^{-slope} on [m_lo, m_hi] by inverse
    CDF, normalised so the masses sum to 1."""
    rng = _rng(seed)
    x = rng.random(n)
    e = 1.0 - slope
    lo, hi = m_lo ** e, m_hi ** e
    m = (lo + x * (hi - lo)) ** (1.0 / e)
    return m / m.sum()


def cluster(kind: str, n: int, seed: int, *, masses: str = "equal"):
    """Positions (n,3) and masses (n,) of one cluster.

    kind: 'plummer', 'dehnen0', 'dehnen1', 'dehnen1.5', 'uniform'.
    masses: 'equal' (1/n each) or 'salpeter'.
    """
    if kind == "plummer":
        pos = plummer(n, seed)
    elif kind.startswith("dehnen"):
        pos = dehnen(n, seed, float(kind[len("dehnen"):]))
    elif kind == "uniform":
        pos = uniform_sphere(n, seed)
    else:
        raise ValueError(f"unknown cluster kind {kind!r}")
    if masses == "equal":
        m = np.full(n, 1.0 / max(n, 1))
    elif masses == "salpeter":
        m = salpeter_masses(n, seed + 7919)
    else:
        raise ValueError(f"unknown mass function {masses!r}")
    return np.ascontiguousarray(pos), np.ascontiguousarray(m)


def log_uniform_sizes(k: int, seed: int, lo: float, hi: float) -> np.ndarray:
    """k integers round(10^U(log10 lo, log10 hi))."""
    rng = _rng(seed)
    return np.rint(10.0 ** rng.uniform(np.log10(lo), np.log10(hi), k)).astype(np.int64)


def _enclosed_mass(kind: str, r: np.ndarray) -> np.ndarray:
    if kind == "plummer":
        return r ** 3 / (r * r + 1.0) ** 1.5
    if kind.startswith("dehnen"):
        g = float(kind[len("dehnen"):])
        return (r / (r + 1.0)) ** (3.0 - g)
    if kind == "uniform":
        return np.minimum(r, 1.0) ** 3
    raise ValueError(f"unknown cluster kind {kind!r}")


def drift_velocities(kind: str, pos: np.ndarray, seed: int) -> np.ndarray:
    """Velocities for drift steps: an isotropic Gaussian whose 1-D dispersion
    is the local circular speed over sqrt(3), sigma^2 = M(<r) / (3 r) (G = 1,
    total mass 1).  They only move particles between force evaluations; the
    force metric does not depend on them."""
    rng = _rng(seed)
    r = np.sqrt(np.einsum("ij,ij->i", pos, pos))
    sig = np.sqrt(_enclosed_mass(kind, r) / (3.0 * np.maximum(r, 1e-300)))
    return sig[:, None] * rng.standard_normal((pos.shape[0], 3))
