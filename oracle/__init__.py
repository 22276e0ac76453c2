"""CPU oracle for Dehnen's fast multipole method (test infrastructure only).

This package is the reference the GPU path is checked against: a plain FP64
direct summation (the exact result, eq. (1) and eq:f) and a plain recursive
FMM following the paper's phases.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library under
``paper_1405_2255_amd`` never does.  It shares no code with that library.

Functions take and return numpy float64 arrays.  Complex harmonic arrays have
(p+1)^2 entries at index n*n + n + m, -n <= m <= n.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        d, i64, ip = C.c_double, C.c_int64, C.c_int
        P = C.c_void_p
        _lib.or_direct.argtypes = [i64, P, P, d, i64, P, ip, P, P, P]
        _lib.or_direct.restype = ip
        _lib.or_direct_jerk.argtypes = [i64, P, P, P, d, i64, P, ip, P]
        _lib.or_direct_jerk.restype = ip
        _lib.or_upsilon_dot.argtypes = [P, P, ip, P]
        _lib.or_upsilon_dot.restype = None
        _lib.or_p2m_dot.argtypes = [i64, P, P, P, P, ip, P]
        _lib.or_p2m_dot.restype = None
        _lib.or_l2p_dot.argtypes = [P, P, P, P, ip, P]
        _lib.or_l2p_dot.restype = None
        for name in ("or_theta", "or_upsilon"):
            getattr(_lib, name).argtypes = [P, ip, P]
            getattr(_lib, name).restype = None
        _lib.or_p2m.argtypes = [i64, P, P, P, ip, P]
        _lib.or_m2m.argtypes = [P, P, ip, P]
        _lib.or_m2l.argtypes = [P, P, ip, P]
        _lib.or_m2l_rot.argtypes = [P, P, ip, P]
        _lib.or_m2l_rot.restype = None
        _lib.or_swap_matrix.argtypes = [ip, P]
        _lib.or_swap_matrix.restype = None
        _lib.or_l2l.argtypes = [P, P, ip, P]
        _lib.or_l2p.argtypes = [P, P, ip, P, P]
        _lib.or_power.argtypes = [P, ip, P]
        _lib.or_eab_times_mass.argtypes = [P, ip, d, d]
        _lib.or_eab_times_mass.restype = d
        _lib.or_etilde_factor.argtypes = [d, d]
        _lib.or_etilde_factor.restype = d
        _lib.or_fmm.argtypes = [P, i64, P, P, P, P, P, P]
        _lib.or_fmm.restype = ip
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def ncoef(p: int) -> int:
    return (p + 1) * (p + 1)


def idx(n: int, m: int) -> int:
    return n * n + n + m


# --------------------------------------------------------------- direct sum

def direct(pos, mass, G: float = 1.0, sinks=None, threads: int | None = None):
    """Exact FP64 direct sum (compensated).  Returns (pot, acc, f) for the
    sinks (all particles when sinks is None), pot = physical potential."""
    lib = _load()
    pos = _f64(pos)
    mass = _f64(mass)
    n = mass.shape[0]
    assert pos.shape == (n, 3)
    if sinks is not None:
        sinks = np.ascontiguousarray(sinks, dtype=np.int64)
        ns = sinks.shape[0]
    else:
        ns = n
    if threads is None:
        threads = max(1, len(os.sched_getaffinity(0)))
    pot = np.empty(ns)
    acc = np.empty((ns, 3))
    f = np.empty(ns)
    rc = lib.or_direct(n, _ptr(pos), _ptr(mass), float(G), ns, _ptr(sinks), int(threads),
                       _ptr(pot), _ptr(acc), _ptr(f))
    if rc != 0:
        raise ValueError("or_direct: bad arguments")
    return pot, acc, f


def direct_jerk(pos, vel, mass, G: float = 1.0, sinks=None, threads: int | None = None):
    """Exact FP64 jerk (time derivative of the direct-sum acceleration for
    particles moving with vel), compensated sums; (nsinks, 3)."""
    lib = _load()
    pos = _f64(pos)
    vel = _f64(vel)
    mass = _f64(mass)
    n = mass.shape[0]
    assert pos.shape == (n, 3) and vel.shape == (n, 3)
    if sinks is not None:
        sinks = np.ascontiguousarray(sinks, dtype=np.int64)
        ns = sinks.shape[0]
    else:
        ns = n
    if threads is None:
        threads = max(1, len(os.sched_getaffinity(0)))
    jerk = np.empty((ns, 3))
    rc = lib.or_direct_jerk(n, _ptr(pos), _ptr(vel), _ptr(mass), float(G), ns, _ptr(sinks),
                            int(threads), _ptr(jerk))
    if rc != 0:
        raise ValueError("or_direct_jerk: bad arguments")
    return jerk


# ----------------------------------------------------------- harmonics/kernels

def theta(r, p: int) -> np.ndarray:
    r = _f64(r, (3,))
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_theta(_ptr(r), p, _ptr(out))
    return out


def upsilon(r, p: int) -> np.ndarray:
    r = _f64(r, (3,))
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_upsilon(_ptr(r), p, _ptr(out))
    return out


def p2m(pos, mass, z, p: int) -> np.ndarray:
    pos = _f64(pos)
    mass = _f64(mass)
    z = _f64(z, (3,))
    M = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_p2m(mass.shape[0], _ptr(pos), _ptr(mass), _ptr(z), p, _ptr(M))
    return M


def m2m(M, z_minus_zp, p: int) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_m2m(_ptr(M), _ptr(_f64(z_minus_zp, (3,))), p, _ptr(out))
    return out


def m2l(M, sB_minus_zA, p: int) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_m2l(_ptr(M), _ptr(_f64(sB_minus_zA, (3,))), p, _ptr(out))
    return out


def m2l_rot(M, sB_minus_zA, p: int) -> np.ndarray:
    """eq:M2L by the rotation-accelerated kernel of App. A (eq:M2L:z)."""
    M = np.ascontiguousarray(M, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_m2l_rot(_ptr(M), _ptr(_f64(sB_minus_zA, (3,))), p, _ptr(out))
    return out


def swap_matrix(n: int) -> np.ndarray:
    """B_n of eq:Ylm:swap (x <-> z), rows and columns m = -n..n."""
    out = np.zeros((2 * n + 1, 2 * n + 1))
    _load().or_swap_matrix(n, _ptr(out))
    return out


def upsilon_dot(r, v, p: int) -> np.ndarray:
    r = _f64(r, (3,))
    v = _f64(v, (3,))
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_upsilon_dot(_ptr(r), _ptr(v), p, _ptr(out))
    return out


def p2m_dot(pos, vel, mass, z, p: int) -> np.ndarray:
    pos = _f64(pos)
    vel = _f64(vel)
    mass = _f64(mass)
    z = _f64(z, (3,))
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_p2m_dot(mass.shape[0], _ptr(pos), _ptr(vel), _ptr(mass), _ptr(z), p, _ptr(out))
    return out


def l2p_dot(F, Fd, sB_minus_x, v, p: int) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.complex128)
    Fd = np.ascontiguousarray(Fd, dtype=np.complex128)
    d = _f64(sB_minus_x, (3,))
    v = _f64(v, (3,))
    j = np.zeros(3)
    _load().or_l2p_dot(_ptr(F), _ptr(Fd), _ptr(d), _ptr(v), p, _ptr(j))
    return j


def l2l(F, s_minus_sp, p: int) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().or_l2l(_ptr(F), _ptr(_f64(s_minus_sp, (3,))), p, _ptr(out))
    return out


def l2p(F, sB_minus_x, p: int):
    """Returns (Psi_0^0, a) - the negative potential and the acceleration."""
    F = np.ascontiguousarray(F, dtype=np.complex128)
    psi = np.zeros(1)
    acc = np.zeros(3)
    _load().or_l2p(_ptr(F), _ptr(_f64(sB_minus_x, (3,))), p, _ptr(psi), _ptr(acc))
    return float(psi[0]), acc


def power(M, p: int) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.complex128)
    P = np.zeros(p + 1)
    _load().or_power(_ptr(M), p, _ptr(P))
    return P


def eab_times_mass(P, p: int, rho_sB: float, r: float) -> float:
    P = _f64(P)
    return float(_load().or_eab_times_mass(_ptr(P), p, float(rho_sB), float(r)))


def etilde_factor(rho_zA: float, rho_sB: float) -> float:
    return float(_load().or_etilde_factor(float(rho_zA), float(rho_sB)))


# ---------------------------------------------------------------- plain FMM

MAC_A, MAC_F, MAC_THETA = 0, 1, 2
CENTRE_MIDPOINT, CENTRE_ENCLOSING = 0, 1


class _Params(C.Structure):
    _fields_ = [("p", C.c_int), ("eps", C.c_double), ("leaf_size", C.c_int),
                ("mac", C.c_int), ("theta_crit", C.c_double), ("p2p_pairs", C.c_double),
                ("scale_source", C.c_int), ("scale", C.c_void_p), ("G", C.c_double),
                ("eps_particle", C.c_void_p), ("adaptive_order", C.c_int),
                ("vel", C.c_void_p), ("jerk", C.c_void_p), ("centre", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n_cells", "n_leaves", "depth", "n_m2l", "n_p2p_cells", "n_p2p_pairs",
        "n_est_m2l", "n_est_p2p_pairs", "m2l_order_sum", "m2l_macs")]


class _Lists(C.Structure):
    _fields_ = [("m2l", C.c_void_p), ("m2l_cap", C.c_int64), ("m2l_count", C.c_int64),
                ("p2p", C.c_void_p), ("p2p_cap", C.c_int64), ("p2p_count", C.c_int64),
                ("scale_est", C.c_void_p), ("cell_ids", C.c_void_p),
                ("cell_geo", C.c_void_p), ("cell_cap", C.c_int64), ("cell_count", C.c_int64),
                ("order", C.c_void_p)]


def fmm(pos, mass, *, p: int, eps: float, leaf_size: int, G: float = 1.0,
        mac: int = MAC_A, theta_crit: float = 0.5, p2p_pairs: float = 0.0,
        scale=None, want_lists: bool = False, list_cap: int = 1 << 22, eps_particle=None,
        adaptive_order: int = 0, vel=None, centre: int = CENTRE_ENCLOSING,
        _cell_cap: int = 0):
    """Plain CPU FMM.  Returns dict with pot, acc, stats and (optionally) the
    interaction lists (arrays of (source id, sink id), id = level<<40 | begin)
    and the per-particle sink scale used by the acceptance test.
    adaptive_order = q_min > 0: each M2L pair at the lowest order in [q_min, p]
    that passes the criterion (Sec. 7); stats["m2l_order_sum"] sums the orders.
    vel (n, 3): also out["jerk"], the time derivative of acc (Sec. 7, jerk).
    centre: CENTRE_MIDPOINT (box midpoint) or CENTRE_ENCLOSING (approximate
    smallest-enclosing-sphere centre where it gives the smaller radius,
    Sec. 5.1.1).  With want_lists, out["cells"] holds per cell (creation order)
    (id, end), out["cell_geo"] (centre x, y, z, rho, rho about the midpoint)
    and out["order"] the input index of each Morton position."""
    lib = _load()
    pos = _f64(pos)
    mass = _f64(mass)
    n = mass.shape[0]
    prm = _Params(p, eps, leaf_size, mac, theta_crit, p2p_pairs,
                  1 if scale is not None else 0, None, G, None, int(adaptive_order))
    prm.centre = int(centre)
    if scale is not None:
        scale = _f64(scale)
        prm.scale = scale.ctypes.data
    if eps_particle is not None:      # individual accuracy parameters (Sec. 7)
        eps_particle = _f64(eps_particle)
        prm.eps_particle = eps_particle.ctypes.data
    jerk = None
    if vel is not None:               # jerk (Sec. 7)
        vel = _f64(vel)
        assert vel.shape == (n, 3)
        jerk = np.zeros((n, 3))
        prm.vel = vel.ctypes.data
        prm.jerk = jerk.ctypes.data
    pot = np.zeros(n)
    acc = np.zeros((n, 3))
    st = _Stats()
    lists = None
    out = {}
    if jerk is not None:
        out["jerk"] = jerk
    if want_lists:
        m2l_buf = np.zeros((list_cap, 2), dtype=np.int64)
        p2p_buf = np.zeros((list_cap, 2), dtype=np.int64)
        sc = np.zeros(n)
        cell_cap = max(_cell_cap, 2 * n + 64)
        ids = np.zeros((cell_cap, 2), dtype=np.int64)
        geo = np.zeros((cell_cap, 5))
        order = np.zeros(n, dtype=np.int64)
        lists = _Lists(m2l_buf.ctypes.data, list_cap, 0, p2p_buf.ctypes.data, list_cap, 0,
                       sc.ctypes.data, ids.ctypes.data, geo.ctypes.data, cell_cap, 0,
                       order.ctypes.data)
    rc = lib.or_fmm(C.byref(prm), n, _ptr(pos), _ptr(mass), _ptr(pot), _ptr(acc),
                    C.byref(st), C.byref(lists) if lists is not None else None)
    if rc != 0:
        raise RuntimeError(f"or_fmm failed with {rc}")
    out["pot"], out["acc"] = pot, acc
    out["stats"] = {k: getattr(st, k) for k, _ in _Stats._fields_}
    if want_lists:
        if (lists.m2l_count > list_cap or lists.p2p_count > list_cap
                or lists.cell_count > cell_cap):
            return fmm(pos, mass, p=p, eps=eps, leaf_size=leaf_size, G=G, mac=mac,
                       theta_crit=theta_crit, p2p_pairs=p2p_pairs, scale=scale,
                       want_lists=True,
                       list_cap=int(max(list_cap, lists.m2l_count, lists.p2p_count)) + 1,
                       eps_particle=eps_particle, adaptive_order=adaptive_order, vel=vel,
                       centre=centre, _cell_cap=int(lists.cell_count))
        out["m2l"] = m2l_buf[: lists.m2l_count].copy()
        out["p2p"] = p2p_buf[: lists.p2p_count].copy()
        out["cells"] = ids[: lists.cell_count].copy()
        out["cell_geo"] = geo[: lists.cell_count].copy()
        out["order"] = order
        out["scale"] = sc
    return out


# ----------------------------------------------------------- error measures

def force_errors(acc, acc_true, f_true=None):
    """Per-particle delta a / a (and delta a / f when f is given)."""
    da = np.linalg.norm(np.asarray(acc) - np.asarray(acc_true), axis=1)
    a = np.linalg.norm(np.asarray(acc_true), axis=1)
    rel = da / a
    if f_true is None:
        return rel
    return rel, da / np.asarray(f_true)


def error_summary(e) -> dict:
    """rms, median and nearest-rank percentiles of an error sample."""
    e = np.sort(np.asarray(e, dtype=np.float64))
    n = e.shape[0]

    def pct(q):
        k = int(np.ceil(q / 100.0 * n)) - 1
        return float(e[min(max(k, 0), n - 1)])

    return {"rms": float(np.sqrt(np.mean(e * e))), "median": pct(50), "p99": pct(99),
            "p99.9": pct(99.9), "p99.99": pct(99.99), "max": float(e[-1]), "n": n}
