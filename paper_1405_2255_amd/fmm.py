"""Python binding of libfmm (include/fmm.h): argument marshalling only.

Every stage of the force evaluation runs in the HIP kernels of libfmm.so;
torch supplies the device memory and the stream.  Importing this module
loads the in-tree library and raises if it has not been built, so no code
path can silently fall back to something else.

    from paper_1405_2255_amd import fmm
    ctx = fmm.Context()                      # on cuda:0, torch's current stream
    pot, acc = ctx.forces(pos, mass, target_err=1e-7)   # float64 CUDA tensors
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1405_2255_amd.build`")

_lib = C.CDLL(LIB_PATH)

# ---- fmm.h mirror ----------------------------------------------------------
OK, E_INVAL, E_NOMEM, E_HIP, E_NONFINITE, E_UNSUPPORTED, E_BUSY = range(7)
MAC_REL, MAC_SCALED, MAC_THETA = 0, 1, 2
SCALE_ESTIMATE, SCALE_PREVIOUS = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
M2L_AUTO, M2L_DIRECT, M2L_ROTATION = 0, 1, 2
CENTRE_AUTO, CENTRE_MIDPOINT, CENTRE_ENCLOSING = 0, 1, 2
EXPORT_M2L, EXPORT_P2P, EXPORT_SCALE, EXPORT_CELLS, EXPORT_CENTRES = 1, 2, 3, 4, 5
P_MAX = 20
P_MIN, P_MIN_MIXED = 3, 2   # lowest accepted orders (FP64 and jerk calls; mixed precision)

STATUS_NAMES = {OK: "FMM_OK", E_INVAL: "FMM_E_INVAL", E_NOMEM: "FMM_E_NOMEM", E_HIP: "FMM_E_HIP",
                E_NONFINITE: "FMM_E_NONFINITE", E_UNSUPPORTED: "FMM_E_UNSUPPORTED",
                E_BUSY: "FMM_E_BUSY"}

SYMBOLS = ["fmm_build", "fmm_forces", "fmm_forces_batched", "fmm_forces_refit",
           "fmm_forces_active", "fmm_forces_eps", "fmm_forces_jerk", "fmm_forces_jerk_active", "fmm_direct",
           "fmm_direct_sinks", "fmm_direct_sinks_noalloc", "fmm_direct_jerk_sinks",
           "fmm_order_for_error", "fmm_stats", "fmm_footprint_bytes", "fmm_last_error",
           "fmm_destroy", "fmm_export"]


class Opts(C.Structure):
    _fields_ = [("device", C.c_int), ("hip_stream", C.c_void_p), ("leaf_size", C.c_int),
                ("mac", C.c_int), ("theta_crit", C.c_double), ("p2p_factor", C.c_double),
                ("scale_source", C.c_int), ("timing", C.c_int), ("precision", C.c_int),
                ("m2l_kernel", C.c_int), ("centre", C.c_int), ("n_max", C.c_int64),
                ("p_max", C.c_int), ("hbm_budget_bytes", C.c_size_t)]


class Stats(C.Structure):
    _fields_ = [("p", C.c_int), ("n", C.c_int64), ("n_cells", C.c_int64),
                ("n_leaves", C.c_int64), ("depth", C.c_int), ("n_m2l", C.c_int64),
                ("n_p2p_lists", C.c_int64), ("n_p2p_pairs", C.c_int64),
                ("n_est_m2l", C.c_int64), ("n_est_p2p_pairs", C.c_int64),
                ("walk_iterations", C.c_int),
                ("t_tree", C.c_double), ("t_estimate", C.c_double), ("t_up", C.c_double),
                ("t_walk", C.c_double), ("t_m2l", C.c_double), ("t_p2p", C.c_double),
                ("t_down", C.c_double), ("t_total", C.c_double),
                ("t_m2l_kernel", C.c_double), ("t_p2p_kernel", C.c_double),
                ("m2l_launches", C.c_int), ("p2p_launches", C.c_int),
                ("walk_pairs", C.c_int64), ("est_walk_pairs", C.c_int64),
                ("t_sweeps", C.c_double), ("t_est_sweeps", C.c_double),
                ("refitted", C.c_int), ("m2l_rotation", C.c_int)]


_P = C.c_void_p
_lib.fmm_build.argtypes = [C.POINTER(_P), C.POINTER(Opts)]
_lib.fmm_build.restype = C.c_int
_lib.fmm_forces.argtypes = [_P, C.c_int64, _P, _P, C.c_double, C.c_int, C.c_double, _P, _P]
_lib.fmm_forces.restype = C.c_int
_lib.fmm_forces_batched.argtypes = [_P, C.c_int64, _P, _P, _P, C.c_double, C.c_int, C.c_double,
                                    _P, _P]
_lib.fmm_forces_batched.restype = C.c_int
_lib.fmm_forces_refit.argtypes = [_P, C.c_int64, _P, _P, C.c_double, C.c_int, C.c_double, _P,
                                  _P]
_lib.fmm_forces_refit.restype = C.c_int
_lib.fmm_forces_active.argtypes = [_P, C.c_int64, _P, _P, C.c_double, C.c_int, C.c_double,
                                   C.c_int64, _P, C.c_int, _P, _P]
_lib.fmm_forces_active.restype = C.c_int
_lib.fmm_forces_eps.argtypes = [_P, C.c_int64, _P, _P, C.c_double, C.c_int, _P, _P, _P]
_lib.fmm_forces_eps.restype = C.c_int
_lib.fmm_forces_jerk.argtypes = [_P, C.c_int64, _P, _P, _P, C.c_double, C.c_int, C.c_double,
                                 _P, _P, _P]
_lib.fmm_forces_jerk.restype = C.c_int
_lib.fmm_forces_jerk_active.argtypes = [_P, C.c_int64, _P, _P, _P, C.c_double, C.c_int,
                                        C.c_double, C.c_int64, _P, C.c_int, _P, _P, _P]
_lib.fmm_forces_jerk_active.restype = C.c_int
_lib.fmm_direct_jerk_sinks.argtypes = [_P, C.c_int64, _P, _P, _P, C.c_double, C.c_int64, _P, _P]
_lib.fmm_direct_jerk_sinks.restype = C.c_int
_lib.fmm_direct.argtypes = [_P, C.c_int64, _P, _P, C.c_double, _P, _P]
_lib.fmm_direct.restype = C.c_int
_lib.fmm_direct_sinks.argtypes = [_P, C.c_int64, _P, _P, C.c_double, C.c_int64, _P, _P, _P]
_lib.fmm_direct_sinks.restype = C.c_int
_lib.fmm_direct_sinks_noalloc.argtypes = [_P, C.c_int64, _P, _P, C.c_double, C.c_int64, _P, _P,
                                          _P]
_lib.fmm_direct_sinks_noalloc.restype = C.c_int
_lib.fmm_order_for_error.argtypes = [C.c_double]
_lib.fmm_order_for_error.restype = C.c_int
_lib.fmm_stats.argtypes = [_P, C.POINTER(Stats)]
_lib.fmm_stats.restype = C.c_int
_lib.fmm_footprint_bytes.argtypes = [C.c_int64, C.c_int, C.POINTER(Opts)]
_lib.fmm_footprint_bytes.restype = C.c_size_t
_lib.fmm_last_error.argtypes = [_P]
_lib.fmm_last_error.restype = C.c_char_p
_lib.fmm_destroy.argtypes = [_P]
_lib.fmm_destroy.restype = None
_lib.fmm_export.argtypes = [_P, C.c_int, _P, C.c_int64]
_lib.fmm_export.restype = C.c_int64


class FMMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def order_for_error(target_err: float) -> int:
    return int(_lib.fmm_order_for_error(float(target_err)))


def footprint_bytes(n: int, p: int, leaf_size: int = 0) -> int:
    o = Opts(0, None, leaf_size)
    return int(_lib.fmm_footprint_bytes(int(n), int(p), C.byref(o)))


def _dev_ptr(t: torch.Tensor, name: str, shape=None) -> int:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


_PRECISIONS = {"fp64": PREC_FP64, "mixed": PREC_MIXED}
_M2L = {"auto": M2L_AUTO, "direct": M2L_DIRECT, "rotation": M2L_ROTATION}
_MACS = {"a": MAC_REL, "rel": MAC_REL, "f": MAC_SCALED, "scaled": MAC_SCALED,
         "theta": MAC_THETA}
_SCALES = {"estimate": SCALE_ESTIMATE, "previous": SCALE_PREVIOUS}
_CENTRES = {"auto": CENTRE_AUTO, "midpoint": CENTRE_MIDPOINT, "enclosing": CENTRE_ENCLOSING}


class Context:
    """One libfmm context (fmm_build / fmm_destroy) on a device and stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None,
                 leaf_size: int = 0, mac: str = "a", theta_crit: float = 0.5,
                 p2p_factor: float = 0.0, scale_source: str = "estimate",
                 timing: bool = False, precision: str = "fp64", m2l: str = "auto",
                 centre: str = "auto", n_max: int = 0, p_max: int = 0,
                 hbm_budget_bytes: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libfmm needs a GPU")
        self.device = int(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
        o = Opts(self.device, C.c_void_p(self.stream.cuda_stream), int(leaf_size), _MACS[mac],
                 float(theta_crit), float(p2p_factor), _SCALES[scale_source], int(bool(timing)),
                 _PRECISIONS[precision], _M2L[m2l], _CENTRES[centre], int(n_max), int(p_max),
                 int(hbm_budget_bytes))
        self._opts = o
        h = C.c_void_p()
        st = _lib.fmm_build(C.byref(h), C.byref(o))
        if st != OK:
            raise FMMError(st, "fmm_build failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            raise FMMError(st, _lib.fmm_last_error(self._h).decode())

    def forces(self, pos: torch.Tensor, mass: torch.Tensor, G: float = 1.0, p: int = -1,
               target_err: float = 1e-7, pot: torch.Tensor | None = None,
               acc: torch.Tensor | None = None, refit: bool = False):
        """Potential (physical, negative) and acceleration of every particle.
        refit=True recycles the context's tree when n is unchanged."""
        n = pos.shape[0]
        if pot is None:
            pot = torch.empty(n, dtype=torch.float64, device=pos.device)
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        fn = _lib.fmm_forces_refit if refit else _lib.fmm_forces
        self._check(fn(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                    _dev_ptr(mass, "mass", (n,)), float(G), int(p),
                                    float(target_err), _dev_ptr(pot, "pot", (n,)),
                                    _dev_ptr(acc, "acc", (n, 3))))
        return pot, acc

    def forces_batched(self, offsets, pos, mass, G: float = 1.0, p: int = -1,
                       target_err: float = 1e-7, pot=None, acc=None):
        """Independent clusters [offsets[i], offsets[i+1]) in one call."""
        import numpy as np
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        n = pos.shape[0]
        if off[-1] != n:
            raise ValueError("offsets[-1] must equal the number of particles")
        if pot is None:
            pot = torch.empty(n, dtype=torch.float64, device=pos.device)
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_forces_batched(self._h, off.shape[0] - 1,
                                            off.ctypes.data_as(C.c_void_p),
                                            _dev_ptr(pos, "pos", (n, 3)),
                                            _dev_ptr(mass, "mass", (n,)), float(G), int(p),
                                            float(target_err), _dev_ptr(pot, "pot", (n,)),
                                            _dev_ptr(acc, "acc", (n, 3))))
        return pot, acc

    def forces_active(self, pos: torch.Tensor, mass: torch.Tensor, active: torch.Tensor,
                      G: float = 1.0, p: int = -1, target_err: float = 1e-7,
                      refit: bool = False):
        """Potential and acceleration of the listed particles (int64 CUDA
        tensor of input indices), in list order; equal to forces() for them."""
        n = pos.shape[0]
        if not isinstance(active, torch.Tensor) or active.dtype != torch.int64 or not active.is_cuda:
            raise TypeError("active must be an int64 CUDA tensor")
        active = active.contiguous()
        k = active.shape[0]
        pot = torch.empty(k, dtype=torch.float64, device=pos.device)
        acc = torch.empty((k, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_forces_active(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                           _dev_ptr(mass, "mass", (n,)), float(G), int(p),
                                           float(target_err), k, C.c_void_p(active.data_ptr()),
                                           int(bool(refit)), _dev_ptr(pot, "pot", (k,)),
                                           _dev_ptr(acc, "acc", (k, 3))))
        return pot, acc

    def forces_eps(self, pos: torch.Tensor, mass: torch.Tensor, eps_particle: torch.Tensor,
                   G: float = 1.0, p: int = -1):
        """forces() with an individual accuracy parameter per particle (float64
        CUDA tensor, input order)."""
        n = pos.shape[0]
        pot = torch.empty(n, dtype=torch.float64, device=pos.device)
        acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_forces_eps(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                        _dev_ptr(mass, "mass", (n,)), float(G), int(p),
                                        _dev_ptr(eps_particle, "eps_particle", (n,)),
                                        _dev_ptr(pot, "pot", (n,)), _dev_ptr(acc, "acc", (n, 3))))
        return pot, acc

    def forces_jerk(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                    G: float = 1.0, p: int = -1, target_err: float = 1e-6):
        """forces() plus the jerk da/dt for particles moving with vel (float64
        CUDA tensor (n, 3)): returns (pot, acc, jerk)."""
        n = pos.shape[0]
        pot = torch.empty(n, dtype=torch.float64, device=pos.device)
        acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        jerk = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_forces_jerk(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                         _dev_ptr(vel, "vel", (n, 3)),
                                         _dev_ptr(mass, "mass", (n,)), float(G), int(p),
                                         float(target_err), _dev_ptr(pot, "pot", (n,)),
                                         _dev_ptr(acc, "acc", (n, 3)),
                                         _dev_ptr(jerk, "jerk", (n, 3))))
        return pot, acc, jerk

    def forces_jerk_active(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                           active: torch.Tensor, G: float = 1.0, p: int = -1,
                           target_err: float = 1e-6, refit: bool = False):
        """forces_jerk() for the listed sinks only (int64 CUDA tensor of input
        indices): (pot, acc, jerk) in list order."""
        n = pos.shape[0]
        if not isinstance(active, torch.Tensor) or active.dtype != torch.int64 or not active.is_cuda:
            raise TypeError("active must be an int64 CUDA tensor")
        active = active.contiguous()
        k = active.shape[0]
        pot = torch.empty(k, dtype=torch.float64, device=pos.device)
        acc = torch.empty((k, 3), dtype=torch.float64, device=pos.device)
        jerk = torch.empty((k, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_forces_jerk_active(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                                _dev_ptr(vel, "vel", (n, 3)),
                                                _dev_ptr(mass, "mass", (n,)), float(G), int(p),
                                                float(target_err), k,
                                                C.c_void_p(active.data_ptr()), int(bool(refit)),
                                                _dev_ptr(pot, "pot", (k,)),
                                                _dev_ptr(acc, "acc", (k, 3)),
                                                _dev_ptr(jerk, "jerk", (k, 3))))
        return pot, acc, jerk

    def direct(self, pos: torch.Tensor, mass: torch.Tensor, G: float = 1.0):
        """Exact FP64 all-pairs direct summation on the GPU."""
        n = pos.shape[0]
        pot = torch.empty(n, dtype=torch.float64, device=pos.device)
        acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_direct(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                    _dev_ptr(mass, "mass", (n,)), float(G),
                                    _dev_ptr(pot, "pot", (n,)), _dev_ptr(acc, "acc", (n, 3))))
        return pot, acc

    def direct_sinks(self, pos: torch.Tensor, mass: torch.Tensor, sinks: torch.Tensor,
                     G: float = 1.0, pot: torch.Tensor | None = None,
                     acc: torch.Tensor | None = None, noalloc: bool = False):
        """Exact FP64 direct sum for the listed sinks (int64 CUDA tensor).
        noalloc: through fmm_direct_sinks_noalloc (no device allocation by the
        library; pass pot and acc to avoid torch's own allocations too)."""
        n = pos.shape[0]
        if not isinstance(sinks, torch.Tensor) or sinks.dtype != torch.int64 or not sinks.is_cuda:
            raise TypeError("sinks must be an int64 CUDA tensor")
        sinks = sinks.contiguous()
        k = sinks.shape[0]
        if pot is None:
            pot = torch.empty(k, dtype=torch.float64, device=pos.device)
        if acc is None:
            acc = torch.empty((k, 3), dtype=torch.float64, device=pos.device)
        fn = _lib.fmm_direct_sinks_noalloc if noalloc else _lib.fmm_direct_sinks
        self._check(fn(self._h, n, _dev_ptr(pos, "pos", (n, 3)), _dev_ptr(mass, "mass", (n,)),
                       float(G), k, C.c_void_p(sinks.data_ptr()), _dev_ptr(pot, "pot", (k,)),
                       _dev_ptr(acc, "acc", (k, 3))))
        return pot, acc

    def direct_jerk_sinks(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor,
                          sinks: torch.Tensor, G: float = 1.0):
        """Exact FP64 jerk of the listed sinks (int64 CUDA tensor)."""
        n = pos.shape[0]
        if not isinstance(sinks, torch.Tensor) or sinks.dtype != torch.int64 or not sinks.is_cuda:
            raise TypeError("sinks must be an int64 CUDA tensor")
        sinks = sinks.contiguous()
        k = sinks.shape[0]
        jerk = torch.empty((k, 3), dtype=torch.float64, device=pos.device)
        self._check(_lib.fmm_direct_jerk_sinks(self._h, n, _dev_ptr(pos, "pos", (n, 3)),
                                               _dev_ptr(vel, "vel", (n, 3)),
                                               _dev_ptr(mass, "mass", (n,)), float(G), k,
                                               C.c_void_p(sinks.data_ptr()),
                                               _dev_ptr(jerk, "jerk", (k, 3))))
        return jerk

    def stats(self) -> dict:
        s = Stats()
        self._check(_lib.fmm_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def _export(self, what: int, dtype):
        import numpy as np
        nbytes = _lib.fmm_export(self._h, what, None, 0)
        if nbytes < 0:
            raise FMMError(E_INVAL, "export failed")
        buf = np.empty(nbytes // np.dtype(dtype).itemsize, dtype=dtype)
        got = _lib.fmm_export(self._h, what, buf.ctypes.data_as(C.c_void_p), nbytes)
        if got != nbytes:
            raise FMMError(E_INVAL, "export size changed")
        return buf

    def export_m2l(self):
        """(source id, sink id) of every M2L interaction, id = level << 40 | begin."""
        import numpy as np
        return self._export(EXPORT_M2L, np.int64).reshape(-1, 2)

    def export_p2p(self):
        """(sink id, first, end) of every direct-sum entry: source particle
        range [first, end) in Morton order."""
        import numpy as np
        return self._export(EXPORT_P2P, np.int64).reshape(-1, 3)

    def export_scale(self):
        import numpy as np
        return self._export(EXPORT_SCALE, np.float64)

    def export_cells(self):
        """(id, end) per cell."""
        import numpy as np
        return self._export(EXPORT_CELLS, np.int64).reshape(-1, 2)

    def export_centres(self):
        """(x, y, z, rho) per cell, cell order: expansion centre and radius."""
        import numpy as np
        return self._export(EXPORT_CENTRES, np.float64).reshape(-1, 4)
