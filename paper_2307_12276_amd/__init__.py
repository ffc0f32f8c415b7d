"""Python binding of libadl (include/adl.h): the Leja exponential integrator
for 2D anisotropic diffusion with advection on MI355X (gfx950).

This module only marshals arguments: every step of the computation runs in
the HIP kernels of libadl.so.  PyTorch provides device memory (tensors) and
the current stream; nothing here computes on tensors.  If the library is not
built, every entry point raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadl.so")

OK, EINVAL, ENOCONV, EBOUND, ENAN, EHIP, ENOWORKSPACE = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_DIRICHLET = 0, 1
STORAGE_FP64, STORAGE_FP32_FIELDS, STORAGE_FP32_FIELDS_Y = 0, 1, 2
BOUND_GERSHGORIN, BOUND_POWER = 0, 1
QUAD2_AUGMENTED, QUAD2_TWO_SWEEP = 0, 1
LAUNCH_FIRST, LAUNCH_ONE, LAUNCH_TWO, LAUNCH_FOUR, LAUNCH_THREE = 0, 1, 2, 3, 4
MLP_PARAMS, MLP_IN, MLP_OUT, MLP_CACHE_PER_ROW = 9155, 9, 3, 201

_ERRNAMES = {EINVAL: "EINVAL", ENOCONV: "ENOCONV", EBOUND: "EBOUND", ENAN: "ENAN",
             EHIP: "EHIP", ENOWORKSPACE: "ENOWORKSPACE"}


class AdlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class LearnedInfo(ctypes.Structure):
    _fields_ = [("rho_hat", ctypes.c_double), ("alpha", ctypes.c_double), ("gershgorin", ctypes.c_double),
                ("degree_hat", ctypes.c_int), ("substeps_hat", ctypes.c_int),
                ("feats", ctypes.c_float * 9), ("x", ctypes.c_float * 9), ("y", ctypes.c_float * 3)]

    def as_dict(self):
        return {"rho_hat": self.rho_hat, "alpha": self.alpha, "gershgorin": self.gershgorin,
                "degree_hat": self.degree_hat, "substeps_hat": self.substeps_hat,
                "feats": list(self.feats), "x": list(self.x), "y": list(self.y)}


class Stats(ctypes.Structure):
    _fields_ = [("matvecs", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("max_degree", ctypes.c_int), ("last_degree", ctypes.c_int),
                ("substeps", ctypes.c_int), ("fallback", ctypes.c_int),
                ("status", ctypes.c_int), ("reserved_i", ctypes.c_int),
                ("alpha", ctypes.c_double), ("reserved", ctypes.c_double * 3)]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("matvecs", "sweeps", "max_degree", "last_degree",
                                              "substeps", "fallback", "status", "alpha")}


class BinStats(Sequence):
    """Per-bin statistics of a batched step: item i is bin i's dict (built
    on access); `array` is a NumPy structured view of all of them, for
    totals without building 256 dicts per step."""

    def __init__(self, stats):
        self._s = stats

    def __len__(self):
        return len(self._s)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self._s[j].as_dict() for j in range(*i.indices(len(self._s)))]
        return self._s[i].as_dict()

    @property
    def array(self):
        import numpy as np
        return np.ctypeslib.as_array(self._s)


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_F = ctypes.c_float
_SZ = ctypes.c_size_t
_SIG = {
    "adl_last_error": (ctypes.c_char_p, []),
    "adl_workspace_bytes": (_SZ, [_I, _I, _I, _I]),
    "adl_op_create": (_I, [_I, _I, _D, _D, _I, _I, _P, _P, _P, _P, _P, _D, _D, _P, _SZ, _P,
                           ctypes.POINTER(_P)]),
    "adl_op_destroy": (_I, [_P]),
    "adl_op_set_limits": (_I, [_P, _I, _D]),
    "adl_op_set_quad2_mode": (_I, [_P, _I]),
    "adl_op_profile": (_I, [_P, _I]),
    "adl_op_set_tiling": (_I, [_P, _I, _I]),
    "adl_op_set_term_fusion": (_I, [_P, _I]),
    "adl_op_set_streaming": (_I, [_P, _I]),
    "adl_op_set_host_wait": (_I, [_P, _I]),
    "adl_op_host_wait": (_I, [_P, ctypes.POINTER(_I)]),
    "adl_op_get_tiling": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "adl_op_profile_read": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(_D)]),
    "adl_op_profile_read_kind": (_I, [_P, _I, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong)]),
    "adl_apply": (_I, [_P, _P, _P, _P]),
    "adl_spectral_bound": (_I, [_P, _I, _I, _D, ctypes.c_uint64, ctypes.POINTER(_D),
                                ctypes.POINTER(_I), _P]),
    "adl_set_bound": (_I, [_P, _D]),
    "adl_gershgorin_bound_noalloc": (_I, [_I, _I, _D, _D, _I, _P, _P, _P, _P, _P, _D, _D, _P, _P]),
    "adl_last_power_estimate": (_I, [_P, ctypes.POINTER(_D)]),
    "adl_get_bound": (_I, [_P, ctypes.POINTER(_D)]),
    "adl_leja_phi": (_I, [_P, _I, _D, _P, _P, _D, _I, ctypes.POINTER(Stats), _P]),
    "adl_exp_midpoint_step": (_I, [_P, _P, _P, _D, _D, ctypes.POINTER(Stats), _P]),
    "adl_exp_quad2_step": (_I, [_P, _P, _P, _P, _D, _D, _D, _D, ctypes.POINTER(Stats), _P]),
    "adl_batch_workspace_bytes": (_SZ, [_I, ctypes.POINTER(_P), _I]),
    "adl_batch_create": (_I, [_I, ctypes.POINTER(_P), _P, _SZ, _I, ctypes.POINTER(_P)]),
    "adl_batch_destroy": (_I, [_P]),
    "adl_batch_set_tile_rows": (_I, [_P, _I]),
    "adl_batch_get_tile_rows": (_I, [_P, ctypes.POINTER(_I)]),
    "adl_batch_set_term_fusion": (_I, [_P, _I]),
    "adl_batch_autotune": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, _D, ctypes.POINTER(_I), _I,
                                ctypes.POINTER(_I), ctypes.POINTER(_D), _P]),
    "adl_batch_midpoint_step": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, _D, _I,
                                     ctypes.POINTER(Stats), _P]),
    "adl_field_stats": (_I, [_P, _D, _P, _P]),
    "adl_mlp_forward": (_I, [_P, _P, _P, _P, _I, _P]),
    "adl_mlp_backward": (_I, [_P, _P, _P, _P, _I, _P]),
    "adl_mlp_adam_step": (_I, [_P, _P, _P, _P, _I, _F, _F, _F, _F, _P]),
    "adl_mlp_mse_grad": (_I, [_P, _P, _P, _P, _I, _P]),
    "adl_learned_features": (_I, [ctypes.POINTER(_F), _D, ctypes.POINTER(_F)]),
    "adl_learned_targets": (_I, [ctypes.POINTER(_F), _D, _D, _I, _I, ctypes.POINTER(_F)]),
    "adl_learned_decode": (_I, [ctypes.POINTER(_F), _D, ctypes.POINTER(_F), ctypes.POINTER(_D), ctypes.POINTER(_I),
                                ctypes.POINTER(_I)]),
    "adl_learned_bound": (_I, [_P, _D, _P, _P, ctypes.POINTER(LearnedInfo), _P]),
    "adl_learned_bound_many": (_I, [_I, _P, _D, _P, _P, ctypes.POINTER(LearnedInfo), _P]),
    "adl_leja_points": (_I, [_I, ctypes.POINTER(_D)]),
    "adl_newton_coefficients": (_I, [_I, _D, _D, _I, ctypes.POINTER(_D)]),
}


def lib():
    """The loaded libadl.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libadl.so is not built (run paper_2307_12276_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return list(_SIG.keys())


def _check(code: int):
    if code != OK:
        raise AdlError(code, lib().adl_last_error().decode())


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def leja_points(n: int = 501):
    out = (ctypes.c_double * n)()
    _check(lib().adl_leja_points(n, out))
    return list(out)


def newton_coefficients(l: int, alpha: float, h: float, n: int):
    out = (ctypes.c_double * n)()
    _check(lib().adl_newton_coefficients(l, alpha, h, n, out))
    return list(out)


def gershgorin_bound_noalloc(Dxx, Dxy, Dyy, hx: float, hy: float, bc: int, alpha_out, ax=None, ay=None,
                             ax_c: float = 0.0, ay_c: float = 0.0, stream=None):
    """adl_gershgorin_bound_noalloc: the Gershgorin interval end of the
    unscaled FP64 fields [ny][nx] into alpha_out (device tensor of one FP64
    value), enqueued on the stream without allocating or synchronising."""
    import torch
    ny, nx = Dxx.shape
    shape = (ny, nx)
    _check(lib().adl_gershgorin_bound_noalloc(
        int(nx), int(ny), float(hx), float(hy), int(bc), _ptr(Dxx, torch.float64, shape, "Dxx"),
        _ptr(Dxy, torch.float64, shape, "Dxy"), _ptr(Dyy, torch.float64, shape, "Dyy"),
        _ptr(ax, torch.float64, shape, "ax"), _ptr(ay, torch.float64, shape, "ay"), float(ax_c), float(ay_c),
        _ptr(alpha_out, torch.float64, (1,), "alpha_out"), _stream(stream)))
    return alpha_out


def workspace_bytes(nx: int, ny: int, storage: int = STORAGE_FP64, max_degree: int = 0) -> int:
    return int(lib().adl_workspace_bytes(nx, ny, storage, max_degree))


class Op:
    """The operator A of one grid: owns the device workspace (a torch tensor)
    and the library handle."""

    def __init__(self, Dxx, Dxy, Dyy, hx: float, hy: float, bc: int = BC_PERIODIC,
                 storage: int = STORAGE_FP64, ax=None, ay=None, ax_c: float = 0.0,
                 ay_c: float = 0.0, stream=None):
        import torch
        ny, nx = Dxx.shape
        self.nx, self.ny, self.shape = nx, ny, (ny, nx)
        self.storage = storage
        dev = Dxx.device
        nbytes = workspace_bytes(nx, ny, storage)
        if nbytes == 0:
            raise AdlError(EINVAL, "invalid grid size or storage")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._ws_ptr = ctypes.c_void_p(aligned)
        self._ws_bytes = nbytes
        h = ctypes.c_void_p()
        f64 = torch.float64
        _check(lib().adl_op_create(nx, ny, float(hx), float(hy), int(bc), int(storage),
                                   _ptr(Dxx, f64, self.shape, "Dxx"), _ptr(Dxy, f64, self.shape, "Dxy"),
                                   _ptr(Dyy, f64, self.shape, "Dyy"), _ptr(ax, f64, self.shape, "ax"),
                                   _ptr(ay, f64, self.shape, "ay"), float(ax_c), float(ay_c),
                                   self._ws_ptr, nbytes, _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.hx, self.hy, self.bc = hx, hy, bc

    def close(self):
        if getattr(self, "handle", None):
            lib().adl_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _v(self, t, name):
        import torch
        return _ptr(t, torch.float64, self.shape, name)

    def set_limits(self, max_degree: int = 500, rho_max: float = 1600.0):
        _check(lib().adl_op_set_limits(self.handle, int(max_degree), float(rho_max)))

    def set_tiling(self, rows: int = 0, cols_per_lane: int = 0):
        _check(lib().adl_op_set_tiling(self.handle, int(rows), int(cols_per_lane)))

    def set_term_fusion(self, mode=True):
        """Newton terms per launch: True/1 the library's choice (four below
        2^20 points, else three), 2 two with LDS-staged rows, 3 two with
        register frames, 4 four, 5 three with LDS-staged rows, 6 four with
        LDS-staged rows, False/0 one."""
        m = int(mode) if not isinstance(mode, bool) else int(mode)
        _check(lib().adl_op_set_term_fusion(self.handle, m))

    def set_streaming(self, mode: int = -1):
        """Non-temporal hints on the Newton vectors: -1 auto, 0 off, 1 on."""
        _check(lib().adl_op_set_streaming(self.handle, int(mode)))

    def set_host_wait(self, spin: bool = True):
        """How the host awaits a sweep's outcome: spin on a pinned host mirror
        (True, the default) or copy the control block back and synchronise."""
        _check(lib().adl_op_set_host_wait(self.handle, int(bool(spin))))

    def host_wait(self) -> bool:
        m = ctypes.c_int()
        _check(lib().adl_op_host_wait(self.handle, ctypes.byref(m)))
        return bool(m.value)

    def get_tiling(self):
        v, r, nb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().adl_op_get_tiling(self.handle, ctypes.byref(v), ctypes.byref(r), ctypes.byref(nb)))
        return {"cols_per_lane": v.value, "rows": r.value, "nblocks": nb.value}

    def profile(self, enable: bool = True):
        _check(lib().adl_op_profile(self.handle, int(bool(enable))))

    def profile_read_kind(self, kind: int):
        """(kernel ms, launches, algorithmic bytes, Newton terms) of the timed
        Leja launches of one kind (LAUNCH_FIRST / _ONE / _TWO / _THREE / _FOUR); call
        before profile_read, which resets the counters."""
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        b = ctypes.c_double()
        t = ctypes.c_longlong()
        _check(lib().adl_op_profile_read_kind(self.handle, int(kind), ctypes.byref(ms), ctypes.byref(n),
                                              ctypes.byref(b), ctypes.byref(t)))
        return ms.value, n.value, b.value, t.value

    def profile_read(self):
        """(kernel ms, launches, algorithmic bytes) of the timed Leja launches."""
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        b = ctypes.c_double()
        _check(lib().adl_op_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def set_quad2_mode(self, mode: int):
        _check(lib().adl_op_set_quad2_mode(self.handle, int(mode)))

    def apply(self, x, y, stream=None):
        _check(lib().adl_apply(self.handle, self._v(x, "x"), self._v(y, "y"), _stream(stream)))
        return y

    def spectral_bound(self, method: int = BOUND_GERSHGORIN, max_iter: int = 2000, rtol: float = 1e-3,
                       seed: int = 0, stream=None):
        a = ctypes.c_double()
        it = ctypes.c_int()
        _check(lib().adl_spectral_bound(self.handle, int(method), int(max_iter), float(rtol),
                                        int(seed) % (1 << 64), ctypes.byref(a), ctypes.byref(it),
                                        _stream(stream)))
        return a.value, it.value

    def last_power_estimate(self) -> float:
        lam = ctypes.c_double()
        _check(lib().adl_last_power_estimate(self.handle, ctypes.byref(lam)))
        return lam.value

    def set_bound(self, alpha: float):
        _check(lib().adl_set_bound(self.handle, float(alpha)))

    def get_bound(self) -> float:
        a = ctypes.c_double()
        _check(lib().adl_get_bound(self.handle, ctypes.byref(a)))
        return a.value

    def leja_phi(self, l: int, dt: float, v, out, tol: float, max_degree: int = 0, stream=None):
        st = Stats()
        _check(lib().adl_leja_phi(self.handle, int(l), float(dt), self._v(v, "v"), self._v(out, "out"),
                                  float(tol), int(max_degree), ctypes.byref(st), _stream(stream)))
        return st.as_dict()

    def midpoint_step(self, u, S_half, dt: float, tol: float, stream=None):
        st = Stats()
        _check(lib().adl_exp_midpoint_step(self.handle, self._v(u, "u"),
                                           self._v(S_half, "S_half") if S_half is not None else None,
                                           float(dt), float(tol), ctypes.byref(st), _stream(stream)))
        return st.as_dict()

    def quad2_step(self, u, S1, S2, c1: float, c2: float, dt: float, tol: float, stream=None):
        st = Stats()
        _check(lib().adl_exp_quad2_step(self.handle, self._v(u, "u"),
                                        self._v(S1, "S1") if S1 is not None else None,
                                        self._v(S2, "S2") if S2 is not None else None,
                                        float(c1), float(c2), float(dt), float(tol), ctypes.byref(st),
                                        _stream(stream)))
        return st.as_dict()

    def learned_bound(self, dt: float, W, scratch, stream=None):
        import torch
        info = LearnedInfo()
        _check(lib().adl_learned_bound(self.handle, float(dt), _ptr(W, torch.float32, (MLP_PARAMS,), "W"),
                                       _ptr(scratch, torch.float32, None, "scratch"), ctypes.byref(info),
                                       _stream(stream)))
        return info.as_dict()

    def field_stats(self, dt: float, feats, stream=None):
        import torch
        _check(lib().adl_field_stats(self.handle, float(dt), _ptr(feats, torch.float32, (9,), "feats"),
                                     _stream(stream)))
        return feats


def learned_bound_many(ops: Sequence[Op], dt: float, W, scratch, stream=None):
    """Op.learned_bound for every op at once (one readback, one forward pass
    of the network); scratch holds >= 72 floats per op.  Returns the per-op
    info dicts."""
    import torch
    n = len(ops)
    if n < 1:
        raise AdlError(EINVAL, "no ops")
    if scratch is None or scratch.numel() < 72 * n:
        raise AdlError(EINVAL, f"scratch needs {72 * n} floats")
    arr = (ctypes.c_void_p * n)(*[o.handle.value for o in ops])
    infos = (LearnedInfo * n)()
    _check(lib().adl_learned_bound_many(n, arr, float(dt), _ptr(W, torch.float32, (MLP_PARAMS,), "W"),
                                        _ptr(scratch, torch.float32, None, "scratch"), infos, _stream(stream)))
    return [i.as_dict() for i in infos]


class Batch:
    """Many ops advanced together by one persistent launch per step."""

    def __init__(self, ops: Sequence[Op], tile_rows: int = 0):
        import torch
        self.ops = list(ops)
        n = len(self.ops)
        arr = (ctypes.c_void_p * n)(*[o.handle.value for o in self.ops])
        self._arr = arr
        nbytes = int(lib().adl_batch_workspace_bytes(n, arr, 0))
        if nbytes == 0:
            raise AdlError(EINVAL, "invalid batch")
        dev = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        h = ctypes.c_void_p()
        _check(lib().adl_batch_create(n, arr, ctypes.c_void_p(aligned), nbytes, int(tile_rows),
                                      ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().adl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def learned_bound(self, dt: float, W, scratch, stream=None):
        """learned_bound_many over the batch's ops."""
        return learned_bound_many(self.ops, dt, W, scratch, stream)

    def _ptr_arrays(self, us, S_halfs):
        import torch
        n = len(self.ops)
        up = (ctypes.c_void_p * n)(*[_ptr(u, torch.float64, o.shape, "u").value
                                     for u, o in zip(us, self.ops)])
        if S_halfs is None:
            sp = None
        else:
            sp = (ctypes.c_void_p * n)(*[(_ptr(s, torch.float64, o.shape, "S").value if s is not None else None)
                                         for s, o in zip(S_halfs, self.ops)])
        return up, sp

    def set_tile_rows(self, rows: int):
        _check(lib().adl_batch_set_tile_rows(self.handle, int(rows)))

    def get_tile_rows(self) -> int:
        r = ctypes.c_int()
        _check(lib().adl_batch_get_tile_rows(self.handle, ctypes.byref(r)))
        return r.value

    def set_term_fusion(self, mode=True):
        """Newton terms per batched launch: 3 three with LDS-staged blocks
        (the default when every bin has nx even and >= 128), True/1 two after
        a launch of the first term alone (the default otherwise), False/0 one."""
        m = int(mode) if not isinstance(mode, bool) else int(mode)
        _check(lib().adl_batch_set_term_fusion(self.handle, m))

    def autotune(self, us, S_halfs, dt: float, tol: float, candidates=(8, 16, 32), stream=None):
        up, sp = self._ptr_arrays(us, S_halfs)
        cand = (ctypes.c_int * len(candidates))(*candidates)
        best = ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().adl_batch_autotune(self.handle, up, sp, float(dt), float(tol), cand, len(candidates),
                                        ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
        return best.value, ms.value

    def bind(self, us, S_halfs):
        """Validate the bins' state vectors (and sources) once for many steps:
        midpoint_step(None, None, ...) then advances these tensors without
        checking them again (they are kept alive here; they must keep their
        storage, dtype and shape).  bind(None, None) drops them."""
        if us is None:
            self._bound = None
            return
        self._bound = (self._ptr_arrays(us, S_halfs), list(us), None if S_halfs is None else list(S_halfs))

    def midpoint_step(self, us, S_halfs, dt: float, tol: float, use_graph: bool = False,
                      stream=None):
        """One exponential midpoint step of every bin; us=None advances the
        tensors given to bind().  use_graph=True replays the step's launches
        as a captured hipGraph (the same results); eager launches are the
        default, since on this runtime a graph of the ~60 launches of a step
        took ~0.7 ms longer per step than launching them one by one."""
        n = len(self.ops)
        if us is None:
            if getattr(self, "_bound", None) is None:
                raise ValueError("no bound state: pass us and S_halfs, or call bind() first")
            up, sp = self._bound[0]
        else:
            up, sp = self._ptr_arrays(us, S_halfs)
        stats = (Stats * n)()
        _check(lib().adl_batch_midpoint_step(self.handle, up, sp, float(dt), float(tol), int(bool(use_graph)),
                                             stats, _stream(stream)))
        return BinStats(stats)


def mlp_forward(W, X, Y, cache=None, stream=None):
    import torch
    B = X.shape[0]
    _check(lib().adl_mlp_forward(_ptr(W, torch.float32, (MLP_PARAMS,), "W"),
                                 _ptr(X, torch.float32, (B, MLP_IN), "X"),
                                 _ptr(Y, torch.float32, (B, MLP_OUT), "Y"),
                                 _ptr(cache, torch.float32, (B, MLP_CACHE_PER_ROW), "cache") if cache is not None else None,
                                 int(B), _stream(stream)))
    return Y


def mlp_backward(W, cache, dY, dW, stream=None):
    import torch
    B = dY.shape[0]
    _check(lib().adl_mlp_backward(_ptr(W, torch.float32, (MLP_PARAMS,), "W"),
                                  _ptr(cache, torch.float32, (B, MLP_CACHE_PER_ROW), "cache"),
                                  _ptr(dY, torch.float32, (B, MLP_OUT), "dY"),
                                  _ptr(dW, torch.float32, (MLP_PARAMS,), "dW"), int(B), _stream(stream)))
    return dW


def mlp_mse_grad(Y, T, dY, loss=None, stream=None):
    import torch
    B = Y.shape[0]
    f = torch.float32
    _check(lib().adl_mlp_mse_grad(_ptr(Y, f, (B, MLP_OUT), "Y"), _ptr(T, f, (B, MLP_OUT), "T"),
                                  _ptr(dY, f, (B, MLP_OUT), "dY"), _ptr(loss, f, (1,), "loss") if loss is not None else None,
                                  int(B), _stream(stream)))
    return dY


def _f9(a):
    return (ctypes.c_float * len(a))(*[float(v) for v in a])


def learned_features(raw, g: float):
    x = (ctypes.c_float * 9)()
    _check(lib().adl_learned_features(_f9(raw), float(g), x))
    return list(x)


def learned_targets(raw, g: float, rho: float, degree: int, substeps: int):
    y = (ctypes.c_float * 3)()
    _check(lib().adl_learned_targets(_f9(raw), float(g), float(rho), int(degree), int(substeps), y))
    return list(y)


def learned_decode(raw, g: float, y):
    r = ctypes.c_double()
    m = ctypes.c_int()
    K = ctypes.c_int()
    _check(lib().adl_learned_decode(_f9(raw), float(g), _f9(y), ctypes.byref(r), ctypes.byref(m), ctypes.byref(K)))
    return r.value, m.value, K.value


def mlp_adam_step(W, dW, m1, m2, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    f = torch.float32
    _check(lib().adl_mlp_adam_step(_ptr(W, f, (MLP_PARAMS,), "W"), _ptr(dW, f, (MLP_PARAMS,), "dW"),
                                   _ptr(m1, f, (MLP_PARAMS,), "m1"), _ptr(m2, f, (MLP_PARAMS,), "m2"),
                                   int(t), float(lr), float(beta1), float(beta2), float(eps),
                                   _stream(stream)))
