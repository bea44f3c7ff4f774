"""ctypes binding of librpb (include/rpb.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor dtypes,
devices and shapes, passes raw device pointers and torch's current stream, and
turns status codes into exceptions.  There is no CPU fallback: if the library
is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librpb.so")

RPB_OK, RPB_EINVAL, RPB_ENOMEM, RPB_EDEVICE, RPB_ENOCONV, RPB_ENOTSPD, RPB_ENONFINITE = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "RPB_OK", -1: "RPB_EINVAL", -2: "RPB_ENOMEM", -3: "RPB_EDEVICE",
                -4: "RPB_ENOCONV", -5: "RPB_ENOTSPD", -6: "RPB_ENONFINITE"}
RPB_FP64, RPB_MIXED = 0, 1
PRECISIONS = {"fp64": RPB_FP64, "mixed": RPB_MIXED}

# Every symbol include/rpb.h declares.
EXPORTS = (
    "rpb_create", "rpb_destroy", "rpb_last_error", "rpb_version",
    "rpb_mobility_matvec", "rpb_mobility_matvec_rows", "lanczos_sqrt_apply", "rfd_drift",
    "rfd_drift_one_sided", "lanczos_sqrt_apply_precond",
    "rpb_forces", "rpb_normals", "sab_step", "rpb_timing_enable", "rpb_timing_read",
    "rpb_mobility_matvec_batched", "lanczos_sqrt_apply_batched", "sab_step_batched",
    "rpb_step_graph_create", "rpb_step_graph_launch", "rpb_step_graph_status",
    "rpb_step_graph_destroy", "rpb_get_tuning", "rpb_set_tuning", "rpb_autotune",
    "rpb_mobility_matvec_multi", "lanczos_sqrt_apply_multi", "rpb_output_check_enable",
    "rpb_mobility_matvec_noalloc", "lanczos_tridiag_sqrt",
)


class RpbParams(C.Structure):
    _fields_ = [("a", C.c_double), ("eta", C.c_double), ("kT", C.c_double), ("precision", C.c_int),
                ("wall", C.c_int), ("lx", C.c_double), ("ly", C.c_double)]


class RpbSabConfig(C.Structure):
    _fields_ = [("dt", C.c_double), ("delta", C.c_double), ("lanczos_tol", C.c_double),
                ("lanczos_max_iter", C.c_int), ("scheme", C.c_int), ("rfd_precision", C.c_int),
                ("rfd_scheme", C.c_int), ("lanczos_precond", C.c_int), ("f_grav_z", C.c_double),
                ("torque", C.c_double * 3), ("steric_u0", C.c_double),
                ("steric_b", C.c_double), ("seed", C.c_uint64)]


class RpbShape(C.Structure):
    _fields_ = [("tpt", C.c_int), ("target_wgs", C.c_int), ("batch_chunk", C.c_int),
                ("batch_wgs", C.c_int), ("symmetric", C.c_int), ("batch_tpt", C.c_int),
                ("batch_symmetric", C.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class RpbTuning(C.Structure):
    _fields_ = [("fp64", RpbShape), ("mixed", RpbShape)]

    def as_dict(self):
        return {"fp64": self.fp64.as_dict(), "mixed": self.mixed.as_dict()}


class RpbSabState(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("u_prev", C.c_void_p),
                ("step", C.c_int64), ("have_prev", C.c_int)]


class RpbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load librpb.so (raises if it is missing: build it with paper_1612_00474_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found; build it with `python -m paper_1612_00474_amd.build`")
    # torch first: its HIP runtime is then the one the library's libamdhip64 dependency binds
    # to (a second copy of the runtime in the process would not see the device state torch
    # sets up)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.c_void_p
    D = C.c_double
    I64 = C.c_int64
    pp = C.POINTER(RpbParams)
    sig = {
        "rpb_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
        "rpb_destroy": (None, [P]),
        "rpb_last_error": (C.c_char_p, [P]),
        "rpb_version": (C.c_char_p, []),
        "rpb_mobility_matvec": (C.c_int, [P, pp, I64, P, P, P, P, P]),
        "rpb_mobility_matvec_rows": (C.c_int, [P, pp, I64, P, P, P, I64, I64, P, P]),
        "rpb_mobility_matvec_noalloc": (C.c_int, [P, pp, I64, P, P, P, P, P]),
        "lanczos_sqrt_apply": (C.c_int, [P, pp, I64, P, P, D, C.c_int, P, C.POINTER(C.c_int),
                                         C.POINTER(D), P]),
        "lanczos_sqrt_apply_precond": (C.c_int, [P, pp, I64, P, P, D, C.c_int, P,
                                                 C.POINTER(C.c_int), C.POINTER(D), P]),
        "lanczos_tridiag_sqrt": (C.c_int, [P, C.c_int32, P, P, D, P, P]),
        "rfd_drift": (C.c_int, [P, pp, I64, P, P, D, C.c_int, P, P]),
        "rfd_drift_one_sided": (C.c_int, [P, pp, I64, P, P, D, C.c_int, P, P]),
        "rpb_forces": (C.c_int, [P, pp, I64, P, D, D, D, P, P]),
        "rpb_normals": (C.c_int, [P, I64, C.c_uint64, C.c_uint64, C.c_uint64, P, P]),
        "sab_step": (C.c_int, [P, pp, C.POINTER(RpbSabConfig), C.POINTER(RpbSabState), P, P,
                               C.POINTER(C.c_int), C.POINTER(D), P]),
        "rpb_timing_enable": (C.c_int, [P, C.c_int]),
        "rpb_output_check_enable": (C.c_int, [P, C.c_int]),
        "rpb_timing_read": (C.c_int, [P, C.c_int, C.POINTER(D), C.POINTER(I64), C.POINTER(D)]),
        "rpb_mobility_matvec_batched": (C.c_int, [P, pp, C.c_int32, P, P, P, P, P, P]),
        "lanczos_sqrt_apply_batched": (C.c_int, [P, pp, C.c_int32, P, P, P, D, C.c_int, P, P, P, P]),
        "sab_step_batched": (C.c_int, [P, pp, C.POINTER(RpbSabConfig), C.c_int32, P, P, P, I64,
                                       C.c_int, P, P, P, P, P]),
        "rpb_step_graph_create": (C.c_int, [P, pp, C.POINTER(RpbSabConfig), C.c_int32, P, P, P,
                                            I64, C.c_int, C.POINTER(C.c_void_p), P]),
        "rpb_step_graph_launch": (C.c_int, [P, P]),
        "rpb_step_graph_status": (C.c_int, [P, C.POINTER(I64), P, P, P]),
        "rpb_step_graph_destroy": (None, [P]),
        "rpb_get_tuning": (C.c_int, [P, C.POINTER(RpbTuning)]),
        "rpb_set_tuning": (C.c_int, [P, C.POINTER(RpbTuning)]),
        "rpb_autotune": (C.c_int, [P, pp, C.c_int32, P, P, C.c_int, C.POINTER(RpbTuning),
                                   C.POINTER(D), P]),
        "rpb_mobility_matvec_multi": (C.c_int, [P, pp, I64, P, C.c_int32, P, P, P]),
        "lanczos_sqrt_apply_multi": (C.c_int, [P, pp, I64, P, C.c_int32, P, D, C.c_int, P, P,
                                               P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _vec3(t, name, n=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{name} must have shape (n, 3), got {tuple(t.shape)}")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"{name} has {t.shape[0]} rows, expected {n}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _offsets(offs, n=None):
    import numpy as np
    o = np.ascontiguousarray(np.asarray(offs, dtype=np.int64))
    if o.ndim != 1 or o.size < 2 or o[0] != 0 or np.any(np.diff(o) < 0):
        raise ValueError("offs must be 1-D non-decreasing int64 prefix sums starting at 0")
    if n is not None and o[-1] != n:
        raise ValueError(f"offs[-1] = {o[-1]} but the arrays hold {n} spheres")
    return o


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data)


RFD_SCHEMES = {"centred": 0, "one_sided": 1}


def _sab_config(dt, delta, lanczos_tol, lanczos_max_iter, scheme, rfd_precision, f_grav_z,
                torque, steric_u0, steric_b, seed, rfd_scheme="centred", lanczos_precond=False):
    if scheme not in ("sab", "em"):
        raise ValueError(f"scheme must be 'sab' or 'em', not {scheme!r}")
    return RpbSabConfig(dt, delta, lanczos_tol, lanczos_max_iter, 0 if scheme == "sab" else 1,
                        PRECISIONS[rfd_precision], RFD_SCHEMES[rfd_scheme],
                        int(bool(lanczos_precond)), f_grav_z, (C.c_double * 3)(*torque),
                        steric_u0, steric_b, seed)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One librpb context on one device (not thread-safe; one per host thread)."""

    def __init__(self, device: int = 0, a: float = 1.0, eta: float = 1.0, kT: float = 1.0,
                 wall: bool = True, box=None):
        import torch
        # torch owns the device memory and streams this library works on: its HIP runtime
        # must be initialised before the library's first HIP call
        torch.cuda.init()
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.rpb_create(device, C.byref(h))
        if st != RPB_OK:
            raise RpbError(st, f"rpb_create({device}) failed")
        self.h = h
        self.device = device
        self.a, self.eta, self.kT = a, eta, kT
        self.wall = wall          # False: free space (unbounded RPY, no wall force)
        self.box = box            # (L_x, L_y): pseudo-periodic boundaries, single systems

    def close(self):
        if getattr(self, "h", None):
            self.lib.rpb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, precision="fp64"):
        lx, ly = self.box if self.box is not None else (0.0, 0.0)
        return RpbParams(self.a, self.eta, self.kT, PRECISIONS[precision] if isinstance(precision, str)
                         else int(precision), int(bool(self.wall)), float(lx), float(ly))

    def _check(self, st, ok=(RPB_OK,)):
        if st not in ok:
            raise RpbError(st, self.lib.rpb_last_error(self.h).decode())
        return st

    def last_error(self) -> str:
        return self.lib.rpb_last_error(self.h).decode()

    # -- products ------------------------------------------------------------------------
    def matvec(self, pos, force=None, torque=None, precision="fp64", out=None, rows=None):
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        if force is not None:
            _vec3(force, "force", n)
        if torque is not None:
            _vec3(torque, "torque", n)
        p = self.params(precision)
        if rows is None:
            if out is None:
                out = torch.empty_like(pos)
            _vec3(out, "out", n)
            st = self.lib.rpb_mobility_matvec(self.h, C.byref(p), n, _ptr(pos), _ptr(force),
                                              _ptr(torque), _ptr(out), _stream())
        else:
            r0, r1 = rows
            if out is None:
                out = torch.empty((r1 - r0, 3), dtype=torch.float64, device=pos.device)
            _vec3(out, "out", r1 - r0)
            st = self.lib.rpb_mobility_matvec_rows(self.h, C.byref(p), n, _ptr(pos), _ptr(force),
                                                   _ptr(torque), r0, r1, _ptr(out), _stream())
        self._check(st)
        return out

    def matvec_noalloc(self, pos, force=None, torque=None, precision="fp64", out=None):
        """U = M F + M_C T through the entry point that allocates nothing (its intermediates
        live in the library's static per-device scratch array)."""
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        if force is not None:
            _vec3(force, "force", n)
        if torque is not None:
            _vec3(torque, "torque", n)
        if out is None:
            out = torch.empty_like(pos)
        _vec3(out, "out", n)
        p = self.params(precision)
        st = self.lib.rpb_mobility_matvec_noalloc(self.h, C.byref(p), n, _ptr(pos), _ptr(force),
                                                  _ptr(torque), _ptr(out), _stream())
        self._check(st)
        return out

    def lanczos(self, pos, w, tol, max_iter=64, precision="fp64", out=None, allow_noconv=False,
                precond=False, allow_notspd=False):
        """Returns (g, iterations, eps, status); precond: block-diagonal preconditioned form.
        allow_noconv / allow_notspd: return RPB_ENOCONV / RPB_ENOTSPD (with the last iterate)
        instead of raising."""
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        _vec3(w, "w", n)
        if out is None:
            out = torch.empty_like(pos)
        p = self.params(precision)
        it = C.c_int(0)
        eps = C.c_double(0.0)
        fn = self.lib.lanczos_sqrt_apply_precond if precond else self.lib.lanczos_sqrt_apply
        st = fn(self.h, C.byref(p), n, _ptr(pos), _ptr(w), float(tol), int(max_iter), _ptr(out),
                C.byref(it), C.byref(eps), _stream())
        ok = (RPB_OK,) + ((RPB_ENOCONV,) if allow_noconv else ()) + (
            (RPB_ENOTSPD,) if allow_notspd else ())
        self._check(st, ok)
        return out, it.value, eps.value, st

    def tridiag_sqrt(self, alpha, beta, wnorm=1.0):
        """y_k = wnorm T_k^{1/2} e_1 for the leading blocks T_k (k = 1..m) of the symmetric
        tridiagonal (alpha, beta); returns an (m, m) float64 array, row k - 1 holding y_k."""
        import numpy as np
        alpha = np.ascontiguousarray(alpha, dtype=np.float64).ravel()
        beta = np.ascontiguousarray(beta, dtype=np.float64).ravel()
        m = alpha.size
        if beta.size != max(m - 1, 0):
            raise ValueError("beta must have len(alpha) - 1 entries")
        out = np.zeros((m, m), dtype=np.float64)
        st = self.lib.lanczos_tridiag_sqrt(self.h, m, alpha.ctypes.data,
                                           beta.ctypes.data if beta.size else None,
                                           float(wnorm), out.ctypes.data, _stream())
        self._check(st)
        return out

    def rfd(self, pos, w_tilde, delta, precision="fp64", rfd_precision="fp64", out=None,
            rfd_scheme="centred"):
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        _vec3(w_tilde, "w_tilde", n)
        if out is None:
            out = torch.empty_like(pos)
        p = self.params(precision)
        fn = {"centred": self.lib.rfd_drift, "one_sided": self.lib.rfd_drift_one_sided}[rfd_scheme]
        st = fn(self.h, C.byref(p), n, _ptr(pos), _ptr(w_tilde), float(delta),
                PRECISIONS[rfd_precision], _ptr(out), _stream())
        self._check(st)
        return out

    def forces(self, pos, f_grav_z=-1.0, u0=1.0, b=0.1, out=None):
        import torch
        pos = _vec3(pos, "pos")
        if out is None:
            out = torch.empty_like(pos)
        p = self.params("fp64")
        st = self.lib.rpb_forces(self.h, C.byref(p), pos.shape[0], _ptr(pos), float(f_grav_z),
                                 float(u0), float(b), _ptr(out), _stream())
        self._check(st)
        return out

    def normals(self, count, seed, stream_id, step, device="cuda"):
        import torch
        out = torch.empty(count, dtype=torch.float64, device=device)
        st = self.lib.rpb_normals(self.h, int(count), int(seed), int(stream_id), int(step),
                                  _ptr(out), _stream())
        self._check(st)
        return out

    # -- several vectors, one configuration --------------------------------------------
    def _vecs(self, t, name, n):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda":
            raise TypeError(f"{name} must be a float64 GPU tensor")
        if t.dim() != 3 or t.shape[1] != n or t.shape[2] != 3 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous (nvec, {n}, 3) tensor, got "
                             f"{tuple(t.shape)}")
        return t

    def matvec_multi(self, pos, force, precision="fp64", out=None):
        """M F_v for every vector F_v = force[v] of shape (n, 3) (forces only)."""
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        self._vecs(force, "force", n)
        if out is None:
            out = torch.empty_like(force)
        self._vecs(out, "out", n)
        if out.shape[0] != force.shape[0]:
            raise ValueError("out and force must hold the same number of vectors")
        p = self.params(precision)
        st = self.lib.rpb_mobility_matvec_multi(self.h, C.byref(p), n, _ptr(pos), force.shape[0],
                                                _ptr(force), _ptr(out), _stream())
        self._check(st)
        return out

    def lanczos_multi(self, pos, w, tol, max_iter=64, precision="fp64", out=None,
                      allow_noconv=False):
        """M^{1/2} w[v] for every vector; returns (g, iterations per vector, eps per vector,
        status)."""
        import numpy as np
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        self._vecs(w, "w", n)
        if out is None:
            out = torch.empty_like(w)
        self._vecs(out, "out", n)
        if out.shape[0] != w.shape[0]:
            raise ValueError("out and w must hold the same number of vectors")
        nvec = w.shape[0]
        it = np.zeros(max(nvec, 1), dtype=np.int32)
        eps = np.zeros(max(nvec, 1), dtype=np.float64)
        p = self.params(precision)
        st = self.lib.lanczos_sqrt_apply_multi(self.h, C.byref(p), n, _ptr(pos), nvec, _ptr(w),
                                               float(tol), int(max_iter), _ptr(out), _np_ptr(it),
                                               _np_ptr(eps), _stream())
        self._check(st, (RPB_OK, RPB_ENOCONV) if allow_noconv else (RPB_OK,))
        return out, it[:nvec], eps[:nvec], st

    # -- batched suspensions -------------------------------------------------------------
    def matvec_batched(self, pos, offs, force=None, torque=None, precision="fp64", out=None):
        """Products of `len(offs) - 1` independent systems concatenated in `pos`."""
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        o = _offsets(offs, n)
        if force is not None:
            _vec3(force, "force", n)
        if torque is not None:
            _vec3(torque, "torque", n)
        if out is None:
            out = torch.empty_like(pos)
        p = self.params(precision)
        st = self.lib.rpb_mobility_matvec_batched(self.h, C.byref(p), o.size - 1, _np_ptr(o),
                                                  _ptr(pos), _ptr(force), _ptr(torque), _ptr(out),
                                                  _stream())
        self._check(st)
        return out

    def lanczos_batched(self, pos, offs, w, tol, max_iter=64, precision="fp64", out=None,
                        allow_noconv=False):
        """Returns (g, iterations per system, eps per system, status)."""
        import numpy as np
        import torch
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        o = _offsets(offs, n)
        _vec3(w, "w", n)
        if out is None:
            out = torch.empty_like(pos)
        nsys = o.size - 1
        it = np.zeros(nsys, dtype=np.int32)
        eps = np.zeros(nsys, dtype=np.float64)
        p = self.params(precision)
        st = self.lib.lanczos_sqrt_apply_batched(self.h, C.byref(p), nsys, _np_ptr(o), _ptr(pos),
                                                 _ptr(w), float(tol), int(max_iter), _ptr(out),
                                                 _np_ptr(it), _np_ptr(eps), _stream())
        self._check(st, (RPB_OK, RPB_ENOCONV) if allow_noconv else (RPB_OK,))
        return out, it, eps, st

    def sab_step_batched(self, pos, u_prev, offs, step, have_prev, *, dt, delta, lanczos_tol,
                         lanczos_max_iter=64, scheme="sab", rfd_precision="fp64", f_grav_z=-1.0,
                         torque=(0.0, 1.0, 0.0), steric_u0=1.0, steric_b=0.1, seed=0,
                         precision="fp64", w=None, w_tilde=None, rfd_scheme="centred",
                         lanczos_precond=False):
        """One step of every system; updates pos and u_prev in place.
        Returns (iterations per system, eps per system, status)."""
        import numpy as np
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        _vec3(u_prev, "u_prev", n)
        o = _offsets(offs, n)
        nsys = o.size - 1
        cfg = _sab_config(dt, delta, lanczos_tol, lanczos_max_iter, scheme, rfd_precision,
                          f_grav_z, torque, steric_u0, steric_b, seed, rfd_scheme,
                          lanczos_precond)
        it = np.zeros(nsys, dtype=np.int32)
        eps = np.zeros(nsys, dtype=np.float64)
        p = self.params(precision)
        st = self.lib.sab_step_batched(self.h, C.byref(p), C.byref(cfg), nsys, _np_ptr(o),
                                       _ptr(pos), _ptr(u_prev), int(step), int(bool(have_prev)),
                                       _ptr(w), _ptr(w_tilde), _np_ptr(it), _np_ptr(eps),
                                       _stream())
        self._check(st, (RPB_OK, RPB_ENOCONV))
        return it, eps, st

    def step_graph(self, pos, u_prev, offs, step=0, have_prev=False, *, dt, delta, lanczos_tol,
                   lanczos_max_iter=16, scheme="sab", rfd_precision="fp64", f_grav_z=-1.0,
                   torque=(0.0, 1.0, 0.0), steric_u0=1.0, steric_b=0.1, seed=0,
                   precision="fp64", rfd_scheme="centred", lanczos_precond=False):
        """A hipGraph of one batched step bound to pos / u_prev (see StepGraph)."""
        return StepGraph(self, pos, u_prev, offs, step, have_prev,
                         _sab_config(dt, delta, lanczos_tol, lanczos_max_iter, scheme,
                                     rfd_precision, f_grav_z, torque, steric_u0, steric_b, seed,
                                     rfd_scheme, lanczos_precond),
                         precision)

    # -- time step -----------------------------------------------------------------------
    def sab_step(self, state, *, dt, delta, lanczos_tol, lanczos_max_iter=64, scheme="sab",
                 rfd_precision="fp64", f_grav_z=-1.0, torque=(0.0, 1.0, 0.0), steric_u0=1.0,
                 steric_b=0.1, seed=0, precision="fp64", w=None, w_tilde=None,
                 rfd_scheme="centred", lanczos_precond=False):
        """Advance ``state`` (a StepState) by one step; returns (iterations, eps, status)."""
        cfg = _sab_config(dt, delta, lanczos_tol, lanczos_max_iter, scheme, rfd_precision,
                          f_grav_z, torque, steric_u0, steric_b, seed, rfd_scheme,
                          lanczos_precond)
        n = state.pos.shape[0]
        if w is not None:
            _vec3(w, "w", n)
        if w_tilde is not None:
            _vec3(w_tilde, "w_tilde", n)
        s = RpbSabState(n, state.pos.data_ptr(), state.u_prev.data_ptr(), state.step,
                        int(state.have_prev))
        p = self.params(precision)
        it = C.c_int(0)
        eps = C.c_double(0.0)
        st = self.lib.sab_step(self.h, C.byref(p), C.byref(cfg), C.byref(s), _ptr(w), _ptr(w_tilde),
                               C.byref(it), C.byref(eps), _stream())
        self._check(st, (RPB_OK, RPB_ENOCONV))
        state.step = s.step
        state.have_prev = bool(s.have_prev)
        return it.value, eps.value, st

    # -- tuning --------------------------------------------------------------------------
    def tuning(self):
        t = RpbTuning()
        self._check(self.lib.rpb_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, precision, **kw):
        """Change fields of one precision's launch shape (tpt, target_wgs, symmetric,
        batch_tpt, batch_chunk, batch_wgs, batch_symmetric)."""
        cur = self.tuning()
        cur[precision].update(kw)
        t = RpbTuning(RpbShape(**cur["fp64"]), RpbShape(**cur["mixed"]))
        self._check(self.lib.rpb_set_tuning(self.h, C.byref(t)))

    def autotune(self, pos, offs=None, precision="mixed", reps=2):
        """Time the launch-shape candidates on this configuration; returns (shape, best ms)."""
        pos = _vec3(pos, "pos")
        o = _offsets([0, pos.shape[0]] if offs is None else offs, pos.shape[0])
        t = RpbTuning()
        ms = C.c_double(0.0)
        p = self.params(precision)
        self._check(self.lib.rpb_autotune(self.h, C.byref(p), o.size - 1, _np_ptr(o), _ptr(pos),
                                          int(reps), C.byref(t), C.byref(ms), _stream()))
        return t.as_dict()[precision], ms.value

    def output_check(self, enable: bool):
        """Scan each result for NaN / Inf and raise (RPB_ENONFINITE) if one is found."""
        self._check(self.lib.rpb_output_check_enable(self.h, int(enable)))

    # -- timing --------------------------------------------------------------------------
    def timing(self, enable: bool):
        self._check(self.lib.rpb_timing_enable(self.h, int(enable)))

    def timing_read(self, kind=-1):
        """(milliseconds, launches, pair interactions) of pair-kernel launches since the last read.

        ``kind``: -1 for all launches, else 2 * (mixed) + (with torque), plus 4 for the
        batched kernel; 8 + 2 * (mixed) for the multi-vector kernel."""
        ms = C.c_double(0.0)
        k = C.c_int64(0)
        pairs = C.c_double(0.0)
        self._check(self.lib.rpb_timing_read(self.h, int(kind), C.byref(ms), C.byref(k),
                                             C.byref(pairs)))
        return ms.value, k.value, pairs.value


class StepState:
    """Positions and the stored velocity u^{n-1} of a time-stepped suspension (device tensors)."""

    def __init__(self, pos):
        import torch
        self.pos = _vec3(pos, "pos")
        self.u_prev = torch.zeros_like(pos)
        self.step = 0
        self.have_prev = False


class StepGraph:
    """A captured batched SAB step: each launch() advances the bound arrays by one step."""

    def __init__(self, ctx, pos, u_prev, offs, step, have_prev, cfg, precision):
        pos = _vec3(pos, "pos")
        n = pos.shape[0]
        _vec3(u_prev, "u_prev", n)
        self.ctx = ctx
        self.offs = _offsets(offs, n)
        self.nsys = self.offs.size - 1
        self._keep = (pos, u_prev)          # the graph writes into these tensors
        self.cfg = cfg
        p = ctx.params(precision)
        h = C.c_void_p()
        st = ctx.lib.rpb_step_graph_create(ctx.h, C.byref(p), C.byref(cfg), self.nsys,
                                           _np_ptr(self.offs), _ptr(pos), _ptr(u_prev), int(step),
                                           int(bool(have_prev)), C.byref(h), _stream())
        ctx._check(st)
        self.h = h

    def launch(self):
        st = self.ctx.lib.rpb_step_graph_launch(self.h, _stream())
        if st != RPB_OK:
            raise RpbError(st, "rpb_step_graph_launch failed")

    def status(self):
        """(device step counter, iterations per system, eps per system, status) of the last step."""
        import numpy as np
        step = C.c_int64(0)
        it = np.zeros(self.nsys, dtype=np.int32)
        eps = np.zeros(self.nsys, dtype=np.float64)
        st = self.ctx.lib.rpb_step_graph_status(self.h, C.byref(step), _np_ptr(it), _np_ptr(eps),
                                                _stream())
        if st not in (RPB_OK, RPB_ENOCONV):
            raise RpbError(st, "rpb_step_graph_status failed")
        return step.value, it, eps, st

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.rpb_step_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
