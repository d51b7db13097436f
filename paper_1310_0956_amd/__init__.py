"""Python binding of libreco (ctypes): argument marshalling only.

Every operation runs in the HIP kernels of ``libreco.so`` through the C ABI
declared in ``include/reco.h``.  Torch tensors supply device memory and the
current HIP stream; nothing here computes on the data.  Importing fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libreco.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libreco.so not built ({LIB_PATH}); run __graft_entry__.build()")

_lib = C.CDLL(LIB_PATH)

RECO_OK, RECO_PENDING, RECO_ENOTCONV = 0, 1, 2
RECO_EINVAL, RECO_ENOMEM, RECO_EDEVICE, RECO_ENUMERIC, RECO_ENOTFOUND = -1, -2, -3, -4, -5
F32, F64 = 0, 1
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024   # RECO_NOALLOC_SCRATCH_BYTES
PRECOND_NONE, PRECOND_WMG, PRECOND_WMG_HYBRID = 0, 1, 2
PROJ_EXACT, PROJ_JOSEPH = 0, 1   # exact intersection lengths / Joseph's kernel
STATUS_NAMES = {0: "ok", 1: "pending", 2: "not_converged", -1: "einval", -2: "enomem",
                -3: "edevice", -4: "enumeric", -5: "enotfound"}


class GeometryDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_angles", C.c_int32), ("n_bins", C.c_int32),
                ("wmg_levels", C.c_int32), ("dtype", C.c_int32), ("projector", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("lam", C.c_double), ("precond", C.c_int32), ("check_every", C.c_int32),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("fixed_iters", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("relres", C.c_double),
                ("status", C.c_int32), ("reserved", C.c_int32), ("elapsed_ms", C.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "matvecs": self.matvecs, "relres": self.relres,
                "status": STATUS_NAMES.get(self.status, str(self.status)),
                "elapsed_ms": self.elapsed_ms}


_P = C.c_void_p
_S = C.c_int32
_sig = {
    "reco_last_error": (C.c_char_p, []),
    "reco_version": (C.c_char_p, []),
    "reco_create_geometry": (_S, [C.POINTER(GeometryDesc), _P, C.POINTER(_P)]),
    "reco_destroy_geometry": (_S, [_P]),
    "reco_geometry_get_desc": (_S, [_P, C.POINTER(GeometryDesc)]),
    "reco_packet_diagonal": (_S, [_P, C.POINTER(C.c_double)]),
    "reco_count_nnz": (_S, [_P, _P, C.POINTER(C.c_int64)]),
    "reco_project": (_S, [_P, _P, _P, _P]),
    "reco_backproject": (_S, [_P, _P, _P, _P]),
    "reco_wmg_apply": (_S, [_P, _P, _P, C.c_double, _P]),
    "reco_wmg_hybrid_apply": (_S, [_P, _P, _P, C.c_double, _P]),
    "reco_solve_cgls": (_S, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "reco_solve_cgls_noalloc": (_S, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo),
                                     _P]),
    "reco_solve_gmres": (_S, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "reco_solve_bicgstab": (_S, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "reco_solve_sirt": (_S, [_P, _P, _P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "reco_solve_batch": (_S, [_S, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P),
                              C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]),
    "reco_server_create": (_S, [C.c_size_t, _S, C.POINTER(_P)]),
    "reco_server_destroy": (_S, [_P]),
    "reco_submit": (_S, [_P, C.POINTER(GeometryDesc), _P, _P, C.POINTER(SolveOpts),
                         C.POINTER(C.c_uint64)]),
    "reco_poll": (_S, [_P, C.c_uint64, C.POINTER(SolveInfo), C.POINTER(C.c_double)]),
    "reco_clock": (C.c_double, []),
    "reco_timing_enable": (_S, [_S]),
    "reco_timing_read": (_S, [_S, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "reco_timing_reset": (_S, []),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


class RecoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(rc, allow=(RECO_OK,)):
    if rc not in allow:
        raise RecoError(rc, _lib.reco_last_error().decode())
    return rc


def last_error() -> str:
    return _lib.reco_last_error().decode()


def version() -> str:
    return _lib.reco_version().decode()


def clock() -> float:
    return _lib.reco_clock()


TIMED = {"forward": 0, "backward": 1, "wmg": 2, "update": 3, "packet_diag": 4, "prep": 5,
         "batch_graph": 6}


def timing_enable(on=True):
    _check(_lib.reco_timing_enable(1 if on else 0))


def timing_reset():
    _check(_lib.reco_timing_reset())


def timing_read():
    """{family: (launches, total_ms)} for every timed kernel family."""
    out = {}
    for name, k in TIMED.items():
        n, ms = C.c_int64(), C.c_double()
        _check(_lib.reco_timing_read(k, C.byref(n), C.byref(ms)))
        out[name] = (n.value, ms.value)
    return out


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _torch_dtype(dtype):
    import torch
    return torch.float64 if dtype == F64 else torch.float32


class Geometry:
    """A 2D parallel-beam geometry on the GPU (owns tables and the packet diagonal)."""

    def __init__(self, n, n_angles, n_bins, wmg_levels=2, dtype=F32, stream=None,
                 projector=PROJ_EXACT):
        self.desc = GeometryDesc(n, n_angles, n_bins, wmg_levels, dtype, projector)
        h = C.c_void_p()
        _check(_lib.reco_create_geometry(C.byref(self.desc), _stream(stream), C.byref(h)))
        self.handle = h

    @property
    def n(self):
        return self.desc.n

    @property
    def m(self):
        return self.desc.n_angles

    @property
    def nb(self):
        return self.desc.n_bins

    @property
    def dtype(self):
        return _torch_dtype(self.desc.dtype)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.reco_destroy_geometry(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _img(self, t, name):
        self._dev(t, name)
        if tuple(t.shape) not in ((self.n, self.n), (self.n * self.n,)):
            raise ValueError(f"{name} must hold {self.n}x{self.n} elements")
        return C.c_void_p(t.data_ptr())

    def _sino(self, t, name):
        self._dev(t, name)
        if tuple(t.shape) not in ((self.m, self.nb), (self.m * self.nb,)):
            raise ValueError(f"{name} must hold {self.m}x{self.nb} elements")
        return C.c_void_p(t.data_ptr())

    def _dev(self, t, name):
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor on the GPU")

    def new_image(self):
        import torch
        return torch.empty((self.n, self.n), dtype=self.dtype, device="cuda")

    def new_sinogram(self):
        import torch
        return torch.empty((self.m, self.nb), dtype=self.dtype, device="cuda")

    # -- operators -----------------------------------------------------------
    def project(self, x, out=None, stream=None):
        out = self.new_sinogram() if out is None else out
        _check(_lib.reco_project(self.handle, self._img(x, "x"), self._sino(out, "b"),
                                 _stream(stream)))
        return out

    def backproject(self, b, out=None, stream=None):
        out = self.new_image() if out is None else out
        _check(_lib.reco_backproject(self.handle, self._sino(b, "b"), self._img(out, "x"),
                                     _stream(stream)))
        return out

    def wmg_apply(self, r, out=None, lam=0.0, stream=None):
        out = self.new_image() if out is None else out
        _check(_lib.reco_wmg_apply(self.handle, self._img(r, "r"), self._img(out, "z"),
                                   float(lam), _stream(stream)))
        return out

    def wmg_hybrid_apply(self, r, out=None, lam=0.0, stream=None):
        """z = M^-1 r with the hybrid wavelet cycle and exact coarsest solves."""
        out = self.new_image() if out is None else out
        _check(_lib.reco_wmg_hybrid_apply(self.handle, self._img(r, "r"), self._img(out, "z"),
                                          float(lam), _stream(stream)))
        return out

    def packet_diagonal(self):
        import numpy as np
        d = np.empty((self.n, self.n), dtype=np.float64)
        _check(_lib.reco_packet_diagonal(self.handle,
                                         d.ctypes.data_as(C.POINTER(C.c_double))))
        return d

    def count_nnz(self, stream=None):
        v = C.c_int64()
        _check(_lib.reco_count_nnz(self.handle, _stream(stream), C.byref(v)))
        return v.value

    # -- solvers -------------------------------------------------------------
    def _solve(self, fn, b, x, tol, max_iter, lam, precond, restart, fixed_iters, history,
               check_every, stream):
        import numpy as np
        x = self.new_image() if x is None else x
        cap = (fixed_iters or max_iter) if history else 0
        hist = np.zeros(max(cap, 1), dtype=np.float64)
        opts = SolveOpts(float(tol), int(max_iter), int(restart), float(lam), int(precond),
                         int(check_every), hist.ctypes.data_as(C.POINTER(C.c_double)) if cap else None,
                         int(cap), int(fixed_iters or 0))
        info = SolveInfo()
        rc = fn(self.handle, self._sino(b, "b"), self._img(x, "x"), C.byref(opts),
                C.byref(info), _stream(stream))
        _check(rc, allow=(RECO_OK, RECO_ENOTCONV, RECO_ENUMERIC))
        d = info.as_dict()
        if cap:
            d["history"] = hist[:min(info.iters, cap)].copy()
        return x, d

    def solve_cgls(self, b, x=None, tol=1e-3, max_iter=1000, lam=0.0, precond=PRECOND_WMG,
                   fixed_iters=0, history=False, check_every=0, stream=None):
        return self._solve(_lib.reco_solve_cgls, b, x, tol, max_iter, lam, precond, 30,
                           fixed_iters, history, check_every, stream)

    def solve_cgls_noalloc(self, b, x=None, tol=1e-3, max_iter=1000, lam=0.0,
                           precond=PRECOND_WMG, fixed_iters=0, history=False, check_every=0,
                           stream=None):
        """solve_cgls through the allocation-free entry point (fixed scratch array)."""
        return self._solve(_lib.reco_solve_cgls_noalloc, b, x, tol, max_iter, lam, precond, 30,
                           fixed_iters, history, check_every, stream)

    def solve_gmres(self, b, x=None, tol=1e-3, max_iter=1000, lam=0.0, precond=PRECOND_WMG,
                    restart=30, fixed_iters=0, history=False, check_every=0, stream=None):
        return self._solve(_lib.reco_solve_gmres, b, x, tol, max_iter, lam, precond, restart,
                           fixed_iters, history, check_every, stream)

    def solve_bicgstab(self, b, x=None, tol=1e-3, max_iter=1000, lam=0.0, precond=PRECOND_WMG,
                       fixed_iters=0, history=False, check_every=0, stream=None):
        return self._solve(_lib.reco_solve_bicgstab, b, x, tol, max_iter, lam, precond, 30,
                           fixed_iters, history, check_every, stream)

    def solve_sirt(self, b, x=None, tol=1e-3, max_iter=1000, fixed_iters=0, history=False,
                   check_every=0, stream=None):
        return self._solve(_lib.reco_solve_sirt, b, x, tol, max_iter, 0.0, PRECOND_NONE, 30,
                           fixed_iters, history, check_every, stream)


def _per(v, n):
    return list(v) if isinstance(v, (list, tuple)) else [v] * n


def solve_batch(geoms, bs, xs, tol=1e-3, max_iter=1000, lam=0.0, precond=PRECOND_WMG,
                fixed_iters=0, check_every=0, stream=None):
    """Solve many CGLS problems together; returns a list of info dicts.

    tol, max_iter, lam, precond and fixed_iters are scalars or per-problem lists."""
    n = len(geoms)
    if not (len(bs) == n and len(xs) == n):
        raise ValueError("geoms, bs and xs must have the same length")
    GA = (C.c_void_p * n)(*[g.handle.value for g in geoms])
    BA = (C.c_void_p * n)(*[g._sino(b, "b").value for g, b in zip(geoms, bs)])
    XA = (C.c_void_p * n)(*[g._img(x, "x").value for g, x in zip(geoms, xs)])
    opts = zip(_per(tol, n), _per(max_iter, n), _per(lam, n), _per(precond, n),
               _per(fixed_iters, n))
    OA = (SolveOpts * n)(*[SolveOpts(float(t), int(mi), 30, float(la), int(pc), int(check_every),
                                     None, 0, int(fi)) for t, mi, la, pc, fi in opts])
    IA = (SolveInfo * n)()
    rc = _lib.reco_solve_batch(n, GA, BA, XA, OA, IA, _stream(stream))
    _check(rc, allow=(RECO_OK, RECO_ENOTCONV, RECO_ENUMERIC))
    return [IA[i].as_dict() for i in range(n)]


class Server:
    """Continuous-batching reconstruction server (scheduler thread in libreco)."""

    def __init__(self, hbm_budget_bytes, max_slots=64):
        h = C.c_void_p()
        _check(_lib.reco_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.handle = h

    def submit(self, n, n_angles, n_bins, wmg_levels, b, x, tol=1e-3, max_iter=1000,
               precond=PRECOND_WMG, lam=0.0, fixed_iters=0, projector=PROJ_EXACT):
        """Queue a request; b and x are float32 device tensors that must stay alive
        (and b unchanged) until poll() returns a result.  The current stream is
        synchronised first so that b is complete when the server reads it."""
        import torch
        for t, size, name in ((b, n_angles * n_bins, "b"), (x, n * n, "x")):
            if (not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()
                    or t.numel() != size):
                raise ValueError(f"{name} must be a contiguous float32 GPU tensor of {size} "
                                 "elements")
        torch.cuda.current_stream().synchronize()
        desc = GeometryDesc(n, n_angles, n_bins, wmg_levels, F32, projector)
        opts = SolveOpts(float(tol), int(max_iter), 30, float(lam), int(precond), 0, None, 0,
                         int(fixed_iters))
        t = C.c_uint64()
        _check(_lib.reco_submit(self.handle, C.byref(desc), C.c_void_p(b.data_ptr()),
                                C.c_void_p(x.data_ptr()), C.byref(opts), C.byref(t)))
        return t.value

    def poll(self, ticket):
        info = SolveInfo()
        ts = (C.c_double * 3)()
        rc = _lib.reco_poll(self.handle, C.c_uint64(ticket), C.byref(info), ts)
        if rc == RECO_PENDING:
            return None
        _check(rc, allow=(RECO_OK, RECO_ENOTCONV, RECO_ENUMERIC))
        d = info.as_dict()
        d["status_code"] = rc
        d["t_submit"], d["t_admit"], d["t_done"] = ts[0], ts[1], ts[2]
        return d

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(_lib.reco_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
