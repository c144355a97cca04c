"""ctypes binding of libamgdd.so (include/amgdd.h).

Argument marshalling only: setup runs in the library's C++ host code and
every solve step runs in its HIP kernels.  Device vectors are torch tensors
on the handle's device; their storage is passed as raw pointers and the
solve runs on torch's current stream.  The library must be built
(python -m paper_1906_10575_amd.build); importing this module raises if it
is not.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamgdd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBREAKDOWN, EUNSUPPORTED = range(7)
FP64, MIXED = 0, 1
STATUS_NAMES = ["OK", "EINVAL", "ENOMEM", "EDEVICE", "ENOCONV", "EBREAKDOWN", "EUNSUPPORTED"]


class AmgddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_coarse", C.c_int), ("max_levels", C.c_int), ("padding", C.c_int),
                ("n_fac", C.c_int), ("precision", C.c_int), ("device", C.c_int), ("use_graph", C.c_int),
                ("tail_level", C.c_int), ("tail_block", C.c_int), ("hybrid_level", C.c_int),
                ("relax_order", C.c_int), ("coarsen", C.c_int), ("interp", C.c_int),
                ("interp_max", C.c_int), ("n_padding_levels", C.c_int),
                ("padding_per_level", C.POINTER(C.c_int))]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("relres", C.c_double), ("rho_asym", C.c_double), ("solve_s", C.c_double),
                ("setup_s", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n_problems", C.c_int), ("n_grids", C.c_int), ("max_levels", C.c_int),
                ("fine_rows", C.c_longlong), ("global_nnz", C.c_longlong), ("composite_real_nnz", C.c_longlong),
                ("composite_rows", C.c_longlong), ("composite_real_rows", C.c_longlong),
                ("composite_stored_nnz", C.c_longlong), ("omissions", C.c_longlong),
                ("composite_overhead", C.c_double), ("setup_hierarchy_s", C.c_double),
                ("setup_composite_s", C.c_double), ("setup_pack_s", C.c_double), ("setup_upload_s", C.c_double),
                ("device_bytes", C.c_longlong), ("tail_level", C.c_int), ("tail_block", C.c_int),
                ("autotune_s", C.c_double), ("composite_nnz", C.c_longlong), ("hybrid_level", C.c_int),
                ("schedule_cached", C.c_int), ("wide_levels", C.c_int),
                ("lds_levels", C.c_int), ("restrict_lds_levels", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("level", C.c_int), ("launches", C.c_int), ("ms", C.c_double),
                ("bytes", C.c_double), ("workgroups", C.c_int), ("block", C.c_int)]


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_IP = C.POINTER(C.c_int)
_DP = C.POINTER(C.c_double)
_LLP = C.POINTER(C.c_longlong)
_H = C.c_void_p

# name -> (restype, argtypes); every function declared in include/amgdd.h
SIGNATURES = {
    "amgdd_params_default": (None, [C.POINTER(Params)]),
    "amgdd_setup_composite": (_I, [_I, _IP, _IP, _DP, _IP, _I, C.POINTER(Params), _P, C.POINTER(_H)]),
    "amgdd_setup_composite_batch": (_I, [_I, _IP, C.POINTER(_IP), C.POINTER(_IP), C.POINTER(_DP), C.POINTER(_IP),
                                         _IP, C.POINTER(Params), _P, C.POINTER(_H)]),
    "amgdd_solve": (_I, [_H, _P, _P, _D, _I, C.POINTER(Info)]),
    "amgdd_solve_noalloc": (_I, [_H, _P, _P, _D, _I, C.POINTER(Info)]),
    "amgv_solve": (_I, [_H, _P, _P, _D, _I, C.POINTER(Info)]),
    "amgdd_solve_adjoint": (_I, [_H, _P, _P, _D, _I, C.POINTER(Info)]),
    "amgdd_face_gradient": (_I, [_H, _P, _P, _P, _P, _I, _P]),
    "amgdd_get_stats": (_I, [_H, C.POINTER(Stats)]),
    "amgdd_get_levels": (_I, [_H, _I, _IP, _IP, _LLP]),
    "amgdd_get_cf": (_I, [_H, _I, _I, C.POINTER(C.c_byte)]),
    "amgdd_get_operator": (_I, [_H, _I, _I, _I, _IP, _IP, _IP, _IP, _DP]),
    "amgdd_get_composite": (_I, [_H, _I, _I, _I, _IP, _IP, _IP, _IP]),
    "amgdd_get_history": (_I, [_H, _I, _DP, _I, _IP]),
    "amgdd_profile": (_I, [_H, _I, _I, C.POINTER(KernelTime), _I, _IP]),
    "amgdd_set_stream": (_I, [_H, _P]),
    "amgdd_last_error": (C.c_char_p, []),
    "amgdd_destroy": (None, [_H]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libamgdd.so and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1906_10575_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int):
    if st != OK:
        raise AmgddError(st, load().amgdd_last_error().decode())


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(_IP)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def default_params() -> Params:
    p = Params()
    load().amgdd_params_default(C.byref(p))
    return p


def _csr_arrays(A):
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int32)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    return indptr, indices, data


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, n=None, dtype=None):
    """Raw device pointer of a contiguous tensor on the HIP device, after
    checking its dtype (float64 unless given) and, when n is given, that it
    holds exactly n elements: the library reads and writes that many."""
    torch = _torch()
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on the HIP device")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, the handle needs exactly {n}")
    return C.c_void_p(t.data_ptr())


class Solver:
    """Handle over one problem or a batch of independent problems.

    A: scipy CSR matrix (or a list of them for a batch), part: int array(s) of
    subdomain ids, nparts: int(s), padding: int(s).  device=-1 gives a
    host-only handle (setup and introspection, no solve).  hybrid_level=L~ > 0
    makes solve() run hybrid AMG-DD V-cycles with AMG-DD on level L~;
    relax="cf" selects CF-ordered l1-Jacobi; coarsen="hmis" and
    interp="ext+i" the paper's best-practice AMG components."""

    def __init__(self, A, part, nparts, padding=1, n_fac=2, precision="fp64", device=0, theta=0.25,
                 max_coarse=16, max_levels=25, use_graph=True, stream=None, tail_level=-2, tail_block=0,
                 hybrid_level=0, relax="l1", coarsen="rs", interp="direct", interp_max=4,
                 padding_per_level=None):
        lib = load()
        batch = isinstance(A, (list, tuple))
        As = list(A) if batch else [A]
        parts = list(part) if batch else [part]
        nps = list(nparts) if batch else [nparts]
        pads = list(padding) if isinstance(padding, (list, tuple)) else [padding] * len(As)
        # per-level padding: one sequence (single problem) or one sequence or
        # None per problem (batch)
        if padding_per_level is None:
            ppl = [None] * len(As)
        elif batch:
            ppl = list(padding_per_level)
        else:
            ppl = [padding_per_level]
        if len(ppl) != len(As):
            raise ValueError("padding_per_level needs one entry per problem")
        ppl = [None if v is None else np.ascontiguousarray(v, dtype=np.int32) for v in ppl]
        prm = default_params()
        prm.theta = theta
        prm.max_coarse = max_coarse
        prm.max_levels = max_levels
        prm.n_fac = n_fac
        prm.precision = MIXED if precision in ("mixed", MIXED) else FP64
        prm.device = device
        prm.use_graph = 1 if use_graph else 0
        prm.tail_level = tail_level
        prm.tail_block = tail_block
        prm.hybrid_level = hybrid_level
        if relax not in ("l1", "cf"):
            raise ValueError(f"relax must be 'l1' or 'cf', not {relax!r}")
        prm.relax_order = 1 if relax == "cf" else 0
        if coarsen not in ("rs", "hmis") or interp not in ("direct", "ext+i"):
            raise ValueError(f"coarsen must be 'rs' or 'hmis' and interp 'direct' or 'ext+i', not {coarsen!r}, {interp!r}")
        prm.coarsen = 1 if coarsen == "hmis" else 0
        prm.interp = 1 if interp == "ext+i" else 0
        prm.interp_max = interp_max
        if stream is None and device >= 0:
            torch = _torch()
            stream = torch.cuda.current_stream(device).cuda_stream
        self._keep = []
        h = _H()
        arrs = [_csr_arrays(a) for a in As]
        pts = [np.ascontiguousarray(p, dtype=np.int32) for p in parts]
        self.sizes = [int(a.shape[0]) for a in As]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        def set_levels(pr, v):
            pr.n_padding_levels = 0 if v is None else int(v.size)
            pr.padding_per_level = None if v is None else _iptr(v)

        if not batch:
            prm.padding = pads[0]
            set_levels(prm, ppl[0])
            st = lib.amgdd_setup_composite(self.sizes[0], _iptr(arrs[0][0]), _iptr(arrs[0][1]), _dptr(arrs[0][2]),
                                           _iptr(pts[0]), int(nps[0]), C.byref(prm), C.c_void_p(stream), C.byref(h))
        else:
            n = len(As)
            prms = (Params * n)()
            for i in range(n):
                prms[i] = prm
                prms[i].padding = int(pads[i])
                set_levels(prms[i], ppl[i])
            ns = np.array(self.sizes, dtype=np.int32)
            rp = (_IP * n)(*[_iptr(a[0]) for a in arrs])
            ci = (_IP * n)(*[_iptr(a[1]) for a in arrs])
            va = (_DP * n)(*[_dptr(a[2]) for a in arrs])
            pp = (_IP * n)(*[_iptr(p) for p in pts])
            npa = np.array(nps, dtype=np.int32)
            st = lib.amgdd_setup_composite_batch(n, _iptr(ns), rp, ci, va, pp, _iptr(npa), prms, C.c_void_p(stream),
                                                 C.byref(h))
        _check(st)
        self._h = h
        self.device = device
        self.n_problems = len(As)
        self.n = int(self.offsets[-1])

    # ---------------------------------------------------------------- solves
    def _solve(self, fn, b, x, rtol, maxit):
        torch = _torch()
        bp = _dev_ptr(b, "b", self.n)
        if x is None:
            x = torch.zeros_like(b)
        info = Info()
        st = fn(self._h, bp, _dev_ptr(x, "x", self.n), float(rtol), int(maxit), C.byref(info))
        if st not in (OK, ENOCONV):
            _check(st)
        return x, info, st

    def solve(self, b, x=None, rtol=1e-8, maxit=100):
        """AMG-DD iterations; returns (x, Info, status) with status OK or ENOCONV."""
        return self._solve(load().amgdd_solve, b, x, rtol, maxit)

    def solve_noalloc(self, b, x=None, rtol=1e-8, maxit=100):
        """AMG-DD iterations with no device allocation inside the library call
        (x must be given for that: with x=None a zero tensor is allocated here)."""
        return self._solve(load().amgdd_solve_noalloc, b, x, rtol, maxit)

    def vsolve(self, b, x=None, rtol=1e-8, maxit=100):
        """AMG V(1,1) cycles on the same hierarchy."""
        return self._solve(load().amgv_solve, b, x, rtol, maxit)

    def solve_adjoint(self, g, lam=None, rtol=1e-8, maxit=100):
        return self._solve(load().amgdd_solve_adjoint, g, lam, rtol, maxit)

    def face_gradient(self, u, lam, face_i, face_j):
        """dL/dc per face; face_i in [0, n), face_j in [-1, n) (-1: boundary
        face), both of the same length.  Index ranges are checked on the host
        before anything is launched."""
        torch = _torch()
        fi_h = np.asarray(face_i.cpu() if isinstance(face_i, torch.Tensor) else face_i).ravel()
        fj_h = np.asarray(face_j.cpu() if isinstance(face_j, torch.Tensor) else face_j).ravel()
        if fi_h.size != fj_h.size:
            raise ValueError("face_i and face_j must have the same length")
        if fi_h.size and (fi_h.min() < 0 or fi_h.max() >= self.n or fj_h.min() < -1 or fj_h.max() >= self.n):
            raise ValueError(f"face indices out of range: need 0 <= face_i < {self.n} and -1 <= face_j < {self.n}")
        up, lp = _dev_ptr(u, "u", self.n), _dev_ptr(lam, "lam", self.n)
        fi = torch.as_tensor(fi_h.astype(np.int32), device=u.device)
        fj = torch.as_tensor(fj_h.astype(np.int32), device=u.device)
        out = torch.empty(fi.numel(), dtype=torch.float64, device=u.device)
        _check(load().amgdd_face_gradient(self._h, up, lp, C.c_void_p(fi.data_ptr()), C.c_void_p(fj.data_ptr()),
                                          int(fi.numel()), C.c_void_p(out.data_ptr())))
        return out

    # ---------------------------------------------------------- introspection
    def stats(self) -> dict:
        s = Stats()
        _check(load().amgdd_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def levels(self, prob=0):
        nl = C.c_int()
        _check(load().amgdd_get_levels(self._h, prob, C.byref(nl), None, None))
        n = np.zeros(nl.value, dtype=np.int32)
        z = np.zeros(nl.value, dtype=np.int64)
        _check(load().amgdd_get_levels(self._h, prob, C.byref(nl), _iptr(n), z.ctypes.data_as(_LLP)))
        return n, z

    def cf(self, prob, level):
        n, _ = self.levels(prob)
        out = np.zeros(int(n[level]), dtype=np.int8)
        _check(load().amgdd_get_cf(self._h, prob, level, out.ctypes.data_as(C.POINTER(C.c_byte))))
        return out

    def operator(self, prob, level, which=0):
        from scipy import sparse
        nr, nz = C.c_int(), C.c_int()
        _check(load().amgdd_get_operator(self._h, prob, level, which, C.byref(nr), C.byref(nz), None, None, None))
        rp = np.zeros(nr.value + 1, dtype=np.int32)
        ci = np.zeros(nz.value, dtype=np.int32)
        va = np.zeros(nz.value, dtype=np.float64)
        _check(load().amgdd_get_operator(self._h, prob, level, which, C.byref(nr), C.byref(nz), _iptr(rp), _iptr(ci),
                                         _dptr(va)))
        ncols = int(ci.max()) + 1 if ci.size else 0
        if which == 1:
            ncols = int(self.levels(prob)[0][level + 1])
        else:
            ncols = nr.value
        return sparse.csr_matrix((va, ci, rp), shape=(nr.value, ncols))

    def composite(self, prob, p, level):
        nr, nb, om = C.c_int(), C.c_int(), C.c_int()
        _check(load().amgdd_get_composite(self._h, prob, p, level, C.byref(nr), C.byref(nb), None, C.byref(om)))
        g = np.zeros(nb.value, dtype=np.int32)
        _check(load().amgdd_get_composite(self._h, prob, p, level, C.byref(nr), C.byref(nb), _iptr(g), C.byref(om)))
        return g, nr.value, om.value

    def history(self, prob=0):
        n = C.c_int()
        _check(load().amgdd_get_history(self._h, prob, None, 0, C.byref(n)))
        out = np.zeros(n.value)
        _check(load().amgdd_get_history(self._h, prob, _dptr(out), n.value, C.byref(n)))
        return out

    def profile(self, kind=0, reps=3):
        """Per-launch-site device time of one iteration (kind 0 AMG-DD, 1
        V-cycle): list of dicts name, level, launches, ms, bytes (per iteration)."""
        n = C.c_int()
        _check(load().amgdd_profile(self._h, kind, reps, None, 0, C.byref(n)))
        arr = (KernelTime * max(n.value, 1))()
        _check(load().amgdd_profile(self._h, kind, reps, arr, n.value, C.byref(n)))
        return [dict(name=a.name.decode(), level=a.level, launches=a.launches, ms=a.ms, bytes=a.bytes,
                     workgroups=a.workgroups, block=a.block) for a in arr[: n.value]]

    def set_stream(self, stream):
        _check(load().amgdd_set_stream(self._h, C.c_void_p(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().amgdd_destroy(self._h)
            self._h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols() -> List[str]:
    return list(SIGNATURES)
