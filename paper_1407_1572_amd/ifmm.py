"""Thin Python binding of the IFMM C-ABI (include/ifmm.h).

Argument marshalling only: every step of the factorisation and solve runs in
the gfx950 library ``libifmm.so`` built in this package directory.  Importing
this module does not load the library; constructing a solver does, and fails
loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libifmm.so")

KERNELS = {"inv_r": 0, "exp": 1, "log_a": 2, "inv_r_a": 3, "r2log_a": 4, "dexp_dell": 5}
DIAG = {"rowsum": 0, "const": 1, "vector": 2}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "singular pivot block",
          4: "refinement did not converge", 5: "HIP device error",
          6: "problem exceeds the fixed device workspace"}


class IFMMError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} (status {code})")
        self.code = code


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("ell", C.c_double), ("diag_mode", C.c_int), ("c0", C.c_double),
                ("diag", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("r_max", C.c_int), ("refine_tol", C.c_double), ("refine_maxit", C.c_int),
                ("box_lo", C.c_double * 2), ("box_size", C.c_double), ("profile", C.c_int),
                ("precision", C.c_int)]


class _SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("residual", C.c_double), ("history", C.c_double * 32),
                ("solve_ms", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("kappa", C.c_int), ("p", C.c_int), ("max_rank", C.c_int),
                ("level_max_rank", C.c_int * 16), ("level_mean_rank", C.c_double * 16),
                ("top_size", C.c_int), ("assembly_ms", C.c_double), ("factor_ms", C.c_double),
                ("last_solve_ms", C.c_double), ("factor_bytes", C.c_double),
                ("factor_flops", C.c_double), ("kernel_launches", C.c_int64 * 32),
                ("kernel_ms", C.c_double * 32), ("kernel_flops", C.c_double * 32),
                ("kernel_bytes", C.c_double * 32), ("precision", C.c_int),
                ("level_cap_hits", C.c_int * 16)]


KERNEL_FAMILIES = ["gemm", "add", "unused2", "qr", "rrqr", "formq", "stackqr", "inverse", "elim",
                   "touch_xform", "stack_win", "solve", "elim_other"]
PRECISIONS = {"fp64": 0, "fp32": 1}


def profile_mask(profile) -> int:
    """ifmm_options.profile from True/False (every family / off) or an
    iterable of family names (KERNEL_FAMILIES): only those are timed."""
    if profile is True or profile is False or profile is None:
        return 1 if profile else 0
    mask = 0
    for name in profile:
        mask |= 1 << (KERNEL_FAMILIES.index(name) + 1)
    return mask


_LIBS: dict = {}


def load(path: str | None = None):
    """Load (once) and type the C-ABI library; raises if it is missing."""
    path = path or LIB_PATH
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        raise FileNotFoundError(f"IFMM library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.ifmm_factor.argtypes = [P, C.c_int64, C.POINTER(_Kernel), C.c_double, C.c_int, C.c_int,
                                C.POINTER(_Options), P, C.POINTER(P)]
    lib.ifmm_factor.restype = C.c_int
    lib.ifmm_solve.argtypes = [P, P, P, C.c_int, P, C.POINTER(_SolveInfo)]
    lib.ifmm_solve.restype = C.c_int
    lib.ifmm_matvec.argtypes = [P, P, P, C.c_int, P]
    lib.ifmm_matvec.restype = C.c_int
    lib.ifmm_factor_batched.argtypes = [C.c_int, C.POINTER(P), C.POINTER(C.c_int64), C.POINTER(_Kernel),
                                        C.c_double, C.c_int, C.c_int, C.POINTER(_Options), C.c_int, P,
                                        C.POINTER(P), C.POINTER(C.c_int)]
    lib.ifmm_factor_batched.restype = C.c_int
    lib.ifmm_solve_batched.argtypes = [C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.c_int, C.c_int, P,
                                       C.POINTER(_SolveInfo), C.POINTER(C.c_int)]
    lib.ifmm_solve_batched.restype = C.c_int
    lib.ifmm_matvec_kernel.argtypes = [P, C.POINTER(_Kernel), P, P, C.c_int, P]
    lib.ifmm_matvec_kernel.restype = C.c_int
    lib.ifmm_matvec_noalloc.argtypes = [P, P, P, C.c_int, P]
    lib.ifmm_matvec_noalloc.restype = C.c_int
    lib.ifmm_matvec_noalloc_bytes.argtypes = [P, C.c_int]
    lib.ifmm_matvec_noalloc_bytes.restype = C.c_size_t
    lib.ifmm_diagonal.argtypes = [P, P, P]
    lib.ifmm_diagonal.restype = C.c_int
    lib.ifmm_stats.argtypes = [P, C.POINTER(_Stats)]
    lib.ifmm_stats.restype = C.c_int
    lib.ifmm_ranks.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.c_int]
    lib.ifmm_ranks.restype = C.c_int
    lib.ifmm_destroy.argtypes = [P]
    lib.ifmm_destroy.restype = None
    lib.ifmm_release_cached_memory.argtypes = []
    lib.ifmm_release_cached_memory.restype = None
    lib.ifmm_status_string.argtypes = [C.c_int]
    lib.ifmm_status_string.restype = C.c_char_p
    _LIBS[path] = lib
    return lib


def release_cached_memory(lib_path: str | None = None):
    """Return the device blocks cached by destroyed factors to the runtime."""
    load(lib_path).ifmm_release_cached_memory()


def _stream_handle(t):
    import torch
    if t.is_cuda:
        return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)
    return C.c_void_p(0)


class IFMMSolver:
    """ifmm_factor(points, kernel, eps, leaf_size, rank) / ifmm_solve(b).

    points: torch float64 tensor [N, 2] on the GPU.  b for ``solve`` is [N]
    or [N, nrhs] on the same device.  diag "vector" takes A_ii from
    ``diag_values`` ([N] on the same device, caller's order; c0 unused).
    precision "fp32" stores the factor's
    blocks in FP32 (the mixed-precision factor; pivot inverses, the FMM
    product, residuals and vectors stay FP64 and refinement recovers FP64
    accuracy).
    """

    def __init__(self, points, kernel: str = "inv_r", ell: float = 0.0, diag: str = "rowsum",
                 c0: float = 1.0, eps: float = 1e-8, leaf_size: int = 64, rank: int = 36,
                 r_max: int = 0, refine_tol: float = 0.0, refine_maxit: int = 30,
                 box=None, profile=False, precision: str = "fp64",
                 lib_path: str | None = None, diag_values=None):
        import torch
        self._lib = load(lib_path)
        if lib_path is None and not points.is_cuda:
            raise ValueError("points must be a GPU tensor")
        pts = points.to(torch.float64).contiguous()
        self.n = int(pts.shape[0])
        self.device = pts.device
        dv = None
        if diag == "vector":
            if diag_values is None:
                raise ValueError('diag="vector" needs diag_values')
            dv = diag_values.to(device=pts.device, dtype=torch.float64).contiguous()
            if dv.shape != (self.n,):
                raise ValueError("diag_values must have shape [N]")
        k = _Kernel(KERNELS[kernel], float(ell), DIAG[diag], float(c0),
                    C.c_void_p(dv.data_ptr()) if dv is not None else C.c_void_p(0))
        o = _Options()
        o.r_max = int(r_max)
        o.refine_tol = float(refine_tol)
        o.refine_maxit = int(refine_maxit)
        o.profile = profile_mask(profile)
        o.precision = PRECISIONS[precision]
        if box is not None:
            o.box_lo[0], o.box_lo[1], o.box_size = float(box[0]), float(box[1]), float(box[2])
        h = C.c_void_p()
        st = self._lib.ifmm_factor(C.c_void_p(pts.data_ptr()), self.n, C.byref(k), float(eps),
                                   int(leaf_size), int(rank), C.byref(o), _stream_handle(pts),
                                   C.byref(h))
        if st != 0:
            raise IFMMError(st, "ifmm_factor")
        self._h = h
        self.last_info = None

    @classmethod
    def _from_handle(cls, lib, h, n, device):
        s = cls.__new__(cls)
        s._lib, s._h, s.n, s.device, s.last_info = lib, h, n, device, None
        return s

    def _cols(self, v):
        import torch
        v = v.to(device=self.device, dtype=torch.float64)
        one = v.dim() == 1
        vt = (v.reshape(1, -1) if one else v.t()).contiguous()  # [nrhs][N]
        return vt, one

    def solve(self, b, check: bool = True):
        import torch
        bt, one = self._cols(b)
        xt = torch.empty_like(bt)
        info = _SolveInfo()
        st = self._lib.ifmm_solve(self._h, C.c_void_p(bt.data_ptr()), C.c_void_p(xt.data_ptr()),
                                  int(bt.shape[0]), _stream_handle(bt), C.byref(info))
        self.last_info = {"iterations": info.iterations, "residual": info.residual,
                          "history": list(info.history[:max(1, info.iterations + 1)]),
                          "solve_ms": info.solve_ms, "status": st}
        if st != 0 and (check or st != 4):
            raise IFMMError(st, "ifmm_solve")
        return xt[0] if one else xt.t()

    def matvec(self, x):
        import torch
        xt, one = self._cols(x)
        yt = torch.empty_like(xt)
        st = self._lib.ifmm_matvec(self._h, C.c_void_p(xt.data_ptr()), C.c_void_p(yt.data_ptr()),
                                   int(xt.shape[0]), _stream_handle(xt))
        if st != 0:
            raise IFMMError(st, "ifmm_matvec")
        return yt[0] if one else yt.t()

    def matvec_kernel(self, x, kernel: str, ell: float = 0.0, diag: str = "const", c0: float = 0.0,
                      diag_values=None):
        """y = A_k x for another kernel on this factor's tree and bases (e.g.
        kernel "dexp_dell", diag "const", c0 = 0: dA/d ell of the exp kernel)."""
        import torch
        xt, one = self._cols(x)
        dv = None
        if diag == "vector":
            dv = diag_values.to(device=self.device, dtype=torch.float64).contiguous()
        k = _Kernel(KERNELS[kernel], float(ell), DIAG[diag], float(c0),
                    C.c_void_p(dv.data_ptr()) if dv is not None else C.c_void_p(0))
        yt = torch.empty_like(xt)
        st = self._lib.ifmm_matvec_kernel(self._h, C.byref(k), C.c_void_p(xt.data_ptr()),
                                          C.c_void_p(yt.data_ptr()), int(xt.shape[0]), _stream_handle(xt))
        if st != 0:
            raise IFMMError(st, "ifmm_matvec_kernel")
        return yt[0] if one else yt.t()

    def matvec_noalloc(self, x, out):
        """y = A x into ``out`` ([N] or [N, nrhs] float64, contiguous in the
        ABI's [nrhs][N] layout: a 1-D tensor, or the transpose of a
        contiguous [nrhs, N] tensor) with the library's fixed device
        workspace: no device memory is allocated by the library.  Enqueued on
        the current stream."""
        import torch
        xt, one = self._cols(x)
        yt = out.reshape(1, -1) if one else out.t()
        if not (yt.is_contiguous() and yt.dtype == torch.float64 and yt.shape == xt.shape):
            raise ValueError("out must match x, float64, [nrhs][N] contiguous")
        st = self._lib.ifmm_matvec_noalloc(self._h, C.c_void_p(xt.data_ptr()), C.c_void_p(yt.data_ptr()),
                                           int(xt.shape[0]), _stream_handle(xt))
        if st != 0:
            raise IFMMError(st, "ifmm_matvec_noalloc")
        return out

    def matvec_noalloc_bytes(self, nrhs: int = 1) -> int:
        return int(self._lib.ifmm_matvec_noalloc_bytes(self._h, int(nrhs)))

    def diagonal(self):
        import torch
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        st = self._lib.ifmm_diagonal(self._h, C.c_void_p(d.data_ptr()), _stream_handle(d))
        if st != 0:
            raise IFMMError(st, "ifmm_diagonal")
        return d

    def stats(self) -> dict:
        s = _Stats()
        st = self._lib.ifmm_stats(self._h, C.byref(s))
        if st != 0:
            raise IFMMError(st, "ifmm_stats")
        k = s.kappa
        return {"n": s.n, "kappa": k, "p": s.p, "max_rank": s.max_rank,
                "level_max_rank": {l: s.level_max_rank[l] for l in range(2, k + 1)},
                "level_mean_rank": {l: s.level_mean_rank[l] for l in range(2, k + 1)},
                "level_cap_hits": {l: s.level_cap_hits[l] for l in range(2, k + 1)},
                "top_size": s.top_size, "assembly_ms": s.assembly_ms, "factor_ms": s.factor_ms,
                "last_solve_ms": s.last_solve_ms, "factor_bytes": s.factor_bytes,
                "factor_flops": s.factor_flops,
                "precision": {v: k for k, v in PRECISIONS.items()}.get(s.precision, s.precision),
                # "<family>" computes in FP64, "<family>_f32" in FP32
                "kernels": {name + ("_f32" if q else ""):
                            {"launches": s.kernel_launches[i + 16 * q], "ms": s.kernel_ms[i + 16 * q],
                             "flops": s.kernel_flops[i + 16 * q], "bytes": s.kernel_bytes[i + 16 * q]}
                            for q in (0, 1) for i, name in enumerate(KERNEL_FAMILIES)
                            if s.kernel_launches[i + 16 * q] > 0}}

    def ranks(self, level: int) -> np.ndarray:
        out = (C.c_int * (4 ** level))()
        st = self._lib.ifmm_ranks(self._h, int(level), out, 4 ** level)
        if st != 0:
            raise IFMMError(st, "ifmm_ranks")
        return np.frombuffer(out, dtype=np.int32).copy()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ifmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor_batched(points, kernels, eps: float = 1e-8, leaf_size: int = 64, rank: int = 36,
                   r_max: int = 0, refine_tol: float = 0.0, refine_maxit: int = 30,
                   precision: str = "fp64", threads: int = 0, lib_path: str | None = None):
    """ifmm_factor_batched: factor independent problems concurrently.

    points: list of [N_i, 2] float64 GPU tensors; kernels: list of dicts
    {kind, ell, diag, c0} (one per problem).  Returns a list of IFMMSolver.
    Raises IFMMError if any factorisation failed (the others are freed)."""
    import torch
    lib = load(lib_path)
    cnt = len(points)
    pts = [p.to(torch.float64).contiguous() for p in points]
    P = (C.c_void_p * cnt)(*[p.data_ptr() for p in pts])
    N = (C.c_int64 * cnt)(*[int(p.shape[0]) for p in pts])
    K = (_Kernel * cnt)(*[_Kernel(KERNELS[k["kind"]], float(k.get("ell", 0.0)), DIAG[k.get("diag", "const")],
                                  float(k.get("c0", 1.0)), C.c_void_p(0)) for k in kernels])
    o = _Options()
    o.r_max, o.refine_tol, o.refine_maxit = int(r_max), float(refine_tol), int(refine_maxit)
    o.precision = PRECISIONS[precision]
    H = (C.c_void_p * cnt)()
    S = (C.c_int * cnt)()
    st = lib.ifmm_factor_batched(cnt, P, N, K, float(eps), int(leaf_size), int(rank), C.byref(o), int(threads),
                                 _stream_handle(pts[0]), H, S)
    solvers = [IFMMSolver._from_handle(lib, C.c_void_p(H[i]), int(N[i]), pts[i].device) if H[i] else None
               for i in range(cnt)]
    if st != 0:
        for s in solvers:
            if s is not None:
                s.close()
        raise IFMMError(st, "ifmm_factor_batched")
    return solvers


def solve_batched(solvers, rhs, threads: int = 0):
    """ifmm_solve_batched: x_i = A_i^-1 b_i for every solver concurrently;
    rhs: list of [N_i, nrhs] (or [N_i]) GPU tensors, one nrhs for all.
    Returns the list of solutions; each solver's last_info is set."""
    import torch
    cnt = len(solvers)
    cols = [s._cols(b) for s, b in zip(solvers, rhs)]
    nrhs = int(cols[0][0].shape[0])
    xs = [torch.empty_like(bt) for bt, _ in cols]
    H = (C.c_void_p * cnt)(*[s._h.value for s in solvers])
    B = (C.c_void_p * cnt)(*[bt.data_ptr() for bt, _ in cols])
    X = (C.c_void_p * cnt)(*[x.data_ptr() for x in xs])
    I = (_SolveInfo * cnt)()
    S = (C.c_int * cnt)()
    st = solvers[0]._lib.ifmm_solve_batched(cnt, H, B, X, nrhs, int(threads), _stream_handle(cols[0][0]), I, S)
    for i, s in enumerate(solvers):
        s.last_info = {"iterations": I[i].iterations, "residual": I[i].residual,
                       "history": list(I[i].history[:max(1, I[i].iterations + 1)]),
                       "solve_ms": I[i].solve_ms, "status": S[i]}
    if st != 0 and st != 4:
        raise IFMMError(st, "ifmm_solve_batched")
    return [x[0] if one else x.t() for x, (_, one) in zip(xs, cols)]
