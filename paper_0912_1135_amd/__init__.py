"""MI355X-native randomized orthogonal projection (Rokhlin & Tygert).

Python binding of ``librtproj.so`` (the C ABI declared in include/rtproj.h).
Argument marshalling only: every step runs in the library's gfx950 kernels.
PyTorch supplies device memory and streams.  There is no CPU fallback: if the
library is missing, every call raises.

Layout conventions (torch view of the C layouts):
  A  (m, n) float64 CUDA tensor with unit column stride (row-major m x n)
  B  (k, n) float64 CUDA tensor with unit column stride: row c is right-hand
     side c (column-major n x k in the C ABI); Z and Y have the same shape
  X  (k, m) float64: row c is the least-squares solution for right-hand side c
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtproj.so")
_lib = None

PREC_FP64, PREC_MIXED_FP32, PREC_MIXED_BF16, PREC_MIXED_BF16X3 = 0, 1, 2, 3
STATUS = {0: "OK", 1: "ERR_INVALID_ARG", 2: "ERR_ALLOC", 3: "ERR_DEVICE", 4: "ERR_STATE",
          5: "ERR_RANK", 6: "ERR_NOCONV", 7: "ERR_UNSUPPORTED"}


class RtprojError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("l", ctypes.c_int64), ("np", ctypes.c_int64),
                ("kappa_est", ctypes.c_double), ("rdiag_min", ctypes.c_double), ("precision", ctypes.c_int),
                ("refine_steps", ctypes.c_int), ("refine_last_ratio", ctypes.c_double),
                ("qrcp_blocks", ctypes.c_int), ("sketch_bits", ctypes.c_int), ("w_bits", ctypes.c_int),
                ("gram_bits", ctypes.c_int), ("sketch_escalated", ctypes.c_int), ("gram_cond_est", ctypes.c_double),
                ("t_stage_ms", ctypes.c_double * 16),
                ("stage_calls", ctypes.c_int64 * 16),
                ("qr_mode", ctypes.c_int), ("inverse", ctypes.c_int), ("inverse_iters", ctypes.c_int),
                ("inverse_resid", ctypes.c_double), ("refine_plain", ctypes.c_int), ("refine_comp", ctypes.c_int),
                ("resid_mode", ctypes.c_int), ("refine_status", ctypes.c_int), ("refine_rho_est", ctypes.c_double),
                ("refine_err_est", ctypes.c_double), ("refine_rho_model", ctypes.c_double),
                ("method", ctypes.c_int), ("comp_method", ctypes.c_int)]

STAGES = ["sketch", "qrcp", "rinv_trsm", "w_gemm", "gram_syrk", "gram_inv", "minv_form", "ab",
          "minv", "refine_atx", "refine_ab", "final_atx", "qr_r0", "refine_atx_plain", "refine_ab_plain",
          "final_atx_plain"]
QR_AUTO, QR_DIRECT, QR_TWO_STAGE, QR_TWO_STAGE_WG = 0, 1, 2, 3
INV_AUTO, INV_NEWTON_SCHULZ, INV_CHOLESKY = 0, 1, 2
RESID_AUTO, RESID_PLAIN, RESID_S_ONLY, RESID_FULL = 0, 1, 2, 3
METHOD_RANDOMIZED, METHOD_CLASSICAL, METHOD_KRYLOV = 0, 1, 2
COMP_AUTO, COMP_DOT2, COMP_INT8 = 0, 1, 2


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        i64, u64, vp, ip, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.rtproj_plan_create.argtypes = [i64, i64, i64, u64, ctypes.POINTER(vp)]
        L.rtproj_plan_destroy.argtypes = [vp]
        L.rtproj_plan_set_stream.argtypes = [vp, vp]
        L.rtproj_plan_set_precision.argtypes = [vp, ip]
        L.rtproj_plan_set_refinement.argtypes = [vp, ip, dp]
        L.rtproj_plan_set_qr.argtypes = [vp, ip]
        L.rtproj_plan_set_inverse.argtypes = [vp, ip]
        L.rtproj_plan_set_residual.argtypes = [vp, ip]
        L.rtproj_plan_set_compensation.argtypes = [vp, ip]
        L.rtproj_plan_set_method.argtypes = [vp, ip]
        L.rtproj_plan_set_sketch_matrix.argtypes = [vp, vp, i64]
        L.rtproj_plan_set_krylov.argtypes = [vp, ip]
        L.rtproj_plan_set_autotune.argtypes = [vp, ip]
        L.rtproj_autotune_save.argtypes = [ctypes.c_char_p]
        L.rtproj_autotune_load.argtypes = [ctypes.c_char_p]
        L.rtproj_autotune_entries.restype = ip
        L.rtproj_plan_set_w_bits.argtypes = [vp, ip]
        L.rtproj_plan_status.argtypes = [vp]
        L.rtproj_precondition.argtypes = [vp, vp, i64]
        L.rtproj_project_null.argtypes = [vp, vp, i64, i64, vp, i64]
        L.rtproj_project_row.argtypes = [vp, vp, i64, i64, vp, i64]
        L.rtproj_lstsq.argtypes = [vp, vp, i64, i64, vp, i64]
        L.rtproj_project_all.argtypes = [vp, vp, i64, i64, vp, i64, vp, i64, vp, i64]
        L.rtproj_project_all_noalloc.argtypes = [vp, vp, i64, i64, vp, i64, vp, i64, vp, i64]
        L.rtproj_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.rtproj_plan_set_timing.argtypes = [vp, ip]
        L.rtproj_plan_export.argtypes = [vp, vp, i64, vp, vp, vp]
        L.rtproj_sketch_tables.argtypes = [vp, vp, vp, vp, vp, vp]
        L.rtproj_batch_create.argtypes = [i64, vp, vp, vp, u64, ctypes.POINTER(vp)]
        L.rtproj_batch_destroy.argtypes = [vp]
        L.rtproj_batch_set_stream.argtypes = [vp, vp]
        L.rtproj_batch_set_refinement.argtypes = [vp, ip]
        L.rtproj_batch_set_graph.argtypes = [vp, ip]
        L.rtproj_batch_set_precision.argtypes = [vp, ip]
        L.rtproj_batch_precondition.argtypes = [vp, vp, vp]
        L.rtproj_batch_precondition_scaled.argtypes = [vp, vp, vp, vp]
        L.rtproj_batch_project_all.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rtproj_batch_status.argtypes = [vp, vp]
        L.rtproj_batch_member_info.argtypes = [vp, i64, ctypes.POINTER(_Info)]
        L.rtproj_batch_member_tables.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.rtproj_batch_set_timing.argtypes = [vp, ip]
        L.rtproj_batch_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.rtproj_cplan_create.argtypes = [i64, i64, i64, u64, ctypes.POINTER(vp)]
        L.rtproj_cplan_destroy.argtypes = [vp]
        L.rtproj_cplan_real.argtypes = [vp]
        L.rtproj_cplan_real.restype = vp
        L.rtproj_cprecondition.argtypes = [vp, vp, i64]
        L.rtproj_cproject_all.argtypes = [vp, vp, i64, i64, vp, i64, vp, i64, vp, i64]
        L.rtproj_status_string.argtypes = [ip]
        L.rtproj_status_string.restype = ctypes.c_char_p
        L.rtproj_last_error.restype = ctypes.c_char_p
        for name in ["rtproj_plan_create", "rtproj_plan_destroy", "rtproj_plan_set_stream",
                     "rtproj_plan_set_precision", "rtproj_plan_set_refinement", "rtproj_plan_set_qr", "rtproj_plan_set_inverse",
                     "rtproj_plan_set_residual", "rtproj_plan_set_compensation", "rtproj_plan_set_w_bits", "rtproj_plan_status",
                     "rtproj_plan_set_method", "rtproj_plan_set_sketch_matrix", "rtproj_plan_set_krylov",
                     "rtproj_plan_set_autotune", "rtproj_autotune_save", "rtproj_autotune_load",
                     "rtproj_precondition",
                     "rtproj_project_null", "rtproj_project_row", "rtproj_lstsq", "rtproj_project_all",
                     "rtproj_project_all_noalloc",
                     "rtproj_plan_info", "rtproj_plan_export", "rtproj_sketch_tables",
                     "rtproj_plan_set_timing", "rtproj_batch_create", "rtproj_batch_destroy",
                     "rtproj_batch_set_stream", "rtproj_batch_set_refinement", "rtproj_batch_set_graph",
                     "rtproj_batch_set_precision",
                     "rtproj_batch_precondition", "rtproj_batch_project_all", "rtproj_batch_status",
                     "rtproj_batch_member_info", "rtproj_batch_set_timing", "rtproj_batch_info",
                     "rtproj_batch_precondition_scaled", "rtproj_batch_member_tables", "rtproj_cplan_create",
                     "rtproj_cplan_destroy", "rtproj_cprecondition", "rtproj_cproject_all"]:
            getattr(L, name).restype = ip
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise RtprojError(status, lib().rtproj_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t, name, rows=None, cols=None, device=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit stride along its last dimension")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name} has {t.shape[0]} rows, expected {rows}")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name} has {t.shape[1]} columns, expected {cols}")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} rows overlap (row stride {t.stride(0)} < {t.shape[1]})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


class Plan:
    """A plan for m x n matrices sketched to l columns (rtproj_plan)."""

    def __init__(self, m: int, n: int, l: int, seed: int, stream=None):
        h = ctypes.c_void_p()
        _check(lib().rtproj_plan_create(m, n, l, seed, ctypes.byref(h)))
        self.handle, self.m, self.n, self.l, self.seed = h, m, n, l, seed
        self._A = None
        self.set_stream(stream)

    def close(self):
        if self.handle:
            lib().rtproj_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        """Enqueue on `stream` (a torch.cuda.Stream; default: torch's current stream)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().rtproj_plan_set_stream(self.handle, ctypes.c_void_p(s.cuda_stream)))

    def set_precision(self, precision: int):
        _check(lib().rtproj_plan_set_precision(self.handle, precision))

    def set_qr(self, mode: int):
        """Pivoted-QR method (QR_AUTO, QR_DIRECT, QR_TWO_STAGE, QR_TWO_STAGE_WG)."""
        _check(lib().rtproj_plan_set_qr(self.handle, mode))

    def set_inverse(self, method: int):
        """Gram inverse (INV_AUTO, INV_NEWTON_SCHULZ, INV_CHOLESKY)."""
        _check(lib().rtproj_plan_set_inverse(self.handle, method))

    def set_refinement(self, max_steps: int, rtol: float = 0.0):
        _check(lib().rtproj_plan_set_refinement(self.handle, max_steps, rtol))

    def set_residual(self, mode: int):
        """Arithmetic of the refinement residuals (RESID_AUTO, RESID_PLAIN, RESID_S_ONLY, RESID_FULL)."""
        _check(lib().rtproj_plan_set_residual(self.handle, mode))

    def set_compensation(self, method: int):
        """Form of the compensated products of the refinement: COMP_AUTO (the
        int8 matrix cores from 16 right-hand sides on), COMP_DOT2 (vector
        units) or COMP_INT8 (exact digit products on the int8 matrix cores)."""
        _check(lib().rtproj_plan_set_compensation(self.handle, method))

    def set_method(self, method: int):
        """METHOD_RANDOMIZED (default), METHOD_CLASSICAL (eq. basic_identity
        with a pivoted QR of A A^T, the comparison scheme of Sec. 5) or
        METHOD_KRYLOV (conjugate gradients on P^{-1}A, the iterative variant)."""
        _check(lib().rtproj_plan_set_method(self.handle, method))

    def set_autotune(self, enable: bool):
        """Time candidate configurations of P^{-1}A and its Gram for new shapes."""
        _check(lib().rtproj_plan_set_autotune(self.handle, 1 if enable else 0))

    def set_krylov(self, iters: int):
        """Conjugate-gradient iterations per solve of METHOD_KRYLOV."""
        _check(lib().rtproj_plan_set_krylov(self.handle, iters))

    def set_sketch_matrix(self, G=None):
        """Sketch with a dense (n, l) float64 CUDA tensor G (S = A G) instead
        of the randomized Fourier transform; None restores the latter."""
        if G is None:
            _check(lib().rtproj_plan_set_sketch_matrix(self.handle, None, 0))
        else:
            _check_tensor(G, "G", self.n, self.l)
            _check(lib().rtproj_plan_set_sketch_matrix(self.handle, _ptr(G), G.stride(0)))
        self._G = G  # the plan borrows G

    def set_w_bits(self, bits: int):
        """Precision of P^{-1}A in the reduced-precision modes: 0 automatic, 32 or 64 forced."""
        _check(lib().rtproj_plan_set_w_bits(self.handle, bits))

    def status(self):
        """Waits for the plan's stream; raises RtprojError (ERR_NOCONV) when the
        last projection's refinement did not converge."""
        _check(lib().rtproj_plan_status(self.handle))

    def precondition(self, A):
        _check_tensor(A, "A", self.m, self.n)
        _check(lib().rtproj_precondition(self.handle, _ptr(A), A.stride(0)))
        self._A = A  # the plan borrows A

    def _rhs(self, B):
        _check_tensor(B, "B", None, self.n)
        return B.shape[0]

    def project_null(self, B, out=None):
        import torch
        k = self._rhs(B)
        Z = out if out is not None else torch.empty_like(B)
        _check_tensor(Z, "Z", k, self.n, B.device)
        _check(lib().rtproj_project_null(self.handle, _ptr(B), B.stride(0), k, _ptr(Z), Z.stride(0)))
        return Z

    def project_row(self, B, out=None):
        import torch
        k = self._rhs(B)
        Y = out if out is not None else torch.empty_like(B)
        _check_tensor(Y, "Y", k, self.n, B.device)
        _check(lib().rtproj_project_row(self.handle, _ptr(B), B.stride(0), k, _ptr(Y), Y.stride(0)))
        return Y

    def lstsq(self, B, out=None):
        import torch
        k = self._rhs(B)
        X = out if out is not None else torch.empty((k, self.m), dtype=B.dtype, device=B.device)
        _check_tensor(X, "X", k, self.m, B.device)
        _check(lib().rtproj_lstsq(self.handle, _ptr(B), B.stride(0), k, _ptr(X), X.stride(0)))
        return X

    def project_all(self, B, Z=None, Y=None, X=None, want=(True, True, True)):
        import torch
        k = self._rhs(B)
        if want[0] and Z is None:
            Z = torch.empty_like(B)
        if want[1] and Y is None:
            Y = torch.empty_like(B)
        if want[2] and X is None:
            X = torch.empty((k, self.m), dtype=B.dtype, device=B.device)
        for t, name, rows, cols in ((Z, "Z", k, self.n), (Y, "Y", k, self.n), (X, "X", k, self.m)):
            if t is not None:
                _check_tensor(t, name, rows, cols, B.device)
        _check(lib().rtproj_project_all(self.handle, _ptr(B), B.stride(0), k,
                                        _ptr(Z), Z.stride(0) if Z is not None else 0,
                                        _ptr(Y), Y.stride(0) if Y is not None else 0,
                                        _ptr(X), X.stride(0) if X is not None else 0))
        return Z, Y, X

    def project_all_noalloc(self, B, Z, Y, X):
        """rtproj_project_all_noalloc: as project_all with caller-given outputs
        (None to skip one), the workspace from the library's static array."""
        k = self._rhs(B)
        for t, name, rows, cols in ((Z, "Z", k, self.n), (Y, "Y", k, self.n), (X, "X", k, self.m)):
            if t is not None:
                _check_tensor(t, name, rows, cols, B.device)
        _check(lib().rtproj_project_all_noalloc(self.handle, _ptr(B), B.stride(0), k,
                                                _ptr(Z), Z.stride(0) if Z is not None else 0,
                                                _ptr(Y), Y.stride(0) if Y is not None else 0,
                                                _ptr(X), X.stride(0) if X is not None else 0))
        return Z, Y, X

    def set_timing(self, enable: bool):
        _check(lib().rtproj_plan_set_timing(self.handle, 1 if enable else 0))

    def info(self) -> dict:
        inf = _Info()
        _check(lib().rtproj_plan_info(self.handle, ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in _Info._fields_ if f not in ("t_stage_ms", "stage_calls")}
        d["stage_ms"] = {name: inf.t_stage_ms[i] for i, name in enumerate(STAGES)}
        d["stage_calls"] = {name: inf.stage_calls[i] for i, name in enumerate(STAGES)}
        return d

    def export(self):
        """Device copies of S (m x l), R (m x m), piv (m) and Minv (m x m), the
        approximation of (A A^T)^{-1} that the projections apply."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        S = torch.empty((self.m, self.l), dtype=torch.float64, device=dev)
        R = torch.empty((self.m, self.m), dtype=torch.float64, device=dev)
        piv = torch.empty(self.m, dtype=torch.int32, device=dev)
        Mi = torch.empty((self.m, self.m), dtype=torch.float64, device=dev)
        _check(lib().rtproj_plan_export(self.handle, _ptr(S), self.l, _ptr(R), _ptr(piv), _ptr(Mi)))
        return dict(S=S, R=R, piv=piv, Minv=Mi)

    def sketch_tables(self) -> dict:
        import numpy as np
        dims = np.zeros(3, dtype=np.int64)
        _check(lib().rtproj_sketch_tables(self.handle, dims.ctypes.data, None, None, None, None))
        np_, n1, n2 = (int(v) for v in dims)
        sign = np.empty(np_, dtype=np.int8)
        sigma = np.empty(n1, dtype=np.int32)
        tau = np.empty(n2, dtype=np.int32)
        J = np.empty(self.l, dtype=np.int32)
        _check(lib().rtproj_sketch_tables(self.handle, None, sign.ctypes.data, sigma.ctypes.data,
                                          tau.ctypes.data, J.ctypes.data))
        return dict(np=np_, n1=n1, n2=n2, sign=sign, sigma=sigma, tau=tau, J=J)


def _check_complex(t, name, rows=None, cols=None, device=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit stride along its last dimension")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name} has {t.shape[0]} rows, expected {rows}")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name} has {t.shape[1]} columns, expected {cols}")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} rows overlap")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


class CPlan:
    """A plan for complex m x n matrices (rtproj_cplan): projections with the
    conjugate transpose A^*.  A (m, n), B/Z/Y (k, n), X (k, m) complex128
    CUDA tensors.  ``real`` is the underlying real plan (sizes 2m, 2n, 2l)
    for the setters, info() and status()."""

    def __init__(self, m: int, n: int, l: int, seed: int, stream=None):
        h = ctypes.c_void_p()
        _check(lib().rtproj_cplan_create(m, n, l, seed, ctypes.byref(h)))
        self.handle, self.m, self.n, self.l = h, m, n, l
        real = object.__new__(Plan)
        real.handle = ctypes.c_void_p(lib().rtproj_cplan_real(h))
        real.m, real.n, real.l, real.seed, real._A = 2 * m, 2 * n, 2 * l, seed, None
        real.close = lambda: None   # owned by the complex plan
        self.real = real
        self.real.set_stream(stream)

    def close(self):
        if self.handle:
            lib().rtproj_cplan_destroy(self.handle)
            self.handle = None
            self.real.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def precondition(self, A):
        _check_complex(A, "A", self.m, self.n)
        _check(lib().rtproj_cprecondition(self.handle, _ptr(A), A.stride(0)))

    def project_all(self, B, Z=None, Y=None, X=None, want=(True, True, True)):
        import torch
        _check_complex(B, "B", None, self.n)
        k = B.shape[0]
        if want[0] and Z is None:
            Z = torch.empty_like(B)
        if want[1] and Y is None:
            Y = torch.empty_like(B)
        if want[2] and X is None:
            X = torch.empty((k, self.m), dtype=B.dtype, device=B.device)
        for t, name, rows, cols in ((Z, "Z", k, self.n), (Y, "Y", k, self.n), (X, "X", k, self.m)):
            if t is not None:
                _check_complex(t, name, rows, cols, B.device)
        _check(lib().rtproj_cproject_all(self.handle, _ptr(B), B.stride(0), k,
                                         _ptr(Z), Z.stride(0) if Z is not None else 0,
                                         _ptr(Y), Y.stride(0) if Y is not None else 0,
                                         _ptr(X), X.stride(0) if X is not None else 0))
        return Z, Y, X


def autotune_save(path: str):
    _check(lib().rtproj_autotune_save(path.encode()))


def autotune_load(path: str):
    _check(lib().rtproj_autotune_load(path.encode()))


def autotune_entries() -> int:
    return int(lib().rtproj_autotune_entries())


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))(*[t.data_ptr() if t is not None else None for t in ts])
    return arr


def _i64s(vals):
    return (ctypes.c_int64 * len(vals))(*vals)


class Batch:
    """Many independent problems of uneven sizes, one grouped launch per stage
    (rtproj_batch).  Member i: an m[i] x n[i] matrix sketched to l[i] columns."""

    def __init__(self, ms, ns, ls, seed: int, stream=None):
        assert len(ms) == len(ns) == len(ls) and len(ms) > 0
        h = ctypes.c_void_p()
        self.count = len(ms)
        self.ms, self.ns, self.ls = list(ms), list(ns), list(ls)
        _check(lib().rtproj_batch_create(self.count, _i64s(self.ms), _i64s(self.ns), _i64s(self.ls), seed,
                                         ctypes.byref(h)))
        self.handle = h
        self._A = None
        self.set_stream(stream)

    def close(self):
        if self.handle:
            lib().rtproj_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().rtproj_batch_set_stream(self.handle, ctypes.c_void_p(s.cuda_stream)))

    def set_refinement(self, steps: int):
        _check(lib().rtproj_batch_set_refinement(self.handle, steps))

    def set_graph(self, enable: bool):
        _check(lib().rtproj_batch_set_graph(self.handle, 1 if enable else 0))

    def set_precision(self, precision: int):
        """PREC_FP64 (default), PREC_MIXED_FP32 (binary32 Gram on MFMA) or
        PREC_MIXED_BF16X3 (split-bfloat16 Gram of binary32 P^{-1}A)."""
        _check(lib().rtproj_batch_set_precision(self.handle, precision))

    def precondition(self, As, col_scales=None):
        """As[i]: (m_i, n_i) float64 CUDA tensors; col_scales[i] (optional):
        (n_i,) float64 CUDA tensors, member i then works on A[i] diag(d[i]).
        Both are borrowed (kept referenced here) until the next precondition."""
        assert len(As) == self.count
        for i, A in enumerate(As):
            _check_tensor(A, f"A[{i}]", self.ms[i], self.ns[i])
        if col_scales is None:
            _check(lib().rtproj_batch_precondition(self.handle, _ptrs(As), _i64s([A.stride(0) for A in As])))
        else:
            import torch
            assert len(col_scales) == self.count
            for i, d in enumerate(col_scales):
                if d is not None and (not isinstance(d, torch.Tensor) or d.dtype != torch.float64 or not d.is_cuda
                                      or d.dim() != 1 or d.shape[0] != self.ns[i] or d.stride(0) != 1):
                    raise ValueError(f"col_scales[{i}] must be a contiguous float64 CUDA vector of length n")
            _check(lib().rtproj_batch_precondition_scaled(self.handle, _ptrs(As), _i64s([A.stride(0) for A in As]),
                                                          _ptrs(col_scales)))
        self._A = list(As)  # borrowed
        self._D = list(col_scales) if col_scales is not None else None  # borrowed alike

    def project_all(self, Bs, Zs=None, Ys=None, Xs=None):
        """Bs[i]: (k_i, n_i) float64 CUDA tensors; outputs are allocated when
        not given (pass False to skip one kind)."""
        import torch
        assert len(Bs) == self.count
        ks = []
        for i, B in enumerate(Bs):
            _check_tensor(B, f"B[{i}]", None, self.ns[i])
            ks.append(B.shape[0])

        def outs(given, shape_fn):
            if given is False:
                return None
            if given is None:
                return [torch.empty(shape_fn(i), dtype=torch.float64, device=Bs[i].device) for i in range(self.count)]
            return list(given)

        Z = outs(Zs, lambda i: (ks[i], self.ns[i]))
        Y = outs(Ys, lambda i: (ks[i], self.ns[i]))
        X = outs(Xs, lambda i: (ks[i], self.ms[i]))
        for ts, name, cols in ((Z, "Z", self.ns), (Y, "Y", self.ns), (X, "X", self.ms)):
            if ts is None:
                continue
            if len(ts) != self.count:
                raise ValueError(f"{name} has {len(ts)} members, expected {self.count}")
            for i, t in enumerate(ts):
                _check_tensor(t, f"{name}[{i}]", ks[i], cols[i], Bs[i].device)

        def arr(ts):
            return (_ptrs(ts), _i64s([t.stride(0) for t in ts])) if ts is not None else (None, None)

        (zp, zl), (yp, yl), (xp, xl) = arr(Z), arr(Y), arr(X)
        _check(lib().rtproj_batch_project_all(self.handle, _ptrs(Bs), _i64s([B.stride(0) for B in Bs]), _i64s(ks),
                                              zp, zl, yp, yl, xp, xl))
        return Z, Y, X

    def status(self):
        """Per-member status codes (waits for the batch's stream)."""
        per = (ctypes.c_int * self.count)()
        lib().rtproj_batch_status(self.handle, per)
        return list(per)

    def set_timing(self, enable: bool):
        _check(lib().rtproj_batch_set_timing(self.handle, 1 if enable else 0))

    def info(self) -> dict:
        inf = _Info()
        _check(lib().rtproj_batch_info(self.handle, ctypes.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in _Info._fields_ if f not in ("t_stage_ms", "stage_calls")}
        d["stage_ms"] = {name: inf.t_stage_ms[i] for i, name in enumerate(STAGES)}
        d["stage_calls"] = {name: inf.stage_calls[i] for i, name in enumerate(STAGES)}
        return d

    def member_tables(self, i: int) -> dict:
        """Host copies of member i's sketch tables (signs, permutations, subset)."""
        import numpy as np
        dims = np.zeros(3, dtype=np.int64)
        _check(lib().rtproj_batch_member_tables(self.handle, i, dims.ctypes.data, None, None, None, None))
        np_, n1, n2 = (int(v) for v in dims)
        sign = np.empty(np_, dtype=np.int8)
        sigma = np.empty(n1, dtype=np.int32)
        tau = np.empty(n2, dtype=np.int32)
        J = np.empty(self.ls[i], dtype=np.int32)
        _check(lib().rtproj_batch_member_tables(self.handle, i, None, sign.ctypes.data, sigma.ctypes.data,
                                                tau.ctypes.data, J.ctypes.data))
        return dict(np=np_, n1=n1, n2=n2, sign=sign, sigma=sigma, tau=tau, J=J)

    def member_info(self, i: int) -> dict:
        inf = _Info()
        _check(lib().rtproj_batch_member_info(self.handle, i, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _Info._fields_ if f not in ("t_stage_ms", "stage_calls")}
