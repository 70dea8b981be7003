"""Complex-valued oracle (TEST INFRASTRUCTURE ONLY; imported by tests/ and
bench.py's CPU leg, never by the product).

The paper treats real matrices and states that the method and its analysis
carry over to complex entries unchanged (Sec. 1, end).  For a complex m x n
A of full row rank and a right-hand side b (length n), with A^* the
conjugate transpose:
    x = argmin |A^* x - b| = (A A^*)^{-1} A b,   p = A^* x,   z = b - p.
Written in complex arithmetic throughout (no real embedding):
  1. R from LAPACK's Householder QR of A^* (numpy.linalg.qr with complex
     reflectors; a library step), so that R^* R = A A^* up to rounding;
  2. x = 0, then the refinement of Remark 4.3 with r = b - A^* x and
     s = A r in binary128 complex arithmetic, the correction
     d = R^{-1} R^{-*} s in complex binary64, x += d kept in binary128
     (``orc_project_complex_r`` in oracle.c);
  3. p = A^* x and z = b - p in binary128, rounded once.
"""
from __future__ import annotations

import numpy as np


def project_complex(A: np.ndarray, B: np.ndarray, maxit: int = 12, lib=None):
    """Return (Z, P, X, info) for every column of B (complex n x k, or n).

    info = (refinement steps, last |d| / |x|, maximum over columns)."""
    from . import _load, _ptr
    A = np.ascontiguousarray(A, dtype=np.complex128)
    m, n = A.shape
    vec = B.ndim == 1
    Bc = np.asfortranarray(np.asarray(B, dtype=np.complex128).reshape(n, -1))
    k = Bc.shape[1]
    R = np.ascontiguousarray(np.linalg.qr(A.conj().T, mode="r")[:m, :m])
    Z = np.zeros((n, k), dtype=np.complex128, order="F")
    P = np.zeros((n, k), dtype=np.complex128, order="F")
    X = np.zeros((m, k), dtype=np.complex128, order="F")
    info = np.zeros(2)
    rc = (lib or _load()).orc_project_complex_r(m, n, _ptr(A), n, _ptr(R), m, k, _ptr(Bc), n, _ptr(Z), n, _ptr(P),
                                                n, _ptr(X), m, maxit, _ptr(info))
    if rc != 0:
        raise ValueError(f"orc_project_complex_r failed ({rc})")
    if vec:
        return Z[:, 0], P[:, 0], X[:, 0], info
    return Z, P, X, info
