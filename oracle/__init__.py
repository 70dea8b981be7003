"""CPU oracle for the randomized orthogonal projection (Rokhlin & Tygert).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the GPU library.

* ``project``      -- x = argmin |A^T x - b|, p = A^T x, z = b - p for every
                      column b (Sec. 1 items 1-3, Remark 4.1, eq.
                      basic_identity); Householder QR of A^T plus binary128
                      refinement (Remark 4.3).  Written in C (``oracle.c``).
* ``project_lapack`` -- the same outputs with the Householder QR of A^T
                      taken from LAPACK (numpy.linalg.qr, R only, as a
                      library step), x started at 0 and refined by the same
                      binary128 iteration; for sizes where the unblocked
                      factorization of ``project`` takes minutes.
* ``qrcp``         -- Businger-Golub column-pivoted Householder QR
                      (Sec. 4, eq. QR_decomp).
* ``srft_tables``  -- SplitMix64 draws of the sketch's random tables.
* ``srft_sketch``  -- S = A G for the subsampled randomized Fourier sketch
                      (in ``srft.py``; the sketch of Sec. 4, eq. testing,
                      with G read as an SRFT instead of i.i.d. entries).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (-O2, OpenMP) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def bind(path: str):
    """Load a compiled oracle library from `path` and declare its C signatures."""
    lib = ctypes.CDLL(path)
    i64, u64, dp, ip = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    lib.orc_splitmix64_stream.argtypes = [u64, i64, dp]
    lib.orc_instance_seed.argtypes = [u64, i64]
    lib.orc_instance_seed.restype = u64
    lib.orc_srft_dims.argtypes = [i64, dp, dp, dp]
    lib.orc_srft_tables.argtypes = [u64, i64, i64, dp, dp, dp, dp]
    lib.orc_srft_tables.restype = ip
    lib.orc_qrcp.argtypes = [i64, i64, dp, i64, dp, dp]
    lib.orc_qrcp.restype = ip
    lib.orc_project.argtypes = [i64, i64, dp, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, ip, dp]
    lib.orc_project.restype = ip
    lib.orc_project_r.argtypes = [i64, i64, dp, i64, dp, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, ip, dp]
    lib.orc_project_r.restype = ip
    lib.orc_project_complex_r.argtypes = [i64, i64, dp, i64, dp, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, ip,
                                          dp]
    lib.orc_project_complex_r.restype = ip
    lib.orc_num_threads.restype = ip
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = bind(_LIB_PATH)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().orc_splitmix64_stream(seed, count, _ptr(out))
    return out


def instance_seed(seed: int, i: int) -> int:
    return int(_load().orc_instance_seed(seed, i))


def srft_dims(n: int):
    vals = [ctypes.c_int64() for _ in range(3)]
    _load().orc_srft_dims(n, *[ctypes.byref(v) for v in vals])
    return tuple(v.value for v in vals)


def srft_tables(seed: int, n: int, l: int):
    """Signs (np), sigma (n1), tau (n2) and the sorted subset J (l)."""
    np_, n1, n2 = srft_dims(n)
    sign = np.empty(np_, dtype=np.int8)
    sigma = np.empty(n1, dtype=np.int32)
    tau = np.empty(n2, dtype=np.int32)
    J = np.empty(l, dtype=np.int32)
    rc = _load().orc_srft_tables(seed, n, l, _ptr(sign), _ptr(sigma), _ptr(tau), _ptr(J))
    if rc != 0:
        raise ValueError(f"orc_srft_tables failed ({rc}) for n={n}, l={l}")
    return dict(np=np_, n1=n1, n2=n2, sign=sign, sigma=sigma, tau=tau, J=J)


def qrcp(M: np.ndarray, lib=None):
    """Column-pivoted QR of M (rows x cols, rows >= cols): M[:, piv] = Q R.

    Returns (R, piv) with R upper triangular (cols x cols)."""
    M = np.asarray(M, dtype=np.float64)
    rows, cols = M.shape
    work = np.asfortranarray(M.copy())
    R = np.zeros((cols, cols), dtype=np.float64)
    piv = np.empty(cols, dtype=np.int32)
    rc = (lib or _load()).orc_qrcp(rows, cols, _ptr(work), rows, _ptr(R), _ptr(piv))
    if rc != 0:
        raise ValueError(f"orc_qrcp failed ({rc})")
    return R, piv


def project(A: np.ndarray, B: np.ndarray, maxit: int = 8, lib=None):
    """Return (Z, P, X, info) for every column of B.

    A: (m, n) float64, full row rank.  B: (n,) or (n, k).  Z = B - A^T X,
    P = A^T X, X = argmin |A^T X - B| column by column."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    vec = B.ndim == 1
    Bc = np.asfortranarray(B.reshape(n, -1), dtype=np.float64)
    k = Bc.shape[1]
    Z = np.zeros((n, k), order="F")
    P = np.zeros((n, k), order="F")
    X = np.zeros((m, k), order="F")
    info = np.zeros(2)
    rc = (lib or _load()).orc_project(m, n, _ptr(A), n, k, _ptr(Bc), n, _ptr(Z), n, _ptr(P), n,
                             _ptr(X), m, maxit, _ptr(info))
    if rc != 0:
        raise ValueError(f"orc_project failed ({rc})")
    if vec:
        return Z[:, 0], P[:, 0], X[:, 0], info
    return Z, P, X, info


def project_lapack(A: np.ndarray, B: np.ndarray, maxit: int = 12, lib=None):
    """As ``project``, with R from LAPACK's Householder QR of A^T.

    The semi-normal solve x1 = R^{-1} R^{-T} A b (the first refinement step
    from x = 0) is refined in binary128 exactly as in ``project``, so both
    routes converge to the same x, p and z (to the final rounding)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    R = np.ascontiguousarray(np.linalg.qr(A.T, mode="r")[:m, :m])
    vec = B.ndim == 1
    Bc = np.asfortranarray(B.reshape(n, -1), dtype=np.float64)
    k = Bc.shape[1]
    Z = np.zeros((n, k), order="F")
    P = np.zeros((n, k), order="F")
    X = np.zeros((m, k), order="F")
    info = np.zeros(2)
    rc = (lib or _load()).orc_project_r(m, n, _ptr(A), n, _ptr(R), m, k, _ptr(Bc), n, _ptr(Z), n, _ptr(P), n,
                                        _ptr(X), m, maxit, _ptr(info))
    if rc != 0:
        raise ValueError(f"orc_project_r failed ({rc})")
    if vec:
        return Z[:, 0], P[:, 0], X[:, 0], info
    return Z, P, X, info


def num_threads() -> int:
    return int(_load().orc_num_threads())


from .srft import srft_sketch, srft_matrix  # noqa: E402,F401
