"""Seeded synthetic workloads for the randomized orthogonal projection.

Input generation only: nothing here computes any step of the method.  The
same generators feed the GPU path, the CPU oracle, the tests and the
benchmark.

* A = U diag(sigma) V^T with U (m x m) and V (n x m) Haar-distributed
  orthonormal, sigma log-spaced from 1 down to 1/kappa.  U, and V when n <
  8m, is the QR of a Gaussian matrix with its columns multiplied by the
  signs of R's diagonal (Mezzadri).  For n >= 8m, V is the orthonormal polar
  factor G (G^T G)^{-1/2} of an n x m Gaussian G: for any orthogonal Q, QG
  has the law of G and its polar factor is Q times that of G, so the law of
  V is invariant under rotations, i.e. Haar.  G is then well conditioned
  (cond <= (1 + sqrt(m/n)) / (1 - sqrt(m/n)) < 2.1 up to fluctuations), so
  the polar factor formed from G^T G is orthonormal to a few units of
  rounding, at a tenth of the cost of a QR of G (262144 x 2048: 15 s
  against 110 s on 8 cores).
* Right-hand sides: i.i.d. N(0, 1), stored as a (k, n) C-contiguous array,
  i.e. column-major n x k (column c is row c of the array).
* Complex problems: the same construction with unitary factors and complex
  Gaussian right-hand sides (streams 6, 7, 8).
* Batched workload: instance sizes m_i ~ U{32..512}, n_i = m_i * U{16..64},
  l_i = 4 m_i, k_i ~ U{1..64}.
* Interior-point-shaped sequence: diagonal scalings D_t with entries
  10^U(-6, 6), redrawn for every step t.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 20091210


def rng_for(seed: int, stream: int) -> np.random.Generator:
    """Independent generator number `stream` of master seed `seed`."""
    return np.random.default_rng(np.random.SeedSequence(seed).spawn(stream + 1)[stream])


def haar(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    """rows x cols matrix with Haar-distributed orthonormal columns."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def haar_tall(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    """rows x cols Haar orthonormal columns; the polar factor of a Gaussian
    matrix when rows >= 8 cols, else ``haar``."""
    if rows < 8 * cols:
        return haar(rows, cols, rng)
    g = rng.standard_normal((rows, cols))
    lam, w = np.linalg.eigh(g.T @ g)
    return g @ ((w / np.sqrt(lam)[None, :]) @ w.T)


def log_spaced(m: int, kappa: float) -> np.ndarray:
    if m == 1:
        return np.ones(1)
    return 10.0 ** (-np.log10(kappa) * np.arange(m) / (m - 1))


def make_problem(m: int, n: int, kappa: float, seed: int, with_factors: bool = False):
    """A (m x n, row-major float64) with singular values log-spaced 1 -> 1/kappa."""
    U = haar(m, m, rng_for(seed, 0))
    V = haar_tall(n, m, rng_for(seed, 1))
    s = log_spaced(m, kappa)
    A = np.ascontiguousarray((U * s[None, :]) @ V.T)
    if with_factors:
        return A, U, s, V
    return A


def make_complex_problem(m: int, n: int, kappa: float, seed: int) -> np.ndarray:
    """Complex A = U diag(sigma) V^* (m x n, row-major complex128): U and V
    with orthonormal columns from the QR of complex Gaussian matrices (the
    unitary analogue of Mezzadri's construction, columns multiplied by the
    phases of R's diagonal), sigma log-spaced 1 -> 1/kappa."""
    def unitary(rows, cols, rng):
        g = rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))
        q, r = np.linalg.qr(g)
        d = np.diag(r)
        ph = np.where(np.abs(d) > 0, d / np.abs(d), 1.0)
        return q * ph[None, :]
    U = unitary(m, m, rng_for(seed, 6))
    V = unitary(n, m, rng_for(seed, 7))
    s = log_spaced(m, kappa)
    return np.ascontiguousarray((U * s[None, :]) @ V.conj().T)


def make_complex_rhs(n: int, k: int, seed: int) -> np.ndarray:
    """k complex Gaussian right-hand sides as a (k, n) complex128 array."""
    g = rng_for(seed, 8).standard_normal((2, k, n))
    return np.ascontiguousarray(g[0] + 1j * g[1])


def make_rhs(n: int, k: int, seed: int) -> np.ndarray:
    """k Gaussian right-hand sides as a (k, n) array (column-major n x k)."""
    return np.ascontiguousarray(rng_for(seed, 2).standard_normal((k, n)))


def make_scalings(n: int, steps: int, seed: int) -> np.ndarray:
    """steps x n diagonal scalings with entries 10^U(-6, 6)."""
    return 10.0 ** rng_for(seed, 3).uniform(-6.0, 6.0, size=(steps, n))


@dataclass
class BatchShape:
    m: list = field(default_factory=list)
    n: list = field(default_factory=list)
    l: list = field(default_factory=list)
    k: list = field(default_factory=list)


def make_batch_shapes(count: int, seed: int, m_lo: int = 32, m_hi: int = 512,
                      j_lo: int = 16, j_hi: int = 64, k_lo: int = 1, k_hi: int = 64) -> BatchShape:
    rng = rng_for(seed, 4)
    m = rng.integers(m_lo, m_hi + 1, size=count)
    j = rng.integers(j_lo, j_hi + 1, size=count)
    k = rng.integers(k_lo, k_hi + 1, size=count)
    return BatchShape(m=[int(v) for v in m], n=[int(a * b) for a, b in zip(m, j)],
                      l=[int(4 * v) for v in m], k=[int(v) for v in k])


# The five measured workloads (sizes, spectra, sketch size, right-hand sides).
CONFIGS = {
    "plain_64x4096": dict(m=64, n=4096, l=256, kappa=1e6, k=1, seed=MASTER_SEED + 1),
    "plain_512x65536": dict(m=512, n=65536, l=2048, kappa=1e10, k=16, seed=MASTER_SEED + 2),
    "mixed_2048x262144": dict(m=2048, n=262144, l=8192, kappa=1e8, k=64, seed=MASTER_SEED + 3),
    "batch_256": dict(count=256, kappa=1e6, seed=MASTER_SEED + 4),
    "ipm_1024x131072": dict(m=1024, n=131072, l=4096, kappa=1e4, k=128, steps=32, seed=MASTER_SEED + 5),
}
