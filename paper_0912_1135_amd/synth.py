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
* The paper's own matrices (Sec. 5): A = U [B ... B] V with the circulant B
  of eq. pert_lap and random permutations U, V (eq. test_mat), the dense
  A~ = A + E F / sqrt(m n) (eq. modified), and explicit sketch matrices G:
  Gaussian, or additive lagged Fibonacci uniform on [-1, 1] (streams 9-12).
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


# ------------------------------------------------- the paper's own test matrices

def circulant_b(m: int, kappa: float) -> np.ndarray:
    """The m x m circulant of eq. pert_lap: 6 + d on the diagonal, -4 on the
    first and 1 on the second cyclic off-diagonals, d = 16 / (kappa - 1),
    so that cond(B) = (16 + d) / d = kappa (its eigenvalues are
    d + (2 - 2 cos theta)^2); m >= 5."""
    d = 16.0 / (kappa - 1.0)
    B = np.zeros((m, m))
    for off, v in ((-2, 1.0), (-1, -4.0), (0, 6.0 + d), (1, -4.0), (2, 1.0)):
        B[np.arange(m), (np.arange(m) + off) % m] = v
    return B


def make_paper_matrix(m: int, n: int, kappa: float, seed: int):
    """A = U [B ... B] V (eq. test_mat) as a dense row-major m x n array, with
    U and V uniformly random permutations and n / m copies of B; returns
    (A, row_perm, col_perm): A[i, j] = Bcat[row_perm[i], col_perm[j]], i.e.
    U has its one in column row_perm[i] of row i and V maps column col_perm[j]
    of [B ... B] to column j."""
    if n % m:
        raise ValueError("n must be a multiple of m")
    rng = rng_for(seed, 9)
    rp = rng.permutation(m)
    cp = rng.permutation(n)
    Bcat = np.tile(circulant_b(m, kappa), (1, n // m))
    return np.ascontiguousarray(Bcat[rp][:, cp]), rp, cp


def make_paper_lowrank(m: int, n: int, kappa: float, seed: int) -> np.ndarray:
    """The dense A~ = A + E F / sqrt(m n) of eq. modified: A from
    make_paper_matrix, E (m x 10) and F (10 x n) i.i.d. N(0, 1)."""
    A, _, _ = make_paper_matrix(m, n, kappa, seed)
    rng = rng_for(seed, 10)
    E = rng.standard_normal((m, 10))
    F = rng.standard_normal((10, n))
    return np.ascontiguousarray(A + (E @ F) / np.sqrt(float(m) * n))


def make_gaussian_sketch(n: int, l: int, seed: int) -> np.ndarray:
    """G (n x l, row-major) with i.i.d. N(0, 1) entries (the sketch of
    eq. testing as the paper's Tables 3 and 4 draw it)."""
    return np.ascontiguousarray(rng_for(seed, 11).standard_normal((n, l)))


def make_lfg_sketch(n: int, l: int, seed: int) -> np.ndarray:
    """G (n x l, row-major) from additive lagged Fibonacci sequences uniform
    on [-1, 1], formed with floating-point additions and subtractions only
    (the sketch of the paper's Tables 1, 2, 5 and 6).  Column j is its own
    sequence u_t = u_{t-24} + u_{t-55} (minus 1 when that reaches 1) on
    [0, 1), started from 55 uniform values of a per-column SplitMix64-seeded
    generator, then 2 u - 1.  Lags 24 and 55 are the classical additive
    pair; 24 values follow from each block of 55, so the recurrence advances
    24 rows at a time across all columns."""
    rng = rng_for(seed, 12)
    table = rng.random((55, l))
    out = np.empty((n + 55, l))
    out[:55] = table
    t = 55
    while t < n + 55:
        h = min(24, n + 55 - t)
        u = out[t - 24:t - 24 + h] + out[t - 55:t - 55 + h]
        u -= (u >= 1.0)
        out[t:t + h] = u
        t += h
    return np.ascontiguousarray(2.0 * out[55:] - 1.0)


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
    # the paper's Table 1 / 2 row m = 400, n = 1e6, l = 404 (eq. test_mat), cond 1e8
    "paper_400x1000000": dict(m=400, n=1000000, l=404, kappa=1e8, k=8, seed=MASTER_SEED + 6),
    "complex_512x32768": dict(m=512, n=32768, l=2048, kappa=1e8, k=16, seed=MASTER_SEED + 7),
}
