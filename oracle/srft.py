"""Oracle for the sketch S = A G (Sec. 4, eq. testing), TEST INFRASTRUCTURE ONLY.

The paper draws G with i.i.d. entries and only cites the randomized
preconditioner it builds on; here G is read as a subsampled randomized
Fourier transform.  For every row a of A (length n):

    1. pad a with zeros to length np = max(4, 2^ceil(log2 n));
    2. multiply entry t by the random sign sign[t];
    3. permute: y[t] = (signed, padded a)[pi(t)],
       pi(t) = sigma[t // n2] * n2 + tau[t % n2]   (np = n1 * n2);
    4. Y = DFT(y), Y[k] = sum_t y[t] exp(-2 pi i t k / np);
    5. pack the real orthonormal spectrum
       w[0] = Y[0]/sqrt(np), w[1] = Y[np/2]/sqrt(np),
       w[2k] = sqrt(2) Re Y[k]/sqrt(np), w[2k+1] = sqrt(2) Im Y[k]/sqrt(np)
       for k = 1 .. np/2 - 1;
    6. keep the l entries w[J] (J sorted), scaled by sqrt(np / l).

Lemma 2.4 makes every later result independent of this choice of G (only
the conditioning of P^{-1} A = cond(V^* G) depends on it).  ``numpy.fft`` is
used as a library primitive for step 4; ``srft_matrix`` spells out the same
map with an explicit cosine/sine matrix for tiny sizes.
"""
from __future__ import annotations

import numpy as np


def _permutation(tab):
    n2 = tab["n2"]
    t = np.arange(tab["np"])
    return tab["sigma"][t // n2].astype(np.int64) * n2 + tab["tau"][t % n2]


def srft_sketch(A: np.ndarray, seed: int, l: int) -> np.ndarray:
    """S (m x l, float64) for the row-major A (m x n)."""
    from . import srft_tables

    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    tab = srft_tables(seed, n, l)
    npad = tab["np"]
    x = np.zeros((m, npad))
    x[:, :n] = A
    x *= tab["sign"][None, :].astype(np.float64)
    y = x[:, _permutation(tab)]
    Y = np.fft.fft(y, axis=1)
    w = np.empty((m, npad))
    w[:, 0] = Y[:, 0].real
    w[:, 1] = Y[:, npad // 2].real
    half = npad // 2
    w[:, 2::2] = np.sqrt(2.0) * Y[:, 1:half].real
    w[:, 3::2] = np.sqrt(2.0) * Y[:, 1:half].imag
    w /= np.sqrt(npad)
    return w[:, tab["J"]] * np.sqrt(npad / l)


def srft_matrix(n: int, seed: int, l: int) -> np.ndarray:
    """The n x l matrix G itself, built entry by entry from cosines and sines
    (no FFT).  Only for tiny n."""
    from . import srft_tables

    tab = srft_tables(seed, n, l)
    npad = tab["np"]
    pi = _permutation(tab)
    # y = Pi D pad(a): y[t] = sign[pi(t)] a[pi(t)]; so entry (src, t) of the
    # matrix taking a to y is sign[src] when src = pi(t) < n.
    G = np.zeros((n, l))
    for q, j in enumerate(tab["J"]):
        for t in range(npad):
            src = pi[t]
            if src >= n:
                continue
            if j == 0:
                c = 1.0
            elif j == 1:
                c = np.cos(np.pi * t)  # exp(-i pi t) = (-1)^t
            else:
                k = j // 2
                ang = 2.0 * np.pi * ((t * k) % npad) / npad
                c = np.sqrt(2.0) * (np.cos(ang) if j % 2 == 0 else -np.sin(ang))
            G[src, q] += tab["sign"][src] * c / np.sqrt(npad) * np.sqrt(npad / l)
    return G
