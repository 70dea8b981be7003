"""Exact projections for the paper's structured test matrix (TEST
INFRASTRUCTURE ONLY).

For A = U [B ... B] V (eq. test_mat) with B invertible and U, V
permutations, the rows of [B ... B] span exactly the vectors made of n / m
copies of one m-vector.  With A[i, j] = [B ... B][rp[i], cp[j]], the row
space of A is {w : w[j] depends only on cp[j] mod m}, so the orthogonal
projection of b onto it averages b over each class {j : cp[j] mod m = c}
(n / m entries each):
    p[j] = mean of b over the class of j,   z = b - p,
for every cond(A): the truth for the paper's Tables 1 to 4 at any kappa.
"""
from __future__ import annotations

import numpy as np


def block_average_projection(m: int, col_perm: np.ndarray, B: np.ndarray):
    """(Z, P) for the columns of B (n x k, or n), col_perm as returned by
    synth.make_paper_matrix."""
    cls = np.asarray(col_perm) % m
    vec = B.ndim == 1
    Bc = B.reshape(B.shape[0], -1)
    sums = np.zeros((m, Bc.shape[1]))
    np.add.at(sums, cls, Bc)
    counts = np.bincount(cls, minlength=m)[:, None]
    P = (sums / counts)[cls]
    Z = Bc - P
    if vec:
        return Z[:, 0], P[:, 0]
    return Z, P
