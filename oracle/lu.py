"""Route D: the definition, by dense complex LU (oracle; test infrastructure).

For each Matsubara matrix A = i w_n I - H_s the potential of Eq. (7) needs
ln|det A| and, for the gradient (the paper differentiates Eq. (7) by
autograd), the diagonal of A^-1.  Both are read off P A = L U:

    ln|det A| = sum_k ln|u_kk|
    A^-1      = U^-1 L^-1 P       (solved here column by column)

Partial pivoting picks the largest |Re|+|Im| in the column, the lowest row on
ties (the LAPACK izamax rule).  Any pivot order gives the same exact result.

`leibniz_det` / `adjugate_diag` are the brute-force definitions for tiny
matrices (permutation sum; cofactor / determinant), used as the independent
pin of the LU for 4x4 matrices.
"""
from __future__ import annotations

import itertools

import numpy as np


def lu_pivoted(A: np.ndarray):
    """Packed P A = L U of a square complex matrix.

    Returns (LU, perm) with L unit lower (below the diagonal of LU), U upper
    (on and above it), and perm[k] = original row placed at position k.
    Raises ZeroDivisionError on an exactly singular column.
    """
    LU = np.array(A, dtype=np.complex128, copy=True)
    n = LU.shape[0]
    perm = np.arange(n)
    for k in range(n):
        col = LU[k:, k]
        mag = np.abs(col.real) + np.abs(col.imag)
        p = k + int(np.argmax(mag))          # first maximum = lowest row
        if mag[p - k] == 0.0:
            raise ZeroDivisionError("singular matrix")
        if p != k:
            LU[[k, p], :] = LU[[p, k], :]
            perm[[k, p]] = perm[[p, k]]
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, perm


def logabsdet_lu(LU: np.ndarray) -> float:
    """sum_k ln|u_kk| (the row swaps only change the sign/phase)."""
    return float(np.sum(np.log(np.abs(np.diag(LU)))))


def inverse_lu(LU: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """A^-1 from the packed factors: solve L Y = P, then U X = Y."""
    n = LU.shape[0]
    Y = np.zeros((n, n), dtype=np.complex128)
    Y[np.arange(n), perm] = 1.0                   # rows of P I
    for k in range(n):                            # forward, unit diagonal
        Y[k] -= LU[k, :k] @ Y[:k]
    X = np.zeros_like(Y)
    for k in range(n - 1, -1, -1):                # backward
        X[k] = (Y[k] - LU[k, k + 1:] @ X[k + 1:]) / LU[k, k]
    return X


def diag_inverse_lu(A: np.ndarray) -> np.ndarray:
    LU, perm = lu_pivoted(A)
    return np.diag(inverse_lu(LU, perm)).copy()


def _perm_sign(p) -> int:
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def leibniz_det(A: np.ndarray) -> complex:
    """det A = sum over permutations of sign * prod A[i, p(i)]."""
    n = A.shape[0]
    tot = 0j
    for p in itertools.permutations(range(n)):
        term = complex(_perm_sign(p))
        for i in range(n):
            term *= A[i, p[i]]
        tot += term
    return tot


def adjugate_diag(A: np.ndarray) -> np.ndarray:
    """(A^-1)_ii = det(A without row i and column i) / det A."""
    n = A.shape[0]
    d = leibniz_det(A)
    out = np.empty(n, dtype=np.complex128)
    for i in range(n):
        keep = [j for j in range(n) if j != i]
        out[i] = leibniz_det(A[np.ix_(keep, keep)]) / d
    return out
