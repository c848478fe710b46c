"""Exact rational arithmetic helpers for pinning the oracle on tiny inputs.

Every binary64 number is a dyadic rational, so ``fractions.Fraction`` holds
inputs and all sums/products exactly.  These helpers never round.
"""
from fractions import Fraction

import numpy as np


def F(x) -> Fraction:
    return Fraction(float(x))


def gram_exact(A, B=None):
    """Exact A^T B as a nested list of Fractions."""
    A = np.asarray(A, dtype=np.float64)
    B = A if B is None else np.asarray(B, dtype=np.float64)
    m, ka = A.shape
    kb = B.shape[1]
    Af = [[F(A[r, i]) for i in range(ka)] for r in range(m)]
    Bf = Af if B is A else [[F(B[r, j]) for j in range(kb)] for r in range(m)]
    return [[sum((Af[r][i] * Bf[r][j] for r in range(m)), Fraction(0))
             for j in range(kb)] for i in range(ka)]


def ldlt_exact(G):
    """Exact LDL^T of a symmetric positive definite rational matrix.

    Returns (L unit lower, D list).  Then the Cholesky factor R (upper) of
    G = R^T R satisfies R_jj^2 = D_j and R_ji / R_jj = L_ij exactly."""
    k = len(G)
    L = [[Fraction(int(i == j)) for j in range(k)] for i in range(k)]
    D = [Fraction(0)] * k
    for j in range(k):
        D[j] = G[j][j] - sum((L[j][p] ** 2 * D[p] for p in range(j)), Fraction(0))
        for i in range(j + 1, k):
            L[i][j] = (G[i][j] - sum((L[i][p] * L[j][p] * D[p] for p in range(j)),
                                     Fraction(0))) / D[j]
    return L, D


def dd_value(hi, lo=None) -> Fraction:
    v = F(hi)
    if lo is not None:
        v += F(lo)
    return v
