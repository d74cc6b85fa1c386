"""Closed forms that pin the oracle from outside its own code.

For a linear system x' = A x + b with constant b, one classical RK4 step of
size h is exactly

    x+ = R(hA) x + h S(hA) b,
    R(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24      (the RK4 stability polynomial)
    S(Z) = I + Z/2 + Z^2/6 + Z^3/24            (R(Z) = I + Z S(Z))

whatever the stage bookkeeping.  Evaluated here in exact rational arithmetic
(``fractions.Fraction``), so a wrong stage coefficient, a dropped factor h or
a wrong neighbour in the oracle shows up as a mismatch far above FP64
rounding.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _F(x):
    return Fraction(x) if not isinstance(x, Fraction) else x


def mat(n, fill=0):
    return [[_F(fill) for _ in range(n)] for _ in range(n)]


def eye(n):
    m = mat(n)
    for i in range(n):
        m[i][i] = Fraction(1)
    return m


def matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), Fraction(0)) for j in range(m)]
            for i in range(n)]


def matvec(A, x):
    return [sum((A[i][j] * x[j] for j in range(len(x))), Fraction(0)) for i in range(len(A))]


def add(A, B, s=Fraction(1)):
    return [[A[i][j] + s * B[i][j] for j in range(len(A[0]))] for i in range(len(A))]


def scale(A, s):
    return [[s * a for a in row] for row in A]


def rk4_polys(Z):
    n = len(Z)
    I = eye(n)
    Z2 = matmul(Z, Z)
    Z3 = matmul(Z2, Z)
    Z4 = matmul(Z3, Z)
    R = add(add(add(add(I, Z), Z2, Fraction(1, 2)), Z3, Fraction(1, 6)), Z4, Fraction(1, 24))
    S = add(add(add(I, Z, Fraction(1, 2)), Z2, Fraction(1, 6)), Z3, Fraction(1, 24))
    return R, S


def rk4_linear_exact(A, b, x0, h, N):
    """N exact RK4 steps of x' = A x + b (all arguments converted to Fraction)."""
    h = _F(h)
    A = [[_F(a) for a in row] for row in A]
    b = [_F(v) for v in b]
    x = [_F(v) for v in x0]
    R, S = rk4_polys(scale(A, h))
    hSb = [h * v for v in matvec(S, b)]
    for _ in range(N):
        Rx = matvec(R, x)
        x = [Rx[i] + hSb[i] for i in range(len(x))]
    return x


def tridiag(n, aL, aD, aR):
    """Chain matrix with zero (Dirichlet) ghosts."""
    A = mat(n)
    for i in range(n):
        A[i][i] = _F(aD)
        if i > 0:
            A[i][i - 1] = _F(aL)
        if i < n - 1:
            A[i][i + 1] = _F(aR)
    return A


def embedding_matrix(n, aL, aD, aR):
    """The 2n linear embedding of a LIN3 chain: [[M, N], [N, M]], where M holds
    the diagonal and the nonnegative off-diagonals and N the negative ones."""
    pos = lambda a: _F(a) if a > 0 else Fraction(0)
    neg = lambda a: _F(a) if a < 0 else Fraction(0)
    M = tridiag(n, pos(aL), aD, pos(aR))
    N = tridiag(n, neg(aL), 0, neg(aR))
    big = mat(2 * n)
    for i in range(n):
        for j in range(n):
            big[i][j] = M[i][j]
            big[i][n + j] = N[i][j]
            big[n + i][j] = N[i][j]
            big[n + i][n + j] = M[i][j]
    return big


def to_float(v):
    return np.array([float(x) for x in v], dtype=np.float64)


def rk4_stability(z: float) -> float:
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def bernoulli_rd1(x0: float, t: float) -> float:
    """Exact solution of x' = -2x - x^3 (the one-cell RD chain, h = 1, u = 0).

    With y = x^-2 the equation is linear, y' = 4y + 2, which integrates to
    x(t) = x0 e^{-2t} / sqrt(1 + x0^2 (1 - e^{-4t}) / 2).
    """
    e2 = np.exp(-2.0 * t)
    return x0 * e2 / np.sqrt(1.0 + x0 * x0 * (1.0 - e2 * e2) / 2.0)
