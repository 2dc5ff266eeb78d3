"""Exact rational arithmetic for tiny systems (n <= 8).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Gaussian elimination with partial pivoting (Sec. 2 of arXiv 1511.07174, the
first step of the direct method) carried out in ``fractions.Fraction``: every
pivot comparison and every update is exact, so the pivots and the factors are
the mathematically exact ones.  The determinant is also computed by the
Leibniz permutation sum, which shares nothing with elimination; that is the
brute-force cross-check for n <= 7.
"""
from __future__ import annotations

import itertools
from fractions import Fraction


def to_fractions(A):
    return [[Fraction(x) for x in row] for row in A]


def gepp(A):
    """Exact GEPP.  Returns (L, U, ipiv, info) with ipiv 1-based sequential interchanges,
    ties broken to the lowest row index, and info = first zero pivot (1-based) or 0."""
    M = to_fractions(A)
    n = len(M)
    ipiv = []
    info = 0
    for k in range(n):
        mu = k
        for i in range(k + 1, n):
            if abs(M[i][k]) > abs(M[mu][k]):
                mu = i
        ipiv.append(mu + 1)
        M[k], M[mu] = M[mu], M[k]
        if M[k][k] != 0:
            for i in range(k + 1, n):
                M[i][k] = M[i][k] / M[k][k]
                for j in range(k + 1, n):
                    M[i][j] -= M[i][k] * M[k][j]
        elif info == 0:
            info = k + 1
    L = [[(M[i][j] if j < i else (Fraction(1) if i == j else Fraction(0))) for j in range(n)] for i in range(n)]
    U = [[(M[i][j] if j >= i else Fraction(0)) for j in range(n)] for i in range(n)]
    return L, U, ipiv, info


def solve(A, b):
    """Exact x with A x = b (A nonsingular), by exact GEPP and substitution."""
    L, U, ipiv, info = gepp(A)
    if info:
        raise ZeroDivisionError("singular")
    n = len(L)
    y = [Fraction(v) for v in b]
    for k in range(n):
        p = ipiv[k] - 1
        y[k], y[p] = y[p], y[k]
    for i in range(n):
        y[i] -= sum(L[i][j] * y[j] for j in range(i))
    x = [Fraction(0)] * n
    for i in reversed(range(n)):
        x[i] = (y[i] - sum(U[i][j] * x[j] for j in range(i + 1, n))) / U[i][i]
    return x


def det_leibniz(A):
    """det(A) = sum over permutations of sign * prod a_{i, s(i)}; exact, O(n! n)."""
    M = to_fractions(A)
    n = len(M)
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = Fraction(1)
        for i in range(n):
            prod *= M[i][perm[i]]
            if prod == 0:
                break
        total += -prod if inv % 2 else prod
    return total


def residual(A, x, b):
    """Exact b - A x for float inputs (each float is an exact rational)."""
    n = len(b)
    return [Fraction(b[i]) - sum(Fraction(A[i][j]) * Fraction(x[j]) for j in range(n)) for i in range(n)]
