"""Exact quadrature weights by moment matching (test-side reference).

The weights of an interpolatory rule on n nodes are the unique weights that
integrate x^k exactly for k < n; they solve a Vandermonde system, solved here in
exact rational arithmetic or with 60-digit mpmath.
"""
from fractions import Fraction

import mpmath
import numpy as np

mpmath.mp.dps = 60

def moment_weights(nodes, a, b):
    """Weights w_j with sum_j w_j x_j^k = int_a^b x^k dx, k < n (exact)."""
    n = len(nodes)
    exact = isinstance(nodes[0], Fraction)
    if exact:
        A = [[x**k for x in nodes] + [(b**(k + 1) - a**(k + 1)) / (k + 1)] for k in range(n)]
        for c in range(n):  # Gauss-Jordan in Fractions
            piv = next(r for r in range(c, n) if A[r][c] != 0)
            A[c], A[piv] = A[piv], A[c]
            for r in range(n):
                if r != c and A[r][c] != 0:
                    f = A[r][c] / A[c][c]
                    A[r] = [x - f * y for x, y in zip(A[r], A[c])]
        return [A[j][n] / A[j][j] for j in range(n)]
    V = mpmath.matrix([[x**k for x in nodes] for k in range(n)])
    rhs = mpmath.matrix([(b**(k + 1) - a**(k + 1)) / (k + 1) for k in range(n)])
    return list(mpmath.lu_solve(V, rhs))


def std_nodes(M, family):
    if family == oracle_EQUI:
        return [Fraction(m, M) for m in range(1, M + 1)]
    if M == 2:
        return [Fraction(0), Fraction(1)]
    if M == 3:
        return [Fraction(0), Fraction(1, 2), Fraction(1)]
    r = {4: 1 / mpmath.sqrt(5), 5: mpmath.sqrt(mpmath.mpf(3) / 7)}[M]
    if M == 4:
        return [mpmath.mpf(0), (1 - r) / 2, (1 + r) / 2, mpmath.mpf(1)]
    return [mpmath.mpf(0), (1 - r) / 2, mpmath.mpf(1) / 2, (1 + r) / 2, mpmath.mpf(1)]


oracle_LOB, oracle_EQUI = 0, 1


def reference(M, family, P, dt):
    x = std_nodes(M, family)
    exact = isinstance(x[0], Fraction)
    zero = Fraction(0) if exact else mpmath.mpf(0)
    xs = [zero] + x
    emb = [Fraction(q, P) for q in range(1, P + 1)]
    s = np.zeros((M + 1, M + 1))
    shat = np.zeros((M + 1, P + 1))
    stil = np.zeros((M + 1, P + 1, M + 1))
    spq = np.zeros((M + 1, P + 1, P + 1))
    for m in range(1, M + 1):
        lo, hi = xs[m - 1], xs[m]
        if hi == lo:
            continue
        ln = hi - lo
        w = moment_weights(x, lo, hi)
        s[m, 1:] = [float(v * dt) for v in w]
        for p in range(1, P + 1):
            w = moment_weights(x, lo + ln * (p - 1) / P, lo + ln * p / P)
            stil[m, p, 1:] = [float(v * dt) for v in w]
        we = moment_weights(emb, Fraction(0), Fraction(1))
        shat[m, 1:] = [float(v * ln * dt) for v in we]
        for p in range(1, P + 1):
            we = moment_weights(emb, Fraction(p - 1, P), Fraction(p, P))
            spq[m, p, 1:] = [float(v * ln * dt) for v in we]
    tau = np.array([float(v * dt) for v in xs])
    return tau, s, shat, stil, spq


