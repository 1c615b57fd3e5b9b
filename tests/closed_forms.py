"""Closed forms used to pin the oracle, derived here from the mathematics.

Nothing in this file is copied from the oracle: the finite-difference weights
are obtained by solving the moment equations exactly in rational arithmetic,
and the Fourier symbols follow from applying those weights to a complex
exponential.
"""
import math
from fractions import Fraction

import numpy as np


def solve_exact(A, b):
    """Gaussian elimination over the rationals."""
    n = len(A)
    M = [list(map(Fraction, row)) + [Fraction(bb)] for row, bb in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                fac = M[r][col] / M[col][col]
                M[r] = [x - fac * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def central_weights(deriv, r):
    """Weights c_m, m = -r..r with sum_m c_m m^k = k! [k == deriv] for
    k = 0..2r (exact rationals)."""
    offs = list(range(-r, r + 1))
    A = [[Fraction(m) ** k for m in offs] for k in range(2 * r + 1)]
    b = [Fraction(math.factorial(deriv)) if k == deriv else Fraction(0)
         for k in range(2 * r + 1)]
    return solve_exact(A, b)


def moments(c, kmax):
    r = (len(c) - 1) // 2
    return [sum(Fraction(cm) * Fraction(m) ** k for cm, m in zip(c, range(-r, r + 1)))
            for k in range(kmax + 1)]


W1 = [float(v) for v in central_weights(1, 3)]
W2 = [float(v) for v in central_weights(2, 3)]


def kappa(k, n):
    """First-derivative symbol: D1 exp(i k x) = i kappa exp(i k x) on a
    periodic grid of n points over [0, 2 pi)."""
    ds = 2 * math.pi / n
    th = k * ds
    return sum(W1[m + 3] * math.sin(m * th) for m in range(-3, 4)) / ds


def lam(k, n):
    """Second-derivative symbol: D2 exp(i k x) = lam exp(i k x)."""
    ds = 2 * math.pi / n
    th = k * ds
    return sum(W2[m + 3] * math.cos(m * th) for m in range(-3, 4)) / ds ** 2


def coords(n):
    """Broadcastable [x, y, z] coordinate arrays 2 pi i / n (NumPy order)."""
    nd = len(n)
    out = []
    for a in range(nd):
        c = 2 * math.pi * np.arange(n[a]) / n[a]
        s = [1] * nd
        s[nd - 1 - a] = n[a]
        out.append(c.reshape(s))
    return out


def full(n, v):
    return np.broadcast_to(v, tuple(reversed(n))).astype(np.float64).copy()


def rk3_stability(z):
    """Amplification factor of any 3-stage third-order explicit RK method on
    y' = lambda y with z = dt lambda."""
    return 1 + z + z * z / 2 + z ** 3 / 6


def laplacian_star_exact(ndim, r):
    """Star Laplacian (grid units) from the exact rational weights."""
    c = [float(v) for v in central_weights(2, r)]
    g = np.zeros((2 * r + 1,) * ndim)
    for a in range(ndim):
        idx = [r] * ndim
        for m in range(-r, r + 1):
            idx[a] = r + m
            g[tuple(idx)] += c[m + r]
    return g


def diffusion_star_exact(ndim, r, s):
    g = s * laplacian_star_exact(ndim, r)
    g[(r,) * ndim] += 1.0
    return g


def laplacian_symbol_grid(k, n, r):
    """Symbol of the 1-D (2r)-th order second difference in grid units on the
    mode exp(2 pi i k x / n)."""
    c = [float(v) for v in central_weights(2, r)]
    th = 2 * math.pi * k / n
    return sum(c[m + r] * math.cos(m * th) for m in range(-r, r + 1))
