"""Averaging kernels K in K^{p,q} and K0 in K_0^{p,q} (Definition 2.3, Section 2.3).

The paper defines only the kernel classes: compact support, q continuous
derivatives, a (q+1)-th derivative of bounded variation and p vanishing
moments.  Reading (paper silent on the construction): take

    K(x)  = (1 - x^2)^(q+1) * sum_{i<=p} c_i x^i      on [-1, 1]
    K0(t) = t^(q+1) (1 - t)^(q+1) * sum_{i<=p} d_i t^i on [0, 1]

and zero outside.  The factors vanish to order q+1 at the support ends, so the
functions are C^q with a jump in the (q+1)-th derivative, and the p+1
coefficients are fixed by the moment conditions int K x^r = delta_{r0},
r = 0..p, solved here in exact rational arithmetic.  K0 vanishes for t <= 0 as
the class K_0 requires.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import numpy as np


def _solve_exact(A, b):
    """Gaussian elimination over the rationals."""
    n = len(b)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [M[r][k] - f * M[col][k] for k in range(n + 1)]
    return [M[i][n] / M[i][i] for i in range(n)]


def _moment_sym(q, m):
    """int_{-1}^{1} (1-x^2)^(q+1) x^m dx, exact."""
    if m % 2:
        return Fraction(0)
    n = q + 1
    return sum(Fraction(comb(n, k) * (-1) ** k * 2, 2 * k + m + 1) for k in range(n + 1))


def _moment_one_sided(q, m):
    """int_0^1 t^(q+1+m) (1-t)^(q+1) dt = a! b! / (a+b+1)!, exact."""
    a, b = q + 1 + m, q + 1
    return Fraction(factorial(a) * factorial(b), factorial(a + b + 1))


@lru_cache(maxsize=None)
def space_coeffs(p, q):
    """Exact c_0..c_p of K in K^{p,q}."""
    A = [[_moment_sym(q, r + i) for i in range(p + 1)] for r in range(p + 1)]
    b = [Fraction(1 if r == 0 else 0) for r in range(p + 1)]
    return tuple(_solve_exact(A, b))


@lru_cache(maxsize=None)
def time_coeffs(p, q):
    """Exact d_0..d_p of K0 in K_0^{p,q}."""
    A = [[_moment_one_sided(q, r + i) for i in range(p + 1)] for r in range(p + 1)]
    b = [Fraction(1 if r == 0 else 0) for r in range(p + 1)]
    return tuple(_solve_exact(A, b))


def K(x, p, q):
    """Space kernel K(x), zero outside (-1, 1)."""
    x = np.asarray(x, dtype=np.float64)
    c = [float(v) for v in space_coeffs(p, q)]
    poly = np.zeros_like(x)
    for i, ci in enumerate(c):
        poly = poly + ci * x ** i
    val = (1.0 - x * x) ** (q + 1) * poly
    return np.where(np.abs(x) < 1.0, val, 0.0)


def K0(t, p, q):
    """Time kernel K0(t), zero outside (0, 1)."""
    t = np.asarray(t, dtype=np.float64)
    d = [float(v) for v in time_coeffs(p, q)]
    poly = np.zeros_like(t)
    for i, di in enumerate(d):
        poly = poly + di * t ** i
    val = t ** (q + 1) * (1.0 - t) ** (q + 1) * poly
    return np.where((t > 0.0) & (t < 1.0), val, 0.0)


def space_weights(positions, mu, dx, p, q):
    """Quadrature weights of the scaled kernel K_mu(x) = K(x/mu)/mu on one axis.

    Reading (quadrature of eq. (upscaling) is not stated): the rectangle rule on
    the micro grid, w_j = K(xi_j / mu) dx / mu, with no renormalization.
    """
    return K(np.asarray(positions) / mu, p, q) * dx / mu


def time_weights(M, p, q):
    """w^n = K0(n/M) / M for n = 0..M: trapezoid rule for int_0^eta K0_eta(t) Q(t) dt
    on the time-step grid (both end weights are exactly zero)."""
    n = np.arange(M + 1, dtype=np.float64)
    return K0(n / M, p, q) / M
