"""Exact-rational Bernstein coefficients by interpolation.

TEST INFRASTRUCTURE ONLY.  This is a second, independent route to the
Bernstein coefficients of Sec. II-D, used to pin the oracle's FP64 conversion
and split.  It never uses the conversion matrix or the de Casteljau recurrence:
it evaluates the polynomial exactly at the tensor grid of points
t = (a_1/n_1, ..., a_l/n_l) of the box and solves, one axis at a time, the
Bernstein-Vandermonde system  p(lo + w*t) = sum_J beta_J prod_k b_{j_k,n_k}(t_k),
with b_{j,n}(t) = C(n,j) t^j (1-t)^(n-j), in Fractions.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb
import itertools

import numpy as np


def _frac(x) -> Fraction:
    return x if isinstance(x, Fraction) else Fraction(x)


def eval_exact(mono: np.ndarray, x) -> Fraction:
    """Exact value of the monomial-coefficient tensor at the rational point x."""
    shape = mono.shape
    total = Fraction(0)
    for J in itertools.product(*[range(s) for s in shape]):
        c = mono[J]
        if c == 0:
            continue
        term = _frac(c)
        for k, j in enumerate(J):
            term *= _frac(x[k]) ** j
        total += term
    return total


def _solve(A, b):
    """Exact Gaussian elimination with partial pivoting on Fractions."""
    n = len(A)
    M = [list(map(_frac, row)) + [_frac(v)] for row, v in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def bernstein_exact(mono: np.ndarray, lo, hi) -> np.ndarray:
    """Bernstein coefficients (object array of Fractions) of `mono` over [lo, hi]."""
    mono = np.asarray(mono, dtype=object)
    l = mono.ndim
    deg = [s - 1 for s in mono.shape]
    lo = [_frac(v) for v in lo]
    hi = [_frac(v) for v in hi]
    grids = [[Fraction(a, n) if n > 0 else Fraction(0) for a in range(n + 1)] for n in deg]
    vals = np.empty(mono.shape, dtype=object)
    for A in itertools.product(*[range(s) for s in mono.shape]):
        x = [lo[k] + (hi[k] - lo[k]) * grids[k][A[k]] for k in range(l)]
        vals[A] = eval_exact(mono, x)
    # undo the Bernstein-Vandermonde operator along each axis
    beta = vals
    for k in range(l):
        n = deg[k]
        Bk = [[comb(n, j) * grids[k][a] ** j * (1 - grids[k][a]) ** (n - j)
               for j in range(n + 1)] for a in range(n + 1)]
        moved = np.moveaxis(beta, k, 0)
        out = np.empty(moved.shape, dtype=object)
        for idx in itertools.product(*[range(s) for s in moved.shape[1:]]):
            col = [moved[(a,) + idx] for a in range(n + 1)]
            sol = _solve(Bk, col)
            for j in range(n + 1):
                out[(j,) + idx] = sol[j]
        beta = np.moveaxis(out, 0, k)
    return beta


def to_float(a: np.ndarray) -> np.ndarray:
    return np.vectorize(float, otypes=[np.float64])(a)
