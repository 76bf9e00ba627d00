"""Pins of the oracle's Bernstein primitives (Sec. II-D and II-E) to facts that
do not come from the oracle itself: closed forms, exact rational interpolation,
polynomial values at vertices and at sample points."""
from math import comb

import numpy as np
import pytest

from oracle import exact, ref
from paper_2003_01758_amd.instances import poly_eval, poly_eval_many

pytestmark = pytest.mark.filterwarnings("ignore")


def rel_err(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10, 12])
def test_monomial_closed_form(n):
    # x^k of degree n on [0,1]: beta_i = C(i,k)/C(n,k) for i >= k, else 0
    for k in range(n + 1):
        mono = np.zeros(n + 1)
        mono[k] = 1.0
        beta = ref.to_bernstein(mono, [0.0], [1.0])
        want = np.array([comb(i, k) / comb(n, k) for i in range(n + 1)])
        assert np.max(np.abs(beta - want)) <= 4e-16 * n


@pytest.mark.parametrize("n", [1, 3, 6, 10])
def test_identity_gives_uniform_grid(n):
    # x on [0,1] at degree n: beta_i = i/n
    mono = np.zeros(n + 1)
    mono[1] = 1.0
    beta = ref.to_bernstein(mono, [0.0], [1.0])
    assert np.max(np.abs(beta - np.arange(n + 1) / n)) <= 1e-15


@pytest.mark.parametrize("shape", [(1,), (5,), (3, 4), (5, 5), (3, 2, 4), (3, 3, 3, 3)])
def test_partition_of_unity(shape):
    rng = np.random.default_rng(1)
    c = rng.normal()
    mono = np.zeros(shape)
    mono[(0,) * len(shape)] = c
    lo = rng.uniform(-3, 0, size=len(shape))
    hi = lo + rng.uniform(0.1, 4, size=len(shape))
    beta = ref.to_bernstein(mono, lo, hi)
    assert np.max(np.abs(beta - c)) <= 1e-15 * max(1, abs(c))


@pytest.mark.parametrize("shape", [(5,), (5, 5), (7, 3), (3, 4, 2), (3, 3, 3, 3), (11, 11)])
def test_vertex_coefficients_are_values(shape):
    rng = np.random.default_rng(sum(shape))
    for _ in range(5):
        mono = rng.normal(size=shape)
        lo = rng.uniform(-2, 1, size=len(shape))
        hi = lo + rng.uniform(0.25, 2, size=len(shape))
        beta = ref.to_bernstein(mono, lo, hi)
        for corner in np.ndindex(*(2,) * len(shape)):
            J = tuple((s - 1) * c for s, c in zip(shape, corner))
            x = [hi[k] if corner[k] else lo[k] for k in range(len(shape))]
            val = poly_eval(mono, x)
            scale = poly_eval(np.abs(mono), np.maximum(np.abs(lo), np.abs(hi)))
            assert abs(beta[J] - val) <= 1e-13 * max(1.0, scale)


@pytest.mark.parametrize("shape,box", [
    ((4,), ([0], [1])),
    ((6,), ([-1], [1])),
    ((3, 3), ([-1, -1], [1, 1])),
    ((5, 4), ([-0.5, 0.25], [1.5, 0.75])),
    ((3, 2, 3), ([-1, 0, -2], [1, 1, 2])),
    ((11, 11), ([-1, -1], [1, 1])),
])
def test_conversion_matches_exact_interpolation(shape, box):
    rng = np.random.default_rng(7)
    mono = rng.integers(-9, 10, size=shape).astype(float)
    beta = ref.to_bernstein(mono, box[0], box[1])
    want = exact.to_float(exact.bernstein_exact(mono.astype(int), box[0], box[1]))
    # the affine pre-map on a box straddling 0 sums alternating terms of size up to
    # 2^n times the result, so the FP64 error grows like 2^(sum n)/2 ulps
    growth = 2.0 ** (sum(s - 1 for s in shape) / 2)
    assert rel_err(beta, want) <= 1e-14 * growth


@pytest.mark.parametrize("shape", [(5,), (5, 5), (11, 11), (4, 3, 5), (3, 3, 3, 3)])
def test_split_matches_exact_interpolation(shape):
    rng = np.random.default_rng(11)
    mono = rng.integers(-5, 6, size=shape)
    lo = [-1.0] * len(shape)
    hi = [1.0] * len(shape)
    parent = ref.to_bernstein(mono.astype(float), lo, hi)
    for r in range(len(shape)):
        left, right = ref.split(parent, r)
        mid_hi = list(hi)
        mid_hi[r] = 0.0
        mid_lo = list(lo)
        mid_lo[r] = 0.0
        wl = exact.to_float(exact.bernstein_exact(mono, lo, mid_hi))
        wr = exact.to_float(exact.bernstein_exact(mono, mid_lo, hi))
        growth = 2.0 ** (sum(s - 1 for s in shape) / 2)
        assert rel_err(left, wl) <= 1e-14 * growth
        assert rel_err(right, wr) <= 1e-14 * growth


def test_split_commutes_with_conversion_many_levels():
    # splitting d times towards a dyadic sub-box equals converting on it directly
    rng = np.random.default_rng(3)
    mono = rng.normal(size=(7, 6))
    lo, hi = np.array([-1.0, -2.0]), np.array([1.0, 2.0])
    patch = ref.to_bernstein(mono, lo, hi)
    blo, bhi = lo.copy(), hi.copy()
    for s in range(12):
        r = s % 2
        left, right = ref.split(patch, r)
        mid = 0.5 * (blo[r] + bhi[r])
        if rng.integers(2):
            patch, blo[r] = right, mid
        else:
            patch, bhi[r] = left, mid
    direct = ref.to_bernstein(mono, blo, bhi)
    assert rel_err(patch, direct) <= 1e-12


def test_split_mirror_symmetry():
    # right child of a patch = mirror of the left child of the mirrored patch
    rng = np.random.default_rng(5)
    P = rng.normal(size=(9, 6))
    for r in range(2):
        left, right = ref.split(P, r)
        mleft, mright = ref.split(np.flip(P, axis=r), r)
        assert np.array_equal(right, np.flip(mleft, axis=r))
        assert np.array_equal(left, np.flip(mright, axis=r))


def test_split_is_convex_and_nested():
    # children coefficients lie in the parent's range (convex combinations)
    rng = np.random.default_rng(9)
    P = rng.normal(size=(11, 11)) * 10 ** rng.uniform(-3, 3, size=(11, 11))
    for r in range(2):
        for child in ref.split(P, r):
            assert child.min() >= P.min() and child.max() <= P.max()


@pytest.mark.parametrize("shape", [(5, 5), (11, 11), (5, 5, 5), (3, 3, 3, 3)])
def test_range_enclosure_by_sampling(shape):
    # Theorem (enclosure): min B <= p(x) <= max B on the box
    rng = np.random.default_rng(len(shape) * 13 + shape[0])
    for _ in range(4):
        mono = rng.normal(size=shape)
        lo = rng.uniform(-1, 0.5, size=len(shape))
        hi = lo + rng.uniform(0.05, 1, size=len(shape))
        beta = ref.to_bernstein(mono, lo, hi)
        pts = lo + (hi - lo) * rng.uniform(size=(4000, len(shape)))
        vals = poly_eval_many(mono, pts)
        tol = 1e-12 * max(1.0, np.abs(beta).max())
        assert vals.min() >= beta.min() - tol
        assert vals.max() <= beta.max() + tol


def test_gap_shrinks_quadratically():
    # Theorem (error bound): min p - min B <= zeta * 2^(-2n); halving the box
    # around an interior minimiser divides the gap by about 4
    mono = np.zeros((5, 5))
    mono[2, 0] = 1.0
    mono[0, 2] = 2.0
    mono[1, 1] = 0.5
    mono[4, 0] = 0.3
    mono[1, 0] = -0.2
    # interior minimiser: y = -x/8 and 1.9375 x + 1.2 x^3 = 0.2
    x = 0.1
    for _ in range(50):
        x -= (1.9375 * x + 1.2 * x ** 3 - 0.2) / (1.9375 + 3.6 * x ** 2)
    c = np.array([x, -x / 8]) + np.array([0.3, -0.2]) * 2.0 ** -10
    gaps = []
    for n in range(3, 9):
        h = 2.0 ** -n
        beta = ref.to_bernstein(mono, c - h, c + h)
        g = np.linspace(-h, h, 201)
        X, Y = np.meshgrid(c[0] + g, c[1] + g, indexing="ij")
        pmin = poly_eval_many(mono, np.stack([X.ravel(), Y.ravel()], 1)).min()
        gaps.append(pmin - beta.min())
    ratios = np.array(gaps[:-1]) / np.array(gaps[1:])
    assert np.all(gaps > np.zeros(len(gaps)) - 1e-15)
    assert np.all(ratios > 3.0) and np.all(ratios < 5.0)
