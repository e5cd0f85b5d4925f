"""Pins for the CPU oracle: facts fixed by the paper and by arithmetic, not by the oracle.

Each test would fail for a plausible mistake in the oracle: a dropped or
added term, a wrong skip, a wrong loop order or bound, a transposed operand,
double rather than single precision accumulation, or a wrong count.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -24


def _hex_f32(s):
    return np.float32(float.fromhex(s))


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _rng_case(case, n, seed, int_hi=5, dens=0.6, dyadic=True):
    """Small random inputs: reals with few significant bits, small non-negative ints."""
    r = np.random.default_rng(seed)
    if dyadic:
        real = (r.integers(-64, 64, (n, n)) / 64.0).astype(np.float32)
    else:
        real = r.standard_normal((n, n)).astype(np.float32)
    real[r.random((n, n)) > dens] = 0
    ints = r.integers(0, int_hi + 1, (n, n)).astype(np.int32)
    ints[r.random((n, n)) > dens] = 0
    return (real, ints) if case == "A" else (ints, real)


# --------------------------------------------------------------------------
# Hand-worked fixtures (golden files carry the citations)

@pytest.mark.parametrize("c", _load("order_and_rounding.json")["cases"], ids=lambda c: c["name"])
def test_golden_order_and_rounding(c):
    case = c["case"]
    if case == "A":
        X = np.array([[_hex_f32(v) for v in row] for row in c["X"]], np.float32)
        Y = np.array(c["Y"], np.int32)
    else:
        X = np.array(c["X"], np.int32)
        Y = np.array([[_hex_f32(v) for v in row] for row in c["Y"]], np.float32)
    Z, adds = oracle.strict_f32(case, X, Y)
    assert adds == c["adds"]
    if "Z00" in c:
        assert Z[0, 0].view(np.uint32) == _hex_f32(c["Z00"]).view(np.uint32)
        assert Z[0, 0] != _hex_f32(c["wrong_Z00"])
    if "Z" in c:
        Zexp = np.array([[_hex_f32(v) for v in row] for row in c["Z"]], np.float32)
        assert np.array_equal(Z.view(np.uint32), Zexp.view(np.uint32))
    total, _, _ = oracle.count(case, X, Y)
    assert total == c["adds"]


def test_golden_bf16_rne():
    d = _load("bf16_rne.json")
    xs = np.array([_hex_f32(c["x"]) for c in d["cases"]], np.float32)
    hi, _, _ = oracle.split_bf16x3(xs)
    for c, h in zip(d["cases"], hi):
        assert int(h) == int(c["bf16"], 16), c


def _bf16_exact(h):
    """bfloat16 pattern -> exact rational (normal and zero patterns only)."""
    h = int(h)
    sign = -1 if h & 0x8000 else 1
    e, m = (h >> 7) & 0xFF, h & 0x7F
    assert e != 0xFF
    if e == 0:
        return Fraction(sign * m, 2 ** 133)
    return sign * Fraction(128 + m, 128) * Fraction(2) ** (e - 127)


@pytest.mark.parametrize("c", _load("split_bf16x3.json")["cases"], ids=lambda c: c["x"])
def test_golden_split_bf16x3(c):
    """hi, mid and lo of hand-worked values where the rounding of mid decides the
    patterns (a truncated or round-half-away mid fails), and hi + mid + lo == x."""
    x = _hex_f32(c["x"])
    hi, mid, lo = (int(t[0]) for t in oracle.split_bf16x3(np.array([x], np.float32)))
    assert (hi, mid, lo) == (int(c["hi"], 16), int(c["mid"], 16), int(c["lo"], 16)), c["why"]
    assert _bf16_exact(hi) + _bf16_exact(mid) + _bf16_exact(lo) == Fraction(float(x))


# --------------------------------------------------------------------------
# Brute force against exact rationals (n <= 8)

def _exact_product(case, X, Y):
    n = X.shape[0]
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    Yf = [[Fraction(float(v)) for v in row] for row in Y]
    return [[sum((Xf[i][k] * Yf[k][j] for k in range(n)), Fraction(0)) for j in range(n)]
            for i in range(n)]


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (8, 4), (8, 5)])
def test_bruteforce_exact_rational(case, n, seed):
    X, Y = _rng_case(case, n, seed, dyadic=False)
    exact = _exact_product(case, X, Y)
    Z64 = oracle.product_f64(case, X, Y)
    Z32, adds = oracle.strict_f32(case, X, Y)
    real, ints = (X, Y) if case == "A" else (Y, X)
    for i in range(n):
        for j in range(n):
            # binary64 sum of n exact terms: |err| <= gamma_{n-1} * sum |terms|
            s_abs = sum(abs(Fraction(float(X[i, k])) * Fraction(float(Y[k, j]))) for k in range(n))
            g64 = (n * 2.0 ** -53) / (1 - n * 2.0 ** -53)
            assert abs(Fraction(float(Z64[i, j])) - exact[i][j]) <= Fraction(g64) * s_abs
            # binary32 repeated addition: m additions of terms; Higham's recursive summation
            # bound |err| <= gamma_{m-1} * sum |terms| with sum |terms| = s_abs
            m = sum(int(ints[k, j] if case == "A" else ints[i, k]) for k in range(n)
                    if (X[i, k] != 0 and Y[k, j] != 0))
            g32 = (max(m - 1, 0) * U) / (1 - max(m - 1, 0) * U)
            assert abs(Fraction(float(Z32[i, j])) - exact[i][j]) <= Fraction(g32) * s_abs


@pytest.mark.parametrize("case", ["A", "B"])
def test_bruteforce_count_tiny(case):
    for seed in range(6):
        X, Y = _rng_case(case, 6, seed)
        n = 6
        brute = 0
        for i in range(n):
            for k in range(n):
                for j in range(n):
                    base, rep = (X[i, k], Y[k, j]) if case == "A" else (Y[k, j], X[i, k])
                    if base != 0 and rep > 0:
                        brute += int(rep)
        _, adds = oracle.strict_f32(case, X, Y)
        total, rows, flags = oracle.count(case, X, Y)
        assert adds == brute == total == int(rows.sum())
        assert flags == 0


# --------------------------------------------------------------------------
# Identities that reduce the method to exact arithmetic or library routines

@pytest.mark.parametrize("case", ["A", "B"])
def test_integer_valued_reals_equal_exact_product(case):
    """When every partial sum is an integer below 2^24, repeated addition is exact."""
    r = np.random.default_rng(7)
    n = 40
    real = r.integers(-20, 21, (n, n)).astype(np.float32)
    real[r.random((n, n)) < 0.3] = 0
    ints = r.integers(0, 10, (n, n)).astype(np.int32)
    X, Y = (real, ints) if case == "A" else (ints, real)
    Z, _ = oracle.strict_f32(case, X, Y)
    exact = X.astype(np.int64) @ Y.astype(np.int64)
    assert np.abs(exact).max() < 2 ** 24
    assert np.array_equal(Z, exact.astype(np.float32))
    assert np.array_equal(oracle.product_f64(case, X, Y), exact.astype(np.float64))


def test_identity_caseA():
    w = gen.caseA_n256()
    X = w.X()[:64, :64].copy()
    Z, adds = oracle.caseA_f32(X, np.eye(64, dtype=np.int32))
    assert np.array_equal(Z.view(np.uint32), X.view(np.uint32))
    assert adds == int((X != 0).sum())


def test_identity_caseB():
    r = np.random.default_rng(3)
    Y = r.standard_normal((50, 50)).astype(np.float32)
    Y[r.random((50, 50)) < 0.2] = 0
    Z, adds = oracle.caseB_f32(np.eye(50, dtype=np.int32), Y)
    assert np.array_equal(Z.view(np.uint32), Y.view(np.uint32))
    assert adds == int((Y != 0).sum())


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("zero", ["real", "int"])
def test_zero_density(case, zero):
    X, Y = _rng_case(case, 30, 11)
    if (zero == "real") == (case == "A"):
        X = np.zeros_like(X)
    else:
        Y = np.zeros_like(Y)
    Z, adds = oracle.strict_f32(case, X, Y)
    assert adds == 0
    assert not Z.view(np.uint32).any()  # all +0.0, no -0.0
    assert oracle.count(case, X, Y)[0] == 0


def test_all_ones_rep_is_sequential_row_sum():
    """Case A with Y = 1: each Z[i,j] is the left-to-right binary32 sum of row i of X."""
    r = np.random.default_rng(5)
    n = 300
    X = r.standard_normal((n, n)).astype(np.float32)
    X[r.random((n, n)) < 0.4] = 0
    Z, _ = oracle.caseA_f32(X, np.ones((n, n), np.int32))
    seq = np.add.accumulate(X, axis=1, dtype=np.float32)[:, -1]
    for j in (0, 17, n - 1):
        assert np.array_equal(Z[:, j].view(np.uint32), seq.view(np.uint32))
    assert np.array_equal(Z, np.repeat(Z[:, :1], n, axis=1))
    # pairwise or double accumulation would differ somewhere
    assert not np.array_equal(seq, X.astype(np.float64).sum(axis=1).astype(np.float32))


def test_constant_rep_caseB_is_sequential_repeated_column_sum():
    """Case B with X = c everywhere: Z[i,j] adds Y[0,j] c times, then Y[1,j] c times, ..."""
    r = np.random.default_rng(6)
    n, c = 64, 3
    Y = r.standard_normal((n, n)).astype(np.float32)
    Z, adds = oracle.caseB_f32(np.full((n, n), c, np.int32), Y)
    seq = np.add.accumulate(np.repeat(Y, c, axis=0), axis=0, dtype=np.float32)[-1]
    assert np.array_equal(Z[5].view(np.uint32), seq.view(np.uint32))
    assert adds == n * c * int((Y != 0).sum())


# --------------------------------------------------------------------------
# Structural invariants

def test_transpose_duality():
    """Case A on (X, Y) performs, per element, the same additions as case B on (Y^T, X^T)."""
    r = np.random.default_rng(9)
    n = 70
    X = r.standard_normal((n, n)).astype(np.float32)
    X[r.random((n, n)) < 0.5] = 0
    Y = r.integers(0, 7, (n, n)).astype(np.int32)
    ZA, aA = oracle.caseA_f32(X, Y)
    ZB, aB = oracle.caseB_f32(np.ascontiguousarray(Y.T), np.ascontiguousarray(X.T))
    assert aA == aB
    assert np.array_equal(ZA.view(np.uint32), np.ascontiguousarray(ZB.T).view(np.uint32))


@pytest.mark.parametrize("case", ["A", "B"])
def test_permutation_equivariance(case):
    X, Y = _rng_case(case, 48, 21, int_hi=6, dyadic=False)
    r = np.random.default_rng(1)
    pr, pc = r.permutation(48), r.permutation(48)
    Z, _ = oracle.strict_f32(case, X, Y)
    Zp, _ = oracle.strict_f32(case, X[pr], Y[:, pc])
    assert np.array_equal(Zp.view(np.uint32), Z[pr][:, pc].view(np.uint32))


@pytest.mark.parametrize("case", ["A", "B"])
def test_power_of_two_scaling(case):
    X, Y = _rng_case(case, 40, 31, dyadic=False)
    Z, _ = oracle.strict_f32(case, X, Y)
    for s in (-5, 3):
        f = np.float32(2.0 ** s)
        Xs, Ys = (X * f, Y) if case == "A" else (X, Y * f)
        Zs, _ = oracle.strict_f32(case, Xs, Ys)
        assert np.array_equal(Zs.view(np.uint32), (Z * f).view(np.uint32))


def test_rows_subset_matches_full():
    w = gen.caseB_n4096(n=300)
    X, Y = w.X(), w.Y()
    Z, _ = oracle.caseB_f32(X, Y)
    rows = [0, 7, 150, 299]
    Zr, _ = oracle.caseB_f32(X, Y, rows=rows)
    Zr2, _ = oracle.caseB_f32(X[rows], Y, rows=rows, x_rows_only=True)
    assert np.array_equal(Zr, Z[rows]) and np.array_equal(Zr2, Z[rows])
    Z64 = oracle.product_f64("B", X, Y)
    assert np.array_equal(oracle.product_f64("B", X[rows], Y, rows=rows, x_rows_only=True),
                          Z64[rows])


def test_product_f64_matches_blas():
    w = gen.caseA_n256()
    X, Y = w.X(), w.Y()
    Z64 = oracle.product_f64("A", X, Y)
    assert np.max(np.abs(Z64 - oracle.product_f64_blas(X, Y))) <= 1e-12 * np.abs(Z64).max()


# --------------------------------------------------------------------------
# Counting (Section 2.2)

@pytest.mark.parametrize("case", ["A", "B"])
def test_count_equals_instrumented_counter(case):
    X, Y = _rng_case(case, 120, 41, int_hi=9)
    _, adds = oracle.strict_f32(case, X, Y)
    total, rows, flags = oracle.count(case, X, Y)
    assert total == adds == int(rows.sum()) and flags == 0
    Z1, a1 = oracle.strict_f32(case, X, Y, rows=[3])
    assert a1 == int(rows[3])


def test_count_flags_and_negative_reps():
    X = np.array([[1.0, 2.0], [0.0, 1.0]], np.float32)
    Y = np.array([[-3, 300], [256, 1]], np.int32)
    Z, adds = oracle.caseA_f32(X, Y)
    total, rows, flags = oracle.count("A", X, Y)
    # the negative Rep-factor adds nothing (empty sum)
    assert adds == total == 300 + 256 + 1 + 256 + 1
    assert flags & oracle.NEGATIVE and flags & oracle.ABOVE255 and flags & oracle.ABOVE256
    assert Z[0, 0] == np.float32(2.0 * 256)


def test_count_overflow_saturates():
    n = 64
    X = np.full((n, n), 2 ** 31 - 1, np.int32)
    Y = np.ones((n, n), np.float32)
    total, rows, flags = oracle.count("B", X, Y)
    exact = n * n * n * (2 ** 31 - 1)
    assert exact < 2 ** 64 and total == exact and not flags & oracle.OVERFLOW
    n = 4096
    X = np.full((n, n), 2 ** 31 - 1, np.int32)
    Y = np.ones((n, n), np.float32)
    total, _, flags = oracle.count("B", X, Y)
    assert n ** 3 * (2 ** 31 - 1) >= 2 ** 64
    assert flags & oracle.OVERFLOW and total == 2 ** 64 - 1


def _z_score(case, X, Y, w):
    """(C - mu' d1 d2 n^3) / sigma with sigma from the k-independent terms of the count."""
    n = w.n
    real, ints = (X, Y) if case == "A" else (Y, X)
    if case == "A":
        terms = (X != 0).sum(axis=0).astype(np.float64) * np.maximum(Y, 0).sum(axis=1)
    else:
        terms = np.maximum(X, 0).sum(axis=0).astype(np.float64) * (Y != 0).sum(axis=1)
    total = oracle.count(case, X, Y)[0]
    assert total == int(terms.sum())
    expect = w.expected_adds()
    sigma = math.sqrt(n * terms.var())
    return (total - expect) / sigma


def test_count_statistical_caseA_n256():
    w = gen.caseA_n256()
    X, Y = w.X(), w.Y()
    # mu' d1 d2 n^3: mu' = 5 (Uniform{1..9}), d1 = 0.5, d2 = 0.8
    assert w.expected_adds() == pytest.approx(5 * 0.5 * 0.8 * 256 ** 3)
    assert abs(_z_score("A", X, Y, w)) <= 5


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("d1,d2", [(0.1, 0.5), (1.0, 0.1), (0.5, 1.0)])
def test_count_statistical_sweep(case, d1, d2):
    w = gen.sweep_n2048(case, d1, d2, n=512)
    X, Y = w.X(), w.Y()
    assert abs(_z_score(case, X, Y, w)) <= 5


def test_count_statistical_caseB_n4096_rows():
    w = gen.caseB_n4096(n=1024)
    X, Y = w.X(), w.Y()
    assert abs(_z_score("B", X, Y, w)) <= 5


# --------------------------------------------------------------------------
# Split-precision pins

def test_split_exact_reconstruction():
    w = gen.caseB_n4096(n=512)
    Y = w.Y().ravel()
    r = np.random.default_rng(2)
    # exact for 2^-100 <= |x| < 2^127: below, the third term would need bits under
    # bfloat16's smallest subnormal; at the top, hi can round to infinity
    extra = np.concatenate([r.standard_normal(10000) * 10.0 ** r.integers(-30, 30, 10000),
                            [2.0 ** -100, -3 * 2.0 ** -99, 1.5 * 2.0 ** 126, 0.0, 1.0, -1.0]]
                           ).astype(np.float32)
    for x in (Y, extra):
        hi, mid, lo = oracle.split_bf16x3(x)
        s = oracle.bf16_to_f64(hi) + oracle.bf16_to_f64(mid) + oracle.bf16_to_f64(lo)
        assert np.array_equal(s, x.astype(np.float64))
        # each term carries the leading bits of what the previous left
        h = oracle.bf16_to_f64(hi)
        assert np.all(np.abs(x.astype(np.float64) - h) <= np.abs(h) * 2.0 ** -8)


def test_split_product_in_f64_equals_true_product():
    """sum over the three terms of (term . integer factor) in binary64 == the binary64 product."""
    w = gen.caseB_n4096(n=96)
    X, Y = w.X(), w.Y()
    hi, mid, lo = oracle.split_bf16x3(Y)
    parts = sum(X.astype(np.float64) @ oracle.bf16_to_f64(t).reshape(Y.shape) for t in (hi, mid, lo))
    Z64 = oracle.product_f64("B", X, Y)
    assert np.max(np.abs(parts - Z64)) <= 1e-13 * np.abs(Z64).max()


def test_strict_error_vs_true_product_is_bounded():
    """Strict binary32 repeated addition stays within Higham's bound of the true product."""
    w = gen.caseB_n4096(n=256)
    X, Y = w.X(), w.Y()
    Z32, _ = oracle.caseB_f32(X, Y)
    Z64 = oracle.product_f64("B", X, Y)
    m = X.sum(axis=1).astype(np.float64)[:, None]        # additions per element (upper bound)
    bound = (m * U / (1 - m * U)) * (np.abs(X).astype(np.float64) @ np.abs(Y).astype(np.float64))
    assert np.all(np.abs(Z32 - Z64) <= bound)
    assert 1e-8 < oracle.rel_frobenius(Z32, Z64) < 1e-5


# --------------------------------------------------------------------------
# Rectangular shapes (the same loops with separate i, k, j bounds)

def _rng_rect(case, m, kd, n, seed, int_hi=5, dens=0.6):
    r = np.random.default_rng(seed)
    xs, ys = (m, kd), (kd, n)
    if case == "A":
        X = r.standard_normal(xs).astype(np.float32)
        X[r.random(xs) > dens] = 0
        Y = r.integers(0, int_hi + 1, ys).astype(np.int32)
        Y[r.random(ys) > dens] = 0
    else:
        X = r.integers(0, int_hi + 1, xs).astype(np.int32)
        X[r.random(xs) > dens] = 0
        Y = r.standard_normal(ys).astype(np.float32)
        Y[r.random(ys) > dens] = 0
    return X, Y


RECT = [(1, 5, 3), (4, 1, 6), (3, 7, 2), (6, 3, 1), (2, 8, 5)]


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("m,kd,n", RECT)
def test_rect_bruteforce_exact_rational(case, m, kd, n):
    """m x kd times kd x n: both oracles within their rounding bounds of the exact
    rational product, and the count equal to brute force."""
    X, Y = _rng_rect(case, m, kd, n, 100 * m + 10 * kd + n)
    Z64 = oracle.product_f64(case, X, Y)
    Z32, adds = oracle.strict_f32(case, X, Y)
    assert Z32.shape == Z64.shape == (m, n)
    ints = Y if case == "A" else X
    brute = 0
    for i in range(m):
        for j in range(n):
            terms = [Fraction(float(X[i, k])) * Fraction(float(Y[k, j])) for k in range(kd)]
            exact = sum(terms, Fraction(0))
            s_abs = sum(abs(t) for t in terms)
            g64 = (kd * 2.0 ** -53) / (1 - kd * 2.0 ** -53)
            assert abs(Fraction(float(Z64[i, j])) - exact) <= Fraction(g64) * s_abs
            reps = sum(int(ints[k, j] if case == "A" else ints[i, k]) for k in range(kd)
                       if X[i, k] != 0 and Y[k, j] != 0)
            brute += reps
            g32 = (max(reps - 1, 0) * U) / (1 - max(reps - 1, 0) * U)
            assert abs(Fraction(float(Z32[i, j])) - exact) <= Fraction(g32) * s_abs
    total, rows, flags = oracle.count(case, X, Y)
    assert adds == brute == total == int(rows.sum()) and rows.shape == (m,) and flags == 0


def test_rect_transpose_duality():
    """Case A on an m x kd and a kd x n factor adds, per element, what case B adds on
    the transposed factors (n x kd times kd x m)."""
    X, Y = _rng_rect("A", 13, 29, 7, 5)
    ZA, aA = oracle.caseA_f32(X, Y)
    ZB, aB = oracle.caseB_f32(np.ascontiguousarray(Y.T), np.ascontiguousarray(X.T))
    assert aA == aB and ZA.shape == (13, 7) and ZB.shape == (7, 13)
    assert np.array_equal(ZA.view(np.uint32), np.ascontiguousarray(ZB.T).view(np.uint32))


@pytest.mark.parametrize("case", ["A", "B"])
def test_rect_blocks_of_square_product(case):
    """Rows of Z depend only on their row of X, columns only on their column of Y
    (Section 2.1): a rectangular product of row and column blocks equals the same block
    of the square product, bit for bit, and so do the counts of its rows."""
    X, Y = _rng_case(case, 40, 31, int_hi=6, dyadic=False)
    Z, _ = oracle.strict_f32(case, X, Y)
    Zb, _ = oracle.strict_f32(case, X[5:17], Y[:, 9:30])
    assert np.array_equal(Zb.view(np.uint32), Z[5:17, 9:30].view(np.uint32))
    Zr, _ = oracle.strict_f32(case, X[:, :40], Y[:40, :])
    assert np.array_equal(Zr.view(np.uint32), Z.view(np.uint32))
    # columns beyond a kd-slice change: a shorter reduction is a different product
    Zk, _ = oracle.strict_f32(case, X[:, :20], Y[:20, :])
    Zk2, _ = oracle.strict_f32(case, np.hstack([X[:, :20], 0 * X[:, 20:]]), Y)
    assert np.array_equal(Zk.view(np.uint32), Zk2.view(np.uint32))


def test_rect_leading_dimensions_in_c():
    """The C oracle's leading-dimension arguments: a product read out of padded buffers
    equals the compact one, and nothing outside the m x n block of Z is written."""
    import ctypes
    X, Y = _rng_rect("B", 9, 14, 6, 77)
    Zc, ac = oracle.caseB_f32(X, Y)
    ldx, ldy, ldz = 17, 11, 10
    Xp = np.full((9, ldx), 123456, np.int32)
    Xp[:, :14] = X
    Yp = np.full((14, ldy), np.nan, np.float32)
    Yp[:, :6] = Y
    Zp = np.full((9, ldz), -7.0, np.float32)
    a = oracle.lib().afmm_oracle_caseB_f32_ex(9, 14, 6, Xp.ctypes.data, ldx, Yp.ctypes.data, ldy,
                                              Zp.ctypes.data, ldz, None, 9, 0)
    assert a == ac
    assert np.array_equal(Zp[:, :6].view(np.uint32), Zc.view(np.uint32))
    assert (Zp[:, 6:] == -7.0).all()
    tot = np.zeros(1, np.uint64)
    rows = np.zeros(9, np.uint64)
    fl = oracle.lib().afmm_oracle_count_ex(1, 9, 14, 6, Xp.ctypes.data, ldx, Yp.ctypes.data, ldy,
                                           tot.ctypes.data, rows.ctypes.data)
    assert fl == 0 and int(tot[0]) == ac
    del ctypes


@pytest.mark.parametrize("case", ["A", "B"])
def test_threaded_oracle_equals_single_call(case):
    """Row ranges on several threads give the single call's bits and count."""
    X, Y = _rng_case(case, 203, 77, int_hi=9, dyadic=False)
    Z1, a1 = oracle.strict_f32(case, X, Y)
    Z2, a2 = oracle.strict_f32_threaded(case, X, Y, threads=7)
    assert a1 == a2
    assert np.array_equal(Z1.view(np.uint32), Z2.view(np.uint32))
