"""CPU oracle for AFMM -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrappers over ``liboracle.so`` (plain single-threaded C, see
``afmm_oracle.h`` for what each function computes and the readings of the
paper it takes).  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package; the product library
never does, and shares no code with it.

``product_f64_blas`` is the one exception to "plain C": the true product of
Section 2.1 computed with a library matrix product in binary64, used where
the plain loop would take minutes (full n=4096 error checks).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NEGATIVE, ABOVE255, ABOVE256, OVERFLOW, FPENV = 1, 2, 4, 8, 16
U64_MAX = (1 << 64) - 1


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        i64, u64, vp, ci = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        for name in ("afmm_oracle_caseA_f32", "afmm_oracle_caseB_f32"):
            f = getattr(L, name)
            f.argtypes = [i64, vp, vp, vp, vp, i64, ci]
            f.restype = u64
            f = getattr(L, name + "_ex")
            f.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, ci]
            f.restype = u64
        L.afmm_oracle_product_f64.argtypes = [ci, i64, vp, vp, vp, vp, i64, ci]
        L.afmm_oracle_product_f64.restype = None
        L.afmm_oracle_product_f64_ex.argtypes = [ci, i64, i64, i64, vp, i64, vp, i64, vp, i64,
                                                 vp, i64, ci]
        L.afmm_oracle_product_f64_ex.restype = None
        L.afmm_oracle_count.argtypes = [ci, i64, vp, vp, vp, vp]
        L.afmm_oracle_count.restype = ctypes.c_uint
        L.afmm_oracle_count_ex.argtypes = [ci, i64, i64, i64, vp, i64, vp, i64, vp, vp]
        L.afmm_oracle_count_ex.restype = ctypes.c_uint
        L.afmm_oracle_split_bf16x3.argtypes = [i64, vp, vp, vp, vp]
        L.afmm_oracle_split_bf16x3.restype = None
        _lib = L
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _rows_arg(rows):
    if rows is None:
        return None, None
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    return r, r.ctypes.data


def _shapes(X, Y, r, x_rows_only):
    """(m, kd, n, output rows) of X (m x kd, or the listed rows only) times Y (kd x n)."""
    kd, n = Y.shape
    assert X.shape[1] == kd, (X.shape, Y.shape)
    m = X.shape[0] if not x_rows_only else None
    nout = (m if r is None else len(r))
    if x_rows_only:
        assert r is not None and X.shape[0] == len(r)
        m = int(r.max()) + 1 if len(r) else 0
    return m, kd, n, nout


def _strict(name, X, Y, xdt, ydt, rows, x_rows_only):
    """Rectangular strict loop (X m x kd, Y kd x n; the square case is m = kd = n)."""
    X = _c(X, xdt)
    Y = _c(Y, ydt)
    r, rp = _rows_arg(rows)
    m, kd, n, nout = _shapes(X, Y, r, x_rows_only)
    Z = np.empty((nout, n), dtype=np.float32)
    adds = getattr(lib(), name + "_ex")(m, kd, n, X.ctypes.data, kd, Y.ctypes.data, n,
                                        Z.ctypes.data, n, rp, nout, 1 if x_rows_only else 0)
    if adds == U64_MAX:
        raise RuntimeError("CPU flushes denormals (FTZ/DAZ set); oracle results void")
    return Z, int(adds)


def caseA_f32(X, Y, rows=None, x_rows_only=False):
    """Strict FP32 case A in the paper's (i,k,j,p) order -> (Z rows, additions).
    X is m x kd (or only the listed rows with x_rows_only), Y is kd x n."""
    return _strict("afmm_oracle_caseA_f32", X, Y, np.float32, np.int32, rows, x_rows_only)


def caseB_f32(X, Y, rows=None, x_rows_only=False):
    """Strict FP32 case B in the paper's (i,k,j,p) order -> (Z rows, additions)."""
    return _strict("afmm_oracle_caseB_f32", X, Y, np.int32, np.float32, rows, x_rows_only)


def strict_f32(case, X, Y, rows=None, x_rows_only=False):
    return (caseA_f32 if case == "A" else caseB_f32)(X, Y, rows, x_rows_only)


def strict_f32_threaded(case, X, Y, threads=None):
    """The same strict loop over disjoint row ranges on several host threads (rows
    of Z are independent, Section 2.1, so the result is bit-identical to one
    call; the C loop runs outside the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    m = X.shape[0]
    threads = max(1, min(threads or os.cpu_count() or 1, m))
    bounds = np.linspace(0, m, threads + 1).astype(np.int64)
    parts = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    X = np.ascontiguousarray(X)

    def run(ab):
        rows = np.arange(ab[0], ab[1], dtype=np.int64)
        return strict_f32(case, X[ab[0]:ab[1]], Y, rows=rows, x_rows_only=True)

    with ThreadPoolExecutor(len(parts)) as ex:
        res = list(ex.map(run, parts))
    return np.concatenate([z for z, _ in res]), sum(a for _, a in res)


def product_f64(case, X, Y, rows=None, x_rows_only=False):
    """True product X.Y in binary64 (plain loop, k ascending) for the listed rows."""
    xdt, ydt = (np.float32, np.int32) if case == "A" else (np.int32, np.float32)
    X = _c(X, xdt)
    Y = _c(Y, ydt)
    r, rp = _rows_arg(rows)
    m, kd, n, nout = _shapes(X, Y, r, x_rows_only)
    Z = np.empty((nout, n), dtype=np.float64)
    lib().afmm_oracle_product_f64_ex(0 if case == "A" else 1, m, kd, n, X.ctypes.data, kd,
                                     Y.ctypes.data, n, Z.ctypes.data, n, rp, nout,
                                     1 if x_rows_only else 0)
    return Z


def product_f64_blas(X, Y):
    """True product in binary64 by a library matrix product (large sizes only)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(Y, dtype=np.float64)


def count(case, X, Y):
    """Exact addition count -> (total, per-row counts, flag bits)."""
    xdt, ydt = (np.float32, np.int32) if case == "A" else (np.int32, np.float32)
    X = _c(X, xdt)
    Y = _c(Y, ydt)
    m, kd, n, _ = _shapes(X, Y, None, False)
    tot = np.zeros(1, dtype=np.uint64)
    rows = np.zeros(m, dtype=np.uint64)
    flags = lib().afmm_oracle_count_ex(0 if case == "A" else 1, m, kd, n, X.ctypes.data, kd,
                                       Y.ctypes.data, n, tot.ctypes.data, rows.ctypes.data)
    return int(tot[0]), rows, int(flags)


def split_bf16x3(x):
    """Three-term bfloat16 split of binary32 values -> (hi, mid, lo) bit patterns."""
    x = _c(x, np.float32)
    hi = np.empty(x.shape, np.uint16)
    mid = np.empty(x.shape, np.uint16)
    lo = np.empty(x.shape, np.uint16)
    lib().afmm_oracle_split_bf16x3(x.size, x.ctypes.data, hi.ctypes.data, mid.ctypes.data,
                                   lo.ctypes.data)
    return hi, mid, lo


def bf16_to_f64(h):
    """bfloat16 bit patterns -> binary64 values (exact)."""
    return (np.asarray(h, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel_frobenius(Z, Zref):
    """||Z - Zref||_F / ||Zref||_F in binary64."""
    Z = np.asarray(Z, np.float64)
    Zref = np.asarray(Zref, np.float64)
    den = np.linalg.norm(Zref)
    num = np.linalg.norm(Z - Zref)
    return float(num / den) if den > 0 else float(num)
