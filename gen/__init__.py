"""Seeded synthetic inputs for AFMM workloads (host side).

Only random matrices live here: no step of the method's arithmetic.  The
draws come from ``libafmm_gen.so`` (counter-based SplitMix64, see
``afmm_gen.h``), so any subset of rows of any workload regenerates
bit-identically; the oracle's tests, the GPU parity tests and the benchmark
all draw their inputs from this module.

Workloads follow the paper's setting (Section 2: a real factor whose
non-zeros have density d, an integer "Rep-factor" whose non-zero mean is
mu'), at the shapes the benchmark and the parity tests use.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libafmm_gen.so")
_lib = None

UNIFORM01, UNIFORMPM1, NORMAL = 0, 1, 2
INT_UNIFORM, INT_POISSON, INT_GEOMETRIC = 0, 1, 2

SEED0 = 13082400
# stream ids: X mask/value, Y mask/value; variant v shifts them by 16 * (v + 1)
S_XMASK, S_XVAL, S_YMASK, S_YVAL = 1, 2, 3, 4
S_BATCH_DESC = 0xBA7C


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        i64, u64, f64, i32, vp = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_void_p)
        L.afmm_gen_draw.argtypes = [u64, u64, u64]
        L.afmm_gen_draw.restype = u64
        L.afmm_gen_real.argtypes = [vp, i64, i64, i64, u64, u64, u64, f64, ctypes.c_int]
        L.afmm_gen_real.restype = None
        L.afmm_gen_int.argtypes = [vp, i64, i64, i64, u64, u64, u64, f64, ctypes.c_int,
                                   f64, f64, i32, i32]
        L.afmm_gen_int.restype = None
        _lib = L
    return _lib


def draw(seed: int, stream: int, idx: int) -> int:
    return int(lib().afmm_gen_draw(seed, stream, idx))


@dataclass(frozen=True)
class RealSpec:
    dist: int
    density: float

    def mean_abs_nonzero(self) -> float:
        return {UNIFORM01: 0.5, UNIFORMPM1: 0.5, NORMAL: math.sqrt(2 / math.pi)}[self.dist]


@dataclass(frozen=True)
class IntSpec:
    dist: int
    density: float
    a: float
    b: float = 0.0
    clip_lo: int = 0
    clip_hi: int = 255

    def value_mean(self) -> float:
        """E[v] of a kept entry (clipping ignored: negligible at the used parameters)."""
        if self.dist == INT_UNIFORM:
            return (self.a + self.b) / 2.0
        if self.dist == INT_POISSON:
            return self.a
        return (1.0 - self.a) / self.a

    def value_p_zero(self) -> float:
        if self.dist == INT_UNIFORM:
            return 1.0 / (self.b - self.a + 1) if self.a <= 0 <= self.b else 0.0
        if self.dist == INT_POISSON:
            return math.exp(-self.a)
        return self.a

    def entry_mean(self) -> float:
        return self.density * self.value_mean()

    def mu_prime(self) -> float:
        """Mean of the non-zero entries (the paper's mu')."""
        pnz = self.density * (1.0 - self.value_p_zero())
        return self.entry_mean() / pnz if pnz > 0 else 0.0


@dataclass(frozen=True)
class Workload:
    """One AFMM product: case 'A' (X real, Y integer) or 'B' (X integer, Y real)."""
    name: str
    case: str
    n: int
    real: RealSpec
    int_: IntSpec
    seed: int
    variant: int = -1  # -1: base streams; v >= 0: streams shifted by 16 * (v + 1)

    def streams(self):
        off = 16 * (self.variant + 1) if self.variant >= 0 else 0
        return (S_XMASK + off, S_XVAL + off, S_YMASK + off, S_YVAL + off)

    @property
    def d1(self) -> float:
        return self.real.density if self.case == "A" else self.int_.density

    @property
    def d2(self) -> float:
        return self.int_.density if self.case == "A" else self.real.density

    def expected_adds(self) -> float:
        """mu' * d_real * d_int' * n^3 with d_int' the true non-zero fraction (Section 2.2)."""
        return self.n ** 3 * self.real.density * self.int_.entry_mean()

    def _real_rows(self, which: str, rows):
        sm, sv = (self.streams()[0:2] if which == "X" else self.streams()[2:4])
        return _rows(lambda out, nr, r0: lib().afmm_gen_real(
            out.ctypes.data, nr, self.n, r0, self.seed, sm, sv, self.real.density,
            self.real.dist), np.float32, self.n, rows)

    def _int_rows(self, which: str, rows):
        sm, sv = (self.streams()[0:2] if which == "X" else self.streams()[2:4])
        s = self.int_
        return _rows(lambda out, nr, r0: lib().afmm_gen_int(
            out.ctypes.data, nr, self.n, r0, self.seed, sm, sv, s.density, s.dist,
            float(s.a), float(s.b), s.clip_lo, s.clip_hi), np.int32, self.n, rows)

    def X(self, rows=None) -> np.ndarray:
        return self._real_rows("X", rows) if self.case == "A" else self._int_rows("X", rows)

    def Y(self, rows=None) -> np.ndarray:
        return self._int_rows("Y", rows) if self.case == "A" else self._real_rows("Y", rows)


def _rows(fill, dtype, n, rows):
    if rows is None:
        out = np.empty((n, n), dtype=dtype)
        fill(out, n, 0)
        return out
    rows = [int(r) for r in rows]
    out = np.empty((len(rows), n), dtype=dtype)
    for t, r in enumerate(rows):
        fill(out[t:t + 1], 1, r)
    return out


def _with(w: Workload, **kw) -> Workload:
    d = dict(w.__dict__)
    d.update(kw)
    return Workload(**d)


# ---------------------------------------------------------------------------
# The workloads.  Real factor / integer factor distributions and densities
# follow the paper's experiment design (Section 2.3.1: random reals masked
# to density d, integer factor of mean mu'), at the sizes used here.

def caseA_n256() -> Workload:
    """Case A, n=256: X ~ U(0,1) kept w.p. 0.5, Y ~ U{1..9} kept w.p. 0.8."""
    return Workload("caseA_n256", "A", 256, RealSpec(UNIFORM01, 0.5),
                    IntSpec(INT_UNIFORM, 0.8, 1, 9), SEED0 + 1)


SWEEP_D = (0.1, 0.5, 1.0)


def sweep_n2048(case: str, d1: float, d2: float, n: int = 2048) -> Workload:
    """Cases A/B, n=2048: real ~ U(-1,1), integer ~ U{0..15}; d1 (X) and d2 (Y) swept."""
    a = SWEEP_D.index(d1)
    b = SWEEP_D.index(d2)
    v = 2 * (3 * a + b) + (1 if case == "B" else 0)
    d_real, d_int = (d1, d2) if case == "A" else (d2, d1)
    return Workload(f"sweep_n{n}_{case}_d{d1}_{d2}", case, n, RealSpec(UNIFORMPM1, d_real),
                    IntSpec(INT_UNIFORM, d_int, 0, 15), SEED0 + 2, v)


def caseB_n4096(n: int = 4096) -> Workload:
    """Case B, n=4096: X ~ Poisson(3) clipped to [0,255], kept w.p. 0.3; Y ~ N(0,1) kept w.p. 0.9."""
    return Workload(f"caseB_n{n}", "B", n, RealSpec(NORMAL, 0.9),
                    IntSpec(INT_POISSON, 0.3, 3.0), SEED0 + 3)


def caseA_n16384(n: int = 16384) -> Workload:
    """Case A, n=16384: X ~ U(-1,1) kept w.p. 0.05; Y ~ Geometric(0.3) on {0,1,..} clipped to 255."""
    return Workload(f"caseA_n{n}", "A", n, RealSpec(UNIFORMPM1, 0.05),
                    IntSpec(INT_GEOMETRIC, 1.0, 0.3), SEED0 + 5)


BATCH_R = (3, 15, 63, 255)


def batched_512(count: int = 512, n_lo: int = 32, n_hi: int = 1024):
    """512 products: n log-uniform in [32, 1024], case A/B by coin, d1, d2 ~ U(0.05, 1),
    real ~ U(-1,1), integer ~ U{0..R} with R from {3, 15, 63, 255}."""
    seed = SEED0 + 4
    out = []
    for b in range(count):
        u = lambda f: (draw(seed, S_BATCH_DESC, 8 * b + f) >> 11) * 2.0 ** -53
        n = int(round(math.exp(math.log(n_lo) + u(0) * (math.log(n_hi) - math.log(n_lo)))))
        case = "A" if (draw(seed, S_BATCH_DESC, 8 * b + 1) >> 63) == 0 else "B"
        d1 = 0.05 + 0.95 * u(2)
        d2 = 0.05 + 0.95 * u(3)
        R = BATCH_R[draw(seed, S_BATCH_DESC, 8 * b + 4) >> 62]
        d_real, d_int = (d1, d2) if case == "A" else (d2, d1)
        out.append(Workload(f"batch{b}", case, n, RealSpec(UNIFORMPM1, d_real),
                            IntSpec(INT_UNIFORM, d_int, 0, R), seed, b))
    return out


TABLE1_N = (250, 500, 750, 1000, 1250, 1500, 1750, 2000)
TABLE1_MU = (1, 3, 5, 7, 14, 21)


def table1(n: int, mu: int, y_nonzeros: str) -> Workload:
    """One cell of the paper's Table 1 grid (Section 2.3.1): case A, X ~ U(0,1);
    d1 = 1/3, d2 = 1/2 for mu' <= 7 and d1 = 1/5, d2 = 2/5 for mu' = 14, 21.  The
    distribution of Y's non-zeros is not stated; two readings: 'const' (every
    non-zero equals mu') and 'uniform' (U{1..2 mu' - 1}, mean mu')."""
    d1, d2 = (1 / 3, 1 / 2) if mu <= 7 else (1 / 5, 2 / 5)
    if y_nonzeros == "const":
        ispec = IntSpec(INT_UNIFORM, d2, mu, mu)
    elif y_nonzeros == "uniform":
        ispec = IntSpec(INT_UNIFORM, d2, 1, 2 * mu - 1)
    else:
        raise ValueError(y_nonzeros)
    return Workload(f"table1_n{n}_mu{mu}_{y_nonzeros}", "A", n, RealSpec(UNIFORM01, d1), ispec,
                    SEED0 + 6, 100 * mu + (1 if y_nonzeros == "uniform" else 0))
