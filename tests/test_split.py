"""GPU split-BF16x3 MFMA form against the binary64 true product (tolerance 1e-6 rel. Frobenius)."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
TOL = 1e-6  # relative Frobenius error bound required of the split form


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2400_amd  # noqa: F401
    return torch.device("cuda:0")


def _to(dev, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _split(dev, case, X, Y):
    import paper_1308_2400_amd as afmm
    return afmm.multiply(case, _to(dev, X), _to(dev, Y), "split").cpu().numpy()


def _rand_case(case, n, seed, int_hi=9, dens=0.6):
    r = np.random.default_rng(seed)
    real = r.standard_normal((n, n)).astype(np.float32)
    real[r.random((n, n)) > dens] = 0
    ints = r.integers(0, int_hi + 1, (n, n)).astype(np.int32)
    return (real, ints) if case == "A" else (ints, real)


@pytest.mark.parametrize("case", ["A", "B"])
# edges of the GEMM's block tile: 64 rows of the term planes, 256 of the integer plane
@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 517])
def test_split_small_sizes(dev, case, n):
    X, Y = _rand_case(case, n, 200 + n)
    Z = _split(dev, case, X, Y)
    Z64 = oracle.product_f64(case, X, Y)
    assert oracle.rel_frobenius(Z, Z64) <= TOL
    # every element, not just the norm: |err| <= 1e-6 * (|X| |Y|)[i,j] (+ tiny absolute slack)
    scale = np.abs(X).astype(np.float64) @ np.abs(Y).astype(np.float64)
    assert np.all(np.abs(Z - Z64) <= TOL * scale + 1e-30)


def test_split_integer_valued_is_exact(dev):
    """Small integers in both factors: every term and partial sum is exact."""
    r = np.random.default_rng(4)
    n = 256
    X = r.integers(-50, 50, (n, n)).astype(np.float32)
    Y = r.integers(0, 200, (n, n)).astype(np.int32)
    Z = _split(dev, "A", X, Y)
    assert np.array_equal(Z, (X.astype(np.int64) @ Y.astype(np.int64)).astype(np.float32))


def test_split_identity(dev):
    r = np.random.default_rng(2)
    Y = r.standard_normal((130, 130)).astype(np.float32)
    Z = _split(dev, "B", np.eye(130, dtype=np.int32), Y)
    assert np.array_equal(Z, Y)


def test_split_caseB_n4096_full(dev):
    w = gen.caseB_n4096()
    X, Y = w.X(), w.Y()
    Z = _split(dev, "B", X, Y)
    Z64 = oracle.product_f64_blas(X, Y)
    err = oracle.rel_frobenius(Z, Z64)
    print(f"split caseB n=4096 rel Frobenius error {err:.3e}")
    assert err <= TOL
    rows = [0, 1234, 4095]
    assert np.allclose(oracle.product_f64("B", X[rows], Y, rows=rows, x_rows_only=True), Z64[rows],
                       rtol=1e-12, atol=1e-9)


def test_split_caseA_n16384_sampled(dev):
    w = gen.caseA_n16384()
    X, Y = w.X(), w.Y()
    Z = _split(dev, "A", X, Y)
    rows = [17 + 256 * t for t in range(0, 64, 4)]
    Z64 = oracle.product_f64("A", X[rows], Y, rows=rows, x_rows_only=True)
    err = oracle.rel_frobenius(Z[rows], Z64)
    print(f"split caseA n=16384 sampled rel Frobenius error {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("case", ["A", "B"])
def test_split_vs_strict_same_ballpark(dev, case):
    import paper_1308_2400_amd as afmm
    w = gen.sweep_n2048(case, 0.5, 0.5, n=700)
    X, Y = w.X(), w.Y()
    Xd, Yd = _to(dev, X), _to(dev, Y)
    Zs = afmm.multiply(case, Xd, Yd, "strict").cpu().numpy()
    Zm = afmm.multiply(case, Xd, Yd, "split").cpu().numpy()
    Z64 = oracle.product_f64(case, X, Y)
    assert oracle.rel_frobenius(Zm, Z64) <= TOL
    assert oracle.rel_frobenius(Zs, Z64) < 1e-5


def _golden_split_values():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "split_bf16x3.json")
    with open(path) as f:
        return [np.float32(float.fromhex(c["x"])) for c in json.load(f)["cases"]]


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1, 7, 67, 200])
def test_split_terms_match_oracle_bitwise(dev, case, n):
    """The GPU conversion pass gives the oracle's hi/mid/lo patterns for every
    real entry (hand-worked rounding cases planted among normal, tiny and zero
    values) and the exact bfloat16 of every integer entry (<= 0 becomes +0)."""
    import ctypes
    import torch
    import paper_1308_2400_amd as afmm
    r = np.random.default_rng(900 + n)
    real = r.standard_normal((n, n)).astype(np.float32)
    flat = real.reshape(-1)
    gold = _golden_split_values()
    for t, v in enumerate(gold):
        if t < flat.size:
            flat[(t * 37) % flat.size] = v
    flat[r.random(flat.size) < 0.2] = 0.0
    flat[r.random(flat.size) < 0.1] *= np.float32(2.0 ** -60)
    ints = r.integers(-3, 257, (n, n)).astype(np.int32)
    X, Y = (real, ints) if case == "A" else (ints, real)
    Xd, Yd = _to(dev, X), _to(dev, Y)
    terms = torch.empty((3, n, n), dtype=torch.int16, device=dev)
    ibf = torch.empty((n, n), dtype=torch.int16, device=dev)
    st = afmm.afmm_split_terms(0 if case == "A" else 1, n, Xd.data_ptr(), Yd.data_ptr(),
                               terms.data_ptr(), ibf.data_ptr(), None, 0,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    got = terms.cpu().numpy().view(np.uint16)
    hi, mid, lo = oracle.split_bf16x3(real)
    assert np.array_equal(got[0], hi)
    assert np.array_equal(got[1], mid)
    assert np.array_equal(got[2], lo)
    # integers: exact in bfloat16 up to 256 (an integer below 2^8 has at most 8
    # significant bits; 256 is a power of two), counts <= 0 contribute nothing
    want = (np.maximum(ints, 0).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(ibf.cpu().numpy().view(np.uint16), want)
