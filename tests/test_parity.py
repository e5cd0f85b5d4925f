"""GPU parity of the strict path and the add count against the CPU oracle.

Strict results must be bit-identical to the oracle's binary32 loop in the paper's
(i, k, j, p) order; counts must be equal.  Sizes span several tiles with ragged
tails; the full-size workloads are checked on sampled rows the oracle computes
one by one.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    import paper_1308_2400_amd  # noqa: F401  (fails loudly when libafmm.so is missing)
    return torch.device("cuda:0")


def _afmm():
    import paper_1308_2400_amd
    return paper_1308_2400_amd


def _to(dev, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _bits_equal(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


def _first_diff(a, b):
    d = np.argwhere(np.asarray(a).view(np.uint32) != np.asarray(b).view(np.uint32))
    return None if d.size == 0 else (tuple(d[0]), a[tuple(d[0])], b[tuple(d[0])], len(d))


def _rand_case(case, n, seed, int_hi=9, d_real=0.6, d_int=0.7, normal=True):
    r = np.random.default_rng(seed)
    real = (r.standard_normal((n, n)) if normal else r.uniform(-1, 1, (n, n))).astype(np.float32)
    real[r.random((n, n)) > d_real] = 0
    ints = r.integers(0, int_hi + 1, (n, n)).astype(np.int32)
    ints[r.random((n, n)) > d_int] = 0
    return (real, ints) if case == "A" else (ints, real)


def _check_strict(dev, case, X, Y, config=None, rows=None):
    afmm = _afmm()
    Z = afmm.multiply(case, _to(dev, X), _to(dev, Y), "strict", config=config).cpu().numpy()
    if rows is None:
        Zref, _ = oracle.strict_f32(case, X, Y)
        got = Z
    else:
        Zref, _ = oracle.strict_f32(case, X[rows], Y, rows=rows, x_rows_only=True)
        got = Z[rows]
    assert _bits_equal(got, Zref), _first_diff(got, Zref)
    return Z


# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 63, 64, 65, 127, 200, 333, 517])
def test_strict_bitexact_sizes(dev, case, n):
    X, Y = _rand_case(case, n, 1000 + n)
    _check_strict(dev, case, X, Y)


CONFIGS = [(0, 8, 8, 8), (0, 8, 8, 8, 2), (0, 4, 8, 8), (0, 8, 4, 8), (0, 8, 4, 8, 2), (0, 4, 4, 8),
           (0, 8, 8, 4), (0, 8, 4, 4), (0, 8, 4, 4, 2), (0, 4, 2, 4, 2),
           (0, 4, 4, 4), (0, 4, 2, 4), (0, 2, 1, 4), (0, 4, 16, 8, 1, 8), (0, 4, 16, 8, 2, 8),
           (0, 6, 16, 4, 1, 8), (0, 8, 8, 8, 2, 8), (0, 4, 16, 16, 1, 16), (0, 4, 16, 16, 2, 16),
           (2, 8, 8, 4), (2, 4, 8, 8), (2, 16, 4, 4),
           (3, 2, 16, 16, 1, 8), (3, 2, 16, 16, 2, 8), (3, 4, 8, 16, 1, 16), (3, 4, 8, 16, 2, 16),
           (3, 2, 8, 16, 2, 16), (3, 2, 16, 8, 1, 4), (3, 2, 16, 8, 2, 4), (3, 1, 16, 16, 1, 8),
           (4, 4, 16, 8, 1, 16), (4, 4, 16, 8, 2, 16), (4, 2, 16, 16, 1, 16), (4, 4, 8, 16, 1, 16),
           (4, 8, 8, 8, 1, 16), (4, 4, 4, 8, 1, 16), (4, 2, 32, 8, 2, 8), (4, 1, 64, 8, 2, 8),
           (7, 1, 64, 8, 1, 16), (7, 1, 16, 16, 1, 16)]
SPARSE = [c for c in CONFIGS if c[0] == 3]


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("cfg", CONFIGS, ids=str)
def test_strict_bitexact_every_config(dev, case, cfg):
    n = 601  # ragged against every tile shape
    X, Y = _rand_case(case, n, 77, int_hi=5, d_real=0.5)
    if not _afmm().config_supported(case, cfg):
        pytest.skip("configuration not compiled")
    _check_strict(dev, case, X, Y, config=cfg)


def test_caseA_n256_full(dev):
    w = gen.caseA_n256()
    _check_strict(dev, "A", w.X(), w.Y())


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [130, 257, 1000])
def test_direct_variant_sizes(dev, case, n):
    """The direct-load variant; n % 4 != 0 in case B falls back to the LDS variant."""
    X, Y = _rand_case(case, n, 300 + n, int_hi=6)
    for cfg in [(2, 8, 8, 4), (2, 16, 4, 4)]:
        _check_strict(dev, case, X, Y, config=cfg)


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1, 7, 130, 515, 1000, 1100])
def test_sparse_variant_sizes(dev, case, n):
    """The sparse-k variant (k with all-zero counts skipped per wave) over ragged sizes,
    dense and very sparse counts; case B with n % 4 != 0 falls back to the LDS variant."""
    for d_int in (0.9, 0.05):
        X, Y = _rand_case(case, n, 500 + n, int_hi=6, d_int=d_int)
        for cfg in SPARSE:
            _check_strict(dev, case, X, Y, config=cfg)


@pytest.mark.parametrize("case", ["A", "B"])
def test_counts_with_top_bit_set(dev, case):
    """Count bytes 128..254 (no escape) in every k position: the packed count words
    then have their top bit set, which must not leak into neighbouring counts when
    the words are widened on the device (regression: sign extension)."""
    n = 72
    r = np.random.default_rng(11)
    X, Y = _rand_case(case, n, 12, int_hi=2)
    ints = X if case == "B" else Y
    ints[:] = r.integers(128, 255, ints.shape)
    ints[r.random(ints.shape) < 0.5] = 0
    for cfg in [(0, 4, 16, 16, 1, 16), (0, 4, 16, 16, 2, 16), (2, 8, 8, 4), (4, 4, 16, 8, 1, 16),
                (4, 4, 4, 8, 1, 16)] + SPARSE:
        _check_strict(dev, case, X, Y, config=cfg)


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("cfg", [(0, 8, 8, 8), (2, 8, 8, 4), (3, 2, 16, 16, 1, 8),
                                 (3, 4, 8, 16, 2, 16)], ids=str)
def test_strict_large_counts_escape(dev, case, cfg):
    """Counts at and above 255 take the escape path (full int32 re-read)."""
    n = 150
    r = np.random.default_rng(5)
    X, Y = _rand_case(case, n, 6, int_hi=3)
    ints = X if case == "B" else Y
    pos = r.random((n, n)) < 0.01
    ints[pos] = r.integers(250, 700, pos.sum())
    ints[0, 0] = 255
    ints[1, 1] = 254
    _check_strict(dev, case, X, Y, config=cfg)


@pytest.mark.parametrize("case", ["A", "B"])
def test_strict_negative_counts_add_nothing(dev, case):
    X, Y = _rand_case(case, 130, 8)
    ints = X if case == "B" else Y
    ints[::3, ::2] = -ints[::3, ::2] - 1
    _check_strict(dev, case, X, Y)


@pytest.mark.parametrize("case", ["A", "B"])
def test_strict_denormals_and_signed_zeros(dev, case):
    """Denormals are kept on both sides; -0.0 bases are skipped like +0.0."""
    n = 96
    X, Y = _rand_case(case, n, 9)
    real = X if case == "A" else Y
    r = np.random.default_rng(3)
    m = r.random((n, n)) < 0.2
    real[m] = (r.standard_normal(m.sum()) * 1e-39).astype(np.float32)  # subnormal binary32
    real[r.random((n, n)) < 0.05] = np.float32(-0.0)
    assert (np.abs(real[m]) < np.finfo(np.float32).tiny).any()
    Z = _check_strict(dev, case, X, Y)
    assert not (np.signbit(Z) & (Z == 0)).any()  # Z is never -0.0


def test_identity(dev):
    w = gen.caseA_n256()
    X = w.X()
    Z = _check_strict(dev, "A", X, np.eye(256, dtype=np.int32))
    assert _bits_equal(Z, X)
    r = np.random.default_rng(1)
    Y = r.standard_normal((200, 200)).astype(np.float32)
    Z = _check_strict(dev, "B", np.eye(200, dtype=np.int32), Y)
    assert _bits_equal(Z, Y)


@pytest.mark.parametrize("case", ["A", "B"])
def test_zero_density(dev, case):
    X, Y = _rand_case(case, 70, 4)
    X = np.zeros_like(X)
    Z = _check_strict(dev, case, X, Y)
    assert not Z.view(np.uint32).any()


# --------------------------------------------------------------------------
# Full-size workloads on sampled rows

def _sample_rows(n, k=12, seed=0):
    r = np.random.default_rng(seed)
    rows = sorted(set([0, n - 1, n // 2] + list(r.choice(n, k, replace=False))))
    return rows


def test_caseB_n4096_sampled(dev):
    w = gen.caseB_n4096()
    X, Y = w.X(), w.Y()
    _check_strict(dev, "B", X, Y, rows=_sample_rows(4096, 16))


@pytest.fixture(scope="module")
def c3_full():
    """The whole n=4096 case-B workload and the oracle's result for all of it
    (the oracle over disjoint row ranges on the host's threads)."""
    w = gen.caseB_n4096()
    X, Y = w.X(), w.Y()
    Zref, adds = oracle.strict_f32_threaded("B", X, Y)
    return X, Y, Zref, adds


@pytest.mark.parametrize("cfg", [None, (3, 2, 16, 16, 2, 8), (0, 4, 16, 16, 1, 16)], ids=str)
def test_caseB_n4096_full_matrix(dev, c3_full, cfg):
    """Every element of the n=4096 case-B product, bit for bit, in the library's
    default configuration (the benchmark's launch) and two others."""
    X, Y, Zref, adds = c3_full
    afmm = _afmm()
    Z = afmm.multiply("B", _to(dev, X), _to(dev, Y), "strict", config=cfg).cpu().numpy()
    assert _bits_equal(Z, Zref), _first_diff(Z, Zref)
    if cfg is None:
        assert afmm.count_adds("B", _to(dev, X), _to(dev, Y)) == adds


@pytest.mark.parametrize("cfg", SPARSE, ids=str)
def test_caseB_n4096_sampled_sparse(dev, cfg):
    w = gen.caseB_n4096()
    X, Y = w.X(), w.Y()
    _check_strict(dev, "B", X, Y, config=cfg, rows=_sample_rows(4096, 8, seed=cfg[1] + cfg[4]))


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("d1", gen.SWEEP_D)
@pytest.mark.parametrize("d2", gen.SWEEP_D)
def test_sweep_n2048_sampled_and_count(dev, case, d1, d2):
    w = gen.sweep_n2048(case, d1, d2)
    X, Y = w.X(), w.Y()
    _check_strict(dev, case, X, Y, rows=_sample_rows(2048, 6, seed=int(d1 * 10 + d2)))
    afmm = _afmm()
    total, rows = afmm.count_adds(case, _to(dev, X), _to(dev, Y), rows=True)
    ot, orows, _ = oracle.count(case, X, Y)
    assert total == ot
    assert np.array_equal(rows.cpu().numpy(), orows)


def test_caseA_n16384_sampled(dev):
    w = gen.caseA_n16384()
    X, Y = w.X(), w.Y()
    rows = [17 + 256 * t for t in range(0, 64, 8)] + [0, 16383]
    _check_strict(dev, "A", X, Y, rows=rows)
    _check_strict(dev, "A", X, Y, config=(3, 2, 16, 16, 1, 8), rows=rows[:4])


# --------------------------------------------------------------------------
# Counting and validation

@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1, 5, 300, 1000])
def test_count_matches_oracle(dev, case, n):
    X, Y = _rand_case(case, n, 50 + n, int_hi=20)
    afmm = _afmm()
    total, rows, flags = afmm.count_adds(case, _to(dev, X), _to(dev, Y), rows=True,
                                          with_flags=True)
    ot, orows, oflags = oracle.count(case, X, Y)
    assert total == ot and np.array_equal(rows.cpu().numpy(), orows) and flags == oflags


def test_count_flags_and_validate(dev):
    afmm = _afmm()
    X, Y = _rand_case("B", 64, 3)
    Xd, Yd = _to(dev, X), _to(dev, Y)
    assert afmm.validate("B", Xd, Yd, "strict") == 0
    assert afmm.validate("B", Xd, Yd, "split") == 0
    X2 = X.copy()
    X2[3, 4] = 300
    assert afmm.validate("B", _to(dev, X2), Yd, "strict") == 0
    assert afmm.validate("B", _to(dev, X2), Yd, "split") == 4
    X2[5, 6] = -1
    assert afmm.validate("B", _to(dev, X2), Yd, "strict") == 3
    _, fl = afmm.count_adds("B", _to(dev, X2), Yd, with_flags=True)
    assert fl == oracle.count("B", X2, Y)[2]


def test_count_overflow_saturates(dev):
    afmm = _afmm()
    n = 4096
    X = np.full((n, n), 2 ** 31 - 1, np.int32)
    Y = np.ones((n, n), np.float32)
    total, fl = afmm.count_adds("B", _to(dev, X), _to(dev, Y), with_flags=True)
    assert total == 2 ** 64 - 1 and fl & afmm.FLAG_OVERFLOW
    assert afmm.validate("B", _to(dev, X), _to(dev, Y)) == 5


def test_caseB_n4096_count_statistics(dev):
    w = gen.caseB_n4096()
    X, Y = w.X(), w.Y()
    total = _afmm().count_adds("B", _to(dev, X), _to(dev, Y))
    assert total == oracle.count("B", X, Y)[0]
    assert abs(total / w.expected_adds() - 1) < 0.01


def test_workspace_caller_and_stream_ordered(dev):
    """Caller workspace, library-allocated workspace and an explicit stream agree."""
    import torch
    afmm = _afmm()
    X, Y = _rand_case("B", 300, 12)
    Xd, Yd = _to(dev, X), _to(dev, Y)
    Z1 = afmm.multiply("B", Xd, Yd)
    Z2 = torch.empty_like(Z1)
    st = afmm.afmm_multiply_caseB(300, Xd.data_ptr(), Yd.data_ptr(), Z2.data_ptr(), 0, None, 0,
                                  None)
    assert st == 0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Z3 = afmm.multiply("B", Xd, Yd)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(Z1, Z2) and torch.equal(Z1, Z3)
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(afmm.AfmmError):
        afmm.multiply("B", Xd, Yd, workspace=small)


def test_concurrent_streams(dev):
    """Products queued alternately on two streams (default-priority, each with its own
    workspace) run concurrently; every result equals the oracle's bits, and the split
    form's results equal a run on its own."""
    import torch
    afmm = _afmm()
    cases = [("B", 700, 41), ("A", 520, 42), ("B", 333, 43), ("A", 901, 44)]
    host = [(c, *_rand_case(c, n, seed, int_hi=12)) for c, n, seed in cases]
    dev_in = [(c, _to(dev, X), _to(dev, Y)) for c, X, Y in host]
    alone = [afmm.multiply(c, Xd, Yd, mode="split_bf16x3") for c, Xd, Yd in dev_in]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for i, (c, Xd, Yd) in enumerate(dev_in):
        s = streams[i % 2]
        with torch.cuda.stream(s):
            n = Xd.shape[0]
            ws = torch.empty(afmm.workspace_size(c, n), dtype=torch.uint8, device=dev)
            split_ws = torch.empty(afmm.workspace_size(c, n, "split_bf16x3"), dtype=torch.uint8,
                                   device=dev)
            outs.append((afmm.multiply(c, Xd, Yd, workspace=ws),
                         afmm.multiply(c, Xd, Yd, mode="split_bf16x3", workspace=split_ws),
                         ws, split_ws))
    for s in streams:
        s.synchronize()
    for (c, X, Y), (Z, Zs, _, _), Za in zip(host, outs, alone):
        Zref, _ = oracle.strict_f32(c, X, Y)
        assert _bits_equal(Z.cpu().numpy(), Zref), c
        assert torch.equal(Zs, Za)
