"""GPU parity of the strict form over the non-zeros of both factors (mapping 7)
against the CPU oracle.

The form lists the non-zero entries of X's rows and of Y's rows (per band of
columns) and walks, for each row of Z, X's list in ascending k and Y's list of
each such k; it must give the oracle's bits exactly like every other form.  Cases
cover ragged sizes, densities from 1 % to 100 % (Y lists longer than 64 entries),
-0.0 bases, counts of 255 and more and negative counts (no additions), an all-zero
factor, and sampled rows in the low-density regime d1 * d2 = 1/n at n = 4096.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

ROWS = [(7, 1, 64, 8, 1, 16), (7, 1, 32, 16, 1, 16), (7, 1, 16, 16, 1, 16), (7, 1, 16, 8, 1, 16)]


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


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def _inputs(case, n, seed, d_real, d_int, int_lo=0, int_hi=6):
    r = np.random.default_rng(seed)
    real = r.uniform(-1, 1, (n, n)).astype(np.float32)
    real[r.random((n, n)) > d_real] = 0
    real[(real == 0) & (r.random((n, n)) < 0.5)] = -0.0
    ints = r.integers(int_lo, int_hi + 1, (n, n)).astype(np.int32)
    ints[r.random((n, n)) > d_int] = 0
    return (real, ints) if case == "A" else (ints, real)


def _check_all(dev, case, X, Y, configs=ROWS):
    afmm = _afmm()
    Zref, _ = oracle.strict_f32(case, X, Y)
    Xd, Yd = _to(dev, X), _to(dev, Y)
    for cfg in configs:
        assert afmm.config_supported(case, cfg), cfg
        Z = afmm.multiply(case, Xd, Yd, "strict", config=cfg).cpu().numpy()
        d = np.argwhere(_bits(Z) != _bits(Zref))
        if len(d):
            pytest.fail(f"{cfg}: {len(d)} elements differ, first {tuple(d[0])}")


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1, 7, 130, 515, 1100])
def test_rows_sizes_and_densities(dev, case, n):
    for d_real, d_int in ((0.01, 0.05), (0.3, 0.7), (1.0, 1.0)):
        X, Y = _inputs(case, n, 700 + n + int(100 * d_real), d_real, d_int)
        _check_all(dev, case, X, Y)


@pytest.mark.parametrize("case", ["A", "B"])
def test_rows_large_and_negative_counts(dev, case):
    """Counts up to 400 (no byte packing here: the lists hold the int32) and
    negative counts, which add nothing."""
    X, Y = _inputs(case, 260, 77, 0.2, 0.3, int_lo=-50, int_hi=400)
    _check_all(dev, case, X, Y)


@pytest.mark.parametrize("case", ["A", "B"])
def test_rows_zero_factor(dev, case):
    afmm = _afmm()
    for d_real, d_int in ((0.0, 0.5), (0.5, 0.0)):
        X, Y = _inputs(case, 200, 3, d_real, d_int)
        Z = afmm.multiply(case, _to(dev, X), _to(dev, Y), "strict", config=ROWS[0]).cpu().numpy()
        assert (_bits(Z) == 0).all()


@pytest.mark.parametrize("case", ["A", "B"])
def test_rows_quadratic_regime_sampled(dev, case):
    """n = 4096 with both densities 1/64 (d1 * d2 = 1/n): sampled rows bit-exact."""
    n, d = 4096, 1.0 / 64
    real_spec = gen.RealSpec(gen.UNIFORMPM1, d)
    int_spec = gen.IntSpec(gen.INT_UNIFORM, d, 1, 7)
    w = gen.Workload(f"quad_{case}", case, n, real_spec, int_spec, 9100 + (case == "B"))
    X, Y = w.X(), w.Y()
    afmm = _afmm()
    Z = afmm.multiply(case, _to(dev, X), _to(dev, Y), "strict", config=ROWS[0]).cpu().numpy()
    rows = [0, 17, 2048, 4095]
    Zr, _ = oracle.strict_f32(case, X[rows], Y, rows=rows, x_rows_only=True)
    assert np.array_equal(_bits(Z[rows]), _bits(Zr))


@pytest.mark.parametrize("case", ["A", "B"])
def test_suggested_configuration(dev, case):
    """afmm_suggest_config: row lists when d_real * d_int * n <= 32 (case A) or 64
    (case B), compacted bases when only the real factor is very sparse (<= 6 %),
    the size-keyed choice otherwise and below n = 1024; the suggested
    configuration gives the default's bits.  (Positive counts are 6/7 of the
    integer mask here.)"""
    afmm = _afmm()
    n = 2048
    for d_real, d_int, mapping in ((0.1, 0.1, 7), (0.05, 0.9, 4), (0.1, 0.5, None),
                                   (0.9, 0.3, None),
                                   # d_real * d_int * n = 61: compacted bases in case A,
                                   # row lists in case B
                                   (0.05, 0.7, 7 if case == "B" else 4),
                                   # d_real * d_int * n = 37: row lists in case B only
                                   (0.12, 0.175, 7 if case == "B" else None)):
        X, Y = _inputs(case, n, 40 + int(100 * d_real), d_real, d_int)
        Xd, Yd = _to(dev, X), _to(dev, Y)
        cfg = afmm.suggest_config(case, Xd, Yd)
        if mapping is None:
            assert cfg == afmm.default_config(case, n)
        else:
            assert cfg[0] == mapping, (d_real, d_int, cfg)
        Z = afmm.multiply(case, Xd, Yd, config=cfg)
        Zd = afmm.multiply(case, Xd, Yd)
        assert np.array_equal(_bits(Z.cpu().numpy()), _bits(Zd.cpu().numpy()))
    X, Y = _inputs(case, 512, 5, 0.05, 0.05)
    assert afmm.suggest_config(case, _to(dev, X), _to(dev, Y)) == afmm.default_config(case, 512)


# Plain calls choose their form on the device: (d_real, d_int) and the mapping
# the choice must land on ("dense": the size-keyed one).  Positive counts are
# 6/7 of the integer mask with int_lo = 0.
PLAIN_REGIMES = [(0.6, 0.7, "dense"), (0.05, 0.95, 4), (0.03, 0.05, 7)]


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1543, 2085])
@pytest.mark.parametrize("regime", PLAIN_REGIMES, ids=lambda r: str(r[2]))
def test_plain_call_chooses_form_bitexact(dev, case, n, regime):
    """afmm_multiply_caseA / caseB without a configuration, on ragged sizes in
    the three density regimes: the form the device picks (read back through
    afmm_plain_form) is the one the full-density rule names, and the result is
    bit-exact on sampled rows and identical in full to that form run
    explicitly, with a caller workspace of exactly afmm_workspace_size bytes."""
    import torch
    afmm = _afmm()
    d_real, d_int, want = regime
    X, Y = _inputs(case, n, 910 + n + int(100 * d_real), d_real, d_int, int_hi=300)
    Xd, Yd = _to(dev, X), _to(dev, Y)
    form = afmm.plain_form(case, Xd, Yd)
    if want == "dense":
        assert form == afmm.default_config(case, n)[0]
    else:
        assert form == want
    assert afmm.suggest_config(case, Xd, Yd)[0] == form
    ws = torch.empty(afmm.workspace_size(case, n), dtype=torch.uint8, device=dev)
    Z = afmm.multiply(case, Xd, Yd, workspace=ws).cpu().numpy()
    rows = [0, 1, n // 2, n - 1]
    Zr, _ = oracle.strict_f32(case, X[rows], Y, rows=rows, x_rows_only=True)
    assert np.array_equal(_bits(Z[rows]), _bits(Zr))
    Ze = afmm.multiply(case, Xd, Yd, config=afmm.suggest_config(case, Xd, Yd)).cpu().numpy()
    assert np.array_equal(_bits(Z), _bits(Ze))


@pytest.mark.parametrize("case", ["A", "B"])
def test_plain_call_quadratic_regime(dev, case):
    """n = 4096, d1 * d2 = 1/n: the plain call takes the row-list form and its
    sampled rows are bit-exact; a workspace one byte short is refused."""
    import torch
    afmm = _afmm()
    n, d = 4096, 1.0 / 64
    w = gen.Workload(f"quad_{case}", case, n, gen.RealSpec(gen.UNIFORMPM1, d),
                     gen.IntSpec(gen.INT_UNIFORM, d, 1, 7), 9100 + (case == "B"))
    X, Y = w.X(), w.Y()
    Xd, Yd = _to(dev, X), _to(dev, Y)
    assert afmm.plain_form(case, Xd, Yd) == 7
    Z = afmm.multiply(case, Xd, Yd).cpu().numpy()
    rows = [0, 17, 2048, 4095]
    Zr, _ = oracle.strict_f32(case, X[rows], Y, rows=rows, x_rows_only=True)
    assert np.array_equal(_bits(Z[rows]), _bits(Zr))
    short = torch.empty(afmm.workspace_size(case, n) - 1, dtype=torch.uint8, device=dev)
    with pytest.raises(afmm.AfmmError):
        afmm.multiply(case, Xd, Yd, workspace=short)


def test_plain_call_small_keeps_size_keyed_form(dev):
    """Below n = 1024 the plain call keeps the size-keyed form whatever the density."""
    afmm = _afmm()
    for case in "AB":
        X, Y = _inputs(case, 700, 4, 0.02, 0.02)
        assert afmm.plain_form(case, _to(dev, X), _to(dev, Y)) == afmm.default_config(case, 700)[0]
