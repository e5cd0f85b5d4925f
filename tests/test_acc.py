"""GPU parity of the compacted-base strict form (mapping 4) against the CPU oracle.

The form lists each k's non-zero bases per band of lane columns and keeps the Z
block in LDS; it must give the oracle's bits exactly like every other form.  Cases
cover ragged sizes, real-factor densities from 2 % (C5-like) to 100 % (segments
longer than 64 entries per lane slot set, walked in several chunks; lanes with
one, two and four slots), bases piled into few residues modulo 64 of the lane
axis (slots handed between lanes), -0.0 bases (skipped like +0.0),
counts of 255 and more (escape path), an all-zero real factor, and sampled rows of
the n=16384 case-A workload.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

ACC = [(4, 4, 16, 8, 1, 16), (4, 4, 16, 8, 2, 16), (4, 4, 16, 8, 4, 16), (4, 2, 16, 16, 1, 16),
       (4, 2, 16, 16, 2, 16), (4, 2, 16, 16, 4, 16), (4, 4, 8, 16, 1, 16), (4, 8, 8, 8, 1, 16),
       (4, 4, 4, 8, 1, 16),
       # two and four entries per lane (bands of 2048 and 4096 columns, 8-k panels)
       (4, 2, 32, 8, 2, 8), (4, 1, 32, 16, 2, 8), (4, 1, 64, 8, 2, 8), (4, 1, 64, 8, 1, 8),
       # 16-k panels, several blocks per CU; waves of one, two and four rows
       (4, 2, 32, 8, 1, 16), (4, 1, 16, 16, 1, 16), (4, 2, 16, 8, 1, 16), (4, 1, 16, 8, 1, 8),
       (4, 1, 16, 16, 1, 8), (4, 1, 32, 8, 1, 8), (4, 2, 16, 8, 1, 8), (4, 1, 16, 8, 1, 16),
       (4, 4, 16, 4, 1, 16), (4, 4, 16, 4, 1, 8), (4, 4, 32, 4, 1, 8)]


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


def _inputs(case, n, seed, d_real, int_hi=6, d_int=0.7):
    r = np.random.default_rng(seed)
    real = r.uniform(-1, 1, (n, n)).astype(np.float32)
    real[r.random((n, n)) > d_real] = 0
    real[(real == 0) & (r.random((n, n)) < 0.5)] = -0.0  # a zero base of either sign
    ints = r.integers(0, int_hi + 1, (n, n)).astype(np.int32)
    ints[r.random((n, n)) > d_int] = 0
    return (real, ints) if case == "A" else (ints, real)


def _check_all(dev, case, X, Y, configs=ACC):
    afmm = _afmm()
    Zref, _ = oracle.strict_f32(case, X, Y)
    Xd, Yd = _to(dev, X), _to(dev, Y)
    for cfg in configs:
        assert afmm.config_supported(case, cfg), cfg
        Z = afmm.multiply(case, Xd, Yd, "strict", config=cfg).cpu().numpy()
        same = np.array_equal(_bits(Z), _bits(Zref))
        if not same:
            d = np.argwhere(_bits(Z) != _bits(Zref))
            pytest.fail(f"{cfg}: {len(d)} elements differ, first {tuple(d[0])}")


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("n", [1, 7, 130, 515, 1100])
def test_acc_sizes_and_densities(dev, case, n):
    for d_real in (0.02, 0.3, 1.0):
        X, Y = _inputs(case, n, 900 + n + int(100 * d_real), d_real)
        _check_all(dev, case, X, Y)


@pytest.mark.parametrize("case", ["A", "B"])
@pytest.mark.parametrize("pattern", ["one_residue", "two_residues", "clustered", "bank_pair",
                                     "lower_full", "upper_full"])
def test_acc_uneven_bank_classes(dev, case, pattern):
    """Non-zero bases piled into few residues modulo 64 of the lane axis (i in
    case A, j in case B): the slots of a k take each lane's own columns first,
    hand the rest to the free slots of the lane 32 away (same LDS bank, other
    half-wave), then to other lanes' free slots alternating between the
    half-waves, passing the excess of a full half-wave to the other one; every
    base must still be added exactly once per k.  bank_pair fills both lanes of
    one bank; lower_full and upper_full leave one half-wave no free slot while
    entries are bound for it."""
    n = 700
    X, Y = _inputs(case, n, 404 + len(pattern), 1.0)
    real = X if case == "A" else Y
    idx = np.arange(n)
    if pattern == "one_residue":
        keep = idx % 64 == 5
    elif pattern == "two_residues":
        keep = (idx % 64 == 5) | (idx % 64 == 40)
    elif pattern == "bank_pair":
        keep = (idx % 64 == 5) | (idx % 64 == 37)
    elif pattern == "lower_full":
        keep = idx % 64 < 48  # lanes 0-47 overflow, lanes 48-63 have free slots
    elif pattern == "upper_full":
        keep = idx % 64 >= 16  # lanes 16-63 overflow, lanes 0-15 have free slots
    else:
        keep = (idx >= 100) & (idx < 100 + 150)  # one run: every residue, two or three each
    if case == "A":
        real[~keep, :] = 0  # lanes run over the rows of X
    else:
        real[:, ~keep] = 0  # lanes run over the columns of Y
    _check_all(dev, case, X, Y)


@pytest.mark.parametrize("case", ["A", "B"])
def test_acc_escape_counts(dev, case):
    """Counts of 255 and more re-read from the int32 factor."""
    n = 200
    X, Y = _inputs(case, n, 31, 0.1)
    ints = Y if case == "A" else X
    r = np.random.default_rng(5)
    ints[:] = r.integers(200, 400, ints.shape)
    ints[r.random(ints.shape) < 0.6] = 0
    _check_all(dev, case, X, Y)


@pytest.mark.parametrize("case", ["A", "B"])
def test_acc_zero_real_factor(dev, case):
    n = 300
    X, Y = _inputs(case, n, 8, 0.0)
    afmm = _afmm()
    for cfg in ACC[:2]:
        Z = afmm.multiply(case, _to(dev, X), _to(dev, Y), "strict", config=cfg).cpu().numpy()
        assert (_bits(Z) == 0).all()  # +0.0 everywhere


def test_acc_caseA_n16384_sampled(dev):
    """The n=16384 case-A workload (real factor 5 % dense) on sampled rows."""
    w = gen.caseA_n16384()
    X, Y = w.X(), w.Y()
    rows = [17, 16383]
    afmm = _afmm()
    Z = afmm.multiply("A", _to(dev, X), _to(dev, Y), "strict", config=ACC[0]).cpu().numpy()
    Zref, _ = oracle.strict_f32("A", X[rows], Y, rows=rows, x_rows_only=True)
    assert np.array_equal(_bits(Z[rows]), _bits(Zref))
