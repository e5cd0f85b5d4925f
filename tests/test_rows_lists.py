"""The row-list form's list builder, read back through afmm_row_lists and compared
with its definition: for every band of `band` columns and every row, the entries
that take part in an addition (a count > 0; a base != 0, so -0.0 is dropped and
NaN kept), as {value bits, column in the band}, in ascending column, and their
number.  Ragged bands (widths not a multiple of 64, a partial last band), a band
wider than the matrix, counts <= 0 and above 255, +-0.0, NaN and infinities."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    import paper_1308_2400_amd  # noqa: F401  (fails loudly when libafmm.so is missing)
    return torch.device("cuda:0")


def _gpu_lists(dev, M, band):
    import torch
    import paper_1308_2400_amd as afmm
    rows, cols = M.shape
    bands = -(-cols // band)
    Md = torch.from_numpy(np.ascontiguousarray(M)).to(dev)
    ent = torch.zeros((bands, rows, band, 2), dtype=torch.int32, device=dev)
    lens = torch.full((bands, rows), -1, dtype=torch.int32, device=dev)
    is_int = 1 if M.dtype == np.int32 else 0
    st = afmm.afmm_row_lists(is_int, Md.data_ptr(), rows, cols, cols, band, ent.data_ptr(),
                             lens.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    torch.cuda.synchronize()
    return ent.cpu().numpy().view(np.uint32), lens.cpu().numpy()


def _check(dev, M, band):
    ent, lens = _gpu_lists(dev, M, band)
    bits = np.ascontiguousarray(M).view(np.uint32)
    if M.dtype == np.int32:
        take = M > 0
    else:
        take = ~(M == 0)  # NaN compares unequal to zero: kept
    rows, cols = M.shape
    for b in range(ent.shape[0]):
        c0 = b * band
        for r in range(rows):
            cs = np.nonzero(take[r, c0:c0 + band])[0]
            assert lens[b, r] == len(cs), (b, r)
            got = ent[b, r, :len(cs)]
            assert np.array_equal(got[:, 1], cs.astype(np.uint32)), (b, r)
            assert np.array_equal(got[:, 0], bits[r, c0 + cs]), (b, r)


def _ints(rows, cols, d, seed):
    r = np.random.default_rng(seed)
    M = r.integers(-3, 300, (rows, cols)).astype(np.int32)
    M[r.random((rows, cols)) > d] = 0
    return M


def _reals(rows, cols, d, seed):
    r = np.random.default_rng(seed)
    M = r.uniform(-1, 1, (rows, cols)).astype(np.float32)
    M[r.random((rows, cols)) > d] = 0
    M[(M == 0) & (r.random((rows, cols)) < 0.5)] = -0.0
    M[r.random((rows, cols)) < 0.01] = np.nan
    M[r.random((rows, cols)) < 0.01] = np.inf
    return M


@pytest.mark.parametrize("band", [64, 100, 256, 2048, 4096])
@pytest.mark.parametrize("d", [0.02, 0.3, 1.0])
def test_row_lists_counts(dev, band, d):
    _check(dev, _ints(37, 2500, d, 5 + band + int(100 * d)), band)


@pytest.mark.parametrize("band", [64, 100, 256, 2048, 4096])
@pytest.mark.parametrize("d", [0.02, 0.3, 1.0])
def test_row_lists_bases(dev, band, d):
    _check(dev, _reals(37, 2500, d, 7 + band + int(100 * d)), band)


def test_row_lists_rejects_bad_arguments(dev):
    import torch
    import paper_1308_2400_amd as afmm
    M = torch.zeros((4, 64), dtype=torch.int32, device=dev)
    e = torch.zeros(4 * 64 * 2, dtype=torch.int32, device=dev)
    ln = torch.zeros(4, dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    for is_int, rows, cols, ld, band in [(2, 4, 64, 64, 64), (1, 0, 64, 64, 64), (1, 4, 0, 64, 64),
                                         (1, 4, 64, 63, 64), (1, 4, 64, 64, 0)]:
        assert afmm.afmm_row_lists(is_int, M.data_ptr(), rows, cols, ld, band, e.data_ptr(),
                                   ln.data_ptr(), s) == 1
