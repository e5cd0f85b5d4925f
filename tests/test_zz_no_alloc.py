"""The allocation-free strict entry point against the allocating one, through
the C ABI: bit-identical results on two calls in a row (the second smaller),
both cases, and the size limit refused on the host."""
import ctypes

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def afmm():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2400_amd
    return paper_1308_2400_amd


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pair(afmm, case, X, Y):
    """(noalloc result, allocating-call result) as uint32 bit patterns."""
    import torch
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).to(dev)
    n = X.shape[0]
    c = 0 if case == "A" else 1
    Z1 = torch.full((n, n), float("nan"), dtype=torch.float32, device=dev)
    Z2 = torch.full((n, n), float("nan"), dtype=torch.float32, device=dev)
    st = afmm.afmm_multiply_noalloc(c, n, Xd.data_ptr(), Yd.data_ptr(), Z1.data_ptr(), _stream())
    assert st == 0, afmm.STATUS.get(st)
    f = afmm.afmm_multiply_caseA if case == "A" else afmm.afmm_multiply_caseB
    st = f(n, Xd.data_ptr(), Yd.data_ptr(), Z2.data_ptr(), 0, None, 0, _stream())
    assert st == 0, afmm.STATUS.get(st)
    torch.cuda.synchronize()
    return Z1.cpu().numpy().view(np.uint32), Z2.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("case", ["A", "B"])
def test_noalloc_matches_allocating_call_twice(afmm, case):
    # first call: a large product with escaped counts (>= 255); second: smaller,
    # so stale scratch contents from the first call would show
    for n, seed, hi in ((1500, 1, 300), (333, 2, 9)):
        r = np.random.default_rng(seed)
        real = r.standard_normal((n, n)).astype(np.float32)
        real[r.random((n, n)) < 0.3] = 0
        ints = r.integers(0, hi + 1, (n, n)).astype(np.int32)
        ints[r.random((n, n)) < 0.5] = 0
        X, Y = (real, ints) if case == "A" else (ints, real)
        a, b = _pair(afmm, case, X, Y)
        assert np.array_equal(a, b), (case, n)


def test_noalloc_c3_workload(afmm):
    w = gen.caseB_n4096()
    a, b = _pair(afmm, "B", w.X(), w.Y())
    assert np.array_equal(a, b)


def test_noalloc_refuses_oversize(afmm):
    """A product whose workspace exceeds the fixed array is refused before any
    launch (no device memory is touched: the pointers are never read)."""
    import torch
    n = 16384
    c = 1
    need = afmm.afmm_workspace_size(c, n, 0)
    assert need > (96 << 20)
    # distinct fake device addresses: the call must return before using them
    base = 1 << 40
    st = afmm.afmm_multiply_noalloc(c, n, base, base + (4 << 30), base + (8 << 30), _stream())
    assert st == 9  # AFMM_ERR_WORKSPACE
    torch.cuda.synchronize()
