"""The compacted-base form's list builder, read back through afmm_base_lists and
compared slot for slot with a host model of its placement rule.

For every band of CT = 64*C columns and every k the builder lists the band's
non-zero bases of row k (-0.0 is zero, NaN is not) as {base bits, 4*column}.
Lane l owns the columns c = l (mod 64): its own come first (ascending), then
the surplus of the lane 32 away (same LDS bank, other half-wave), then other
lanes' surplus, dealt alternately to the other and to the own half-wave in lane
order, a full half-wave passing its excess to the other; the rest of the slots
are sinks {+0.0, 4*(CT + l)}.  The length is ceil(nnz/64) rounded up to a
multiple of E = max(1, C/16), times 64.  Besides equality with the model the
tests check the invariants the kernel relies on: each non-zero base exactly
once per k, lengths as stated, and a lane's own, received-from-partner and
sink slots all in the lane's LDS bank.
"""
import numpy as np
import pytest

from acc_lists_model import model_segment

pytestmark = pytest.mark.gpu

KPAD = 16


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    import paper_1308_2400_amd  # noqa: F401  (fails loudly when libafmm.so is missing)
    return torch.device("cuda:0")


def _gpu_lists(dev, Q, C):
    import torch
    import paper_1308_2400_amd as afmm
    k, n_c = Q.shape
    ct = 64 * C
    bands, kp = -(-n_c // ct), -(-k // KPAD) * KPAD
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).to(dev)
    ent = torch.zeros((bands, kp, ct, 2), dtype=torch.int32, device=dev)
    lens = torch.full((bands, kp), -1, dtype=torch.int32, device=dev)
    st = afmm.afmm_base_lists(Qd.data_ptr(), k, n_c, n_c, C, ent.data_ptr(), lens.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    torch.cuda.synchronize()
    return ent.cpu().numpy().view(np.uint32), lens.cpu().numpy()


def _check(dev, Q, C):
    k, n_c = Q.shape
    ct = 64 * C
    E = max(1, C // 16)
    ent, lens = _gpu_lists(dev, Q, C)
    bits = np.ascontiguousarray(Q, dtype=np.float32).view(np.uint32)
    for b in range(ent.shape[0]):
        c0 = b * ct
        for t in range(ent.shape[1]):
            seg_len = int(lens[b, t])
            if t >= k:
                assert seg_len == 0, (b, t)
                continue
            row = Q[t, c0:c0 + ct]
            cols = [c for c in range(len(row)) if not (row[c] == 0)]  # NaN != 0: kept
            nch = -(-len(cols) // 64)
            want_len = -(-nch // E) * E * 64 if cols else 0
            assert seg_len == want_len, (b, t, seg_len, want_len)
            if not cols:
                continue
            got = ent[b, t, :seg_len]
            model = model_segment(cols, ct)
            for s in range(seg_len // 64):
                for l in range(64):
                    c = model[s][l] if s < nch else None
                    want = (0, 4 * (ct + l)) if c is None else (int(bits[t, c0 + c]), 4 * c)
                    assert tuple(int(v) for v in got[s * 64 + l]) == want, (b, t, s, l, c)
            # invariants the kernel relies on
            listed = sorted(int(o) // 4 for o in got[:, 1] if int(o) // 4 < ct)
            assert listed == cols, (b, t)
            per_lane = np.bincount(np.array(cols) % 64, minlength=64)
            for s in range(nch):
                for l in range(64):
                    c = int(got[s * 64 + l][1]) // 4
                    if c >= ct:
                        assert c == ct + l and int(got[s * 64 + l][0]) == 0
                    elif s < min(int(per_lane[l]), nch):
                        assert c % 64 == l  # the lane's own column first


def _random(k, n_c, d, seed):
    r = np.random.default_rng(seed)
    Q = r.uniform(-1, 1, (k, n_c)).astype(np.float32)
    Q[r.random((k, n_c)) > d] = 0
    Q[(Q == 0) & (r.random((k, n_c)) < 0.5)] = -0.0
    return Q


@pytest.mark.parametrize("C", [1, 4, 16, 32, 64])
@pytest.mark.parametrize("d", [0.02, 0.05, 0.3, 1.0])
def test_base_lists_random(dev, C, d):
    """Ragged k (not a multiple of 16) and n_c (a partial last band)."""
    _check(dev, _random(37, 700 if C <= 16 else 2 * 64 * C + 300, d, 11 + C + int(100 * d)), C)


@pytest.mark.parametrize("pattern", ["one_residue", "bank_pair", "lower_full", "upper_full",
                                     "nan_and_negzero"])
def test_base_lists_uneven_residues(dev, pattern):
    """Bases piled into a few lanes: hand-overs to the lane 32 away, alternation
    between half-waves, and a full half-wave passing its excess on."""
    C, n_c, k = 16, 1024, 20
    Q = _random(k, n_c, 1.0, 77)
    idx = np.arange(n_c)
    if pattern == "one_residue":
        keep = idx % 64 == 5
    elif pattern == "bank_pair":
        keep = (idx % 64 == 5) | (idx % 64 == 37)
    elif pattern == "lower_full":
        keep = idx % 64 < 48
    elif pattern == "upper_full":
        keep = idx % 64 >= 16
    else:
        keep = idx % 3 == 0
        Q[:, idx % 7 == 0] = np.nan  # NaN is a non-zero base
        Q[:, idx % 5 == 0] = -0.0  # -0.0 is not
    Q[:, ~keep] = 0
    _check(dev, Q, C)


def test_base_lists_rejects_bad_arguments(dev):
    import torch
    import paper_1308_2400_amd as afmm
    Q = torch.zeros((4, 64), dtype=torch.float32, device=dev)
    e = torch.zeros(16 * 64 * 2, dtype=torch.int32, device=dev)
    ln = torch.zeros(16, dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    for args in [(0, 64, 64, 1), (4, 64, 63, 1), (4, 64, 64, 0), (4, 64, 64, 65)]:
        k, n_c, ldq, C = args
        assert afmm.afmm_base_lists(Q.data_ptr(), k, n_c, ldq, C, e.data_ptr(), ln.data_ptr(),
                                    s) == 1, args
    assert afmm.afmm_base_lists(None, 4, 64, 64, 1, e.data_ptr(), ln.data_ptr(), s) == 1
