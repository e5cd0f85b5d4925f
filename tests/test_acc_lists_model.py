"""CPU pins of the host model of the compacted-base list placement (the model
the GPU test compares the device lists with, slot for slot).

LDS serves a wave-wide 32-bit access as two half-waves over 32 banks, and
element (row, column) of the Z tile sits in bank (row offset + column) mod 32,
so a slot is conflict-free when its column is in its lane's bank (column =
lane mod 32).  Each bank has one lane per half-wave, so a chunk can hold at most
two columns of one bank without a conflict; the pins check that the placement
leaves exactly the unavoidable excess, sum over banks of max(0, n_bank - 2),
outside their lanes' banks, besides listing each column once with every lane's
own columns first."""
import numpy as np
import pytest

from acc_lists_model import model_segment


def _segments(seed):
    r = np.random.default_rng(seed)
    out = []
    for ct in (64, 256, 1024, 2048, 4096):
        for d in (0.02, 0.05, 0.3, 0.7, 1.0):
            for _ in range(6):
                out.append((ct, sorted(np.nonzero(r.random(ct) < d)[0].tolist())))
    idx = np.arange(1024)
    for keep in (idx % 64 == 5, (idx % 64 == 5) | (idx % 64 == 37), idx % 64 < 48,
                 idx % 64 >= 16, (idx >= 100) & (idx < 250)):
        out.append((1024, idx[keep].tolist()))
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_model_lists_each_column_once_owners_first(seed):
    for ct, cols in _segments(seed):
        if not cols:
            continue
        slots = model_segment(cols, ct)
        nch = -(-len(cols) // 64)
        assert len(slots) == nch
        placed = sorted(c for ch in slots for c in ch if c is not None)
        assert placed == cols
        for l in range(64):
            own = [c for c in cols if c % 64 == l]
            first = [slots[s][l] for s in range(min(len(own), nch))]
            assert first == own[:len(first)], (ct, l)


@pytest.mark.parametrize("seed", [3, 4])
def test_model_lists_only_unavoidable_bank_conflicts(seed):
    for ct, cols in _segments(seed):
        if not cols or len(cols) > 64:
            continue  # one chunk: every column shares the one access per row
        slots = model_segment(cols, ct)[0]
        foreign = sum(1 for l, c in enumerate(slots) if c is not None and c % 32 != l % 32)
        n_bank = np.bincount(np.array(cols) % 32, minlength=32)
        assert foreign == int(np.maximum(n_bank - 2, 0).sum()), (ct, len(cols))
        # a lane's partner (l ^ 32) is in its bank: a surplus column goes there
        # whenever that lane has no column of its own
        for l in range(64):
            mine = [c for c in cols if c % 64 == l]
            theirs = [c for c in cols if c % 64 == (l ^ 32)]
            if len(mine) >= 2 and not theirs:
                assert slots[l ^ 32] == mine[1]
