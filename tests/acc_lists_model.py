"""Host model of the compacted-base list builder's slot placement (used by
test_acc_lists.py on the GPU and test_acc_lists_model.py on the CPU).

Lane l owns the band's columns c = l (mod 64) and takes them first, in
ascending order; a lane with more than nch = ceil(total/64) hands the rest to
the lane 32 away (same LDS bank, other half-wave), then to free slots of other
lanes, dealt alternately to the other and to the own half-wave in lane order, a
full half-wave passing its excess to the other; free slots are sinks (None)."""


def model_segment(cols, ct):
    """Slot list (nch chunks of 64 columns or None) of one segment, the
    placement rule written out lane by lane."""
    a_cols = [[] for _ in range(64)]
    for c in cols:  # ascending, so each lane's list is too
        a_cols[c % 64].append(c)
    total = len(cols)
    nch = -(-total // 64)
    slots = [[None] * 64 for _ in range(nch)]
    a = [len(x) for x in a_cols]
    own = [min(x, nch) for x in a]
    for l in range(64):
        for s in range(own[l]):
            slots[s][l] = a_cols[l][s]
    give, recv = [0] * 64, [0] * 64
    for l in range(64):
        p = l ^ 32
        give[l] = min(a[l] - own[l], nch - own[p])
        recv[l] = min(a[p] - own[p], nch - own[l])
    for l in range(64):
        p = l ^ 32
        for s in range(recv[l]):
            slots[own[l] + s][l] = a_cols[p][own[p] + s]
    holes = [nch - own[l] - recv[l] for l in range(64)]
    up_list, lo_list = [], []
    for l in range(64):
        up = l >= 32
        for j, c in enumerate(a_cols[l][own[l] + give[l]:]):
            # even j to the other half-wave, odd j to the lane's own
            (up_list if (j % 2 == 1) == up else lo_list).append(c)
    ue, le = len(up_list), len(lo_list)
    lst = up_list + lo_list
    uh = sum(holes[32:])
    lh = sum(holes[:32])
    ru = rl = 0
    for l in range(64):
        for s in range(own[l] + recv[l], nch):
            if l >= 32:
                t, ru = ru, ru + 1
                fill = min(ue, uh)
                idx = t if t < fill else (ue + lh + t - fill if le > lh and t - fill < le - lh else -1)
            else:
                t, rl = rl, rl + 1
                fill = min(le, lh)
                idx = ue + t if t < fill else (uh + t - fill if ue > uh and t - fill < ue - uh else -1)
            if idx >= 0:
                slots[s][l] = lst[idx]
    return slots
