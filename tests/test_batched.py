"""Batched persistent path: every product bit-exact against the oracle, exact
per-problem counts, graph replays identical to the eager run."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_1308_2400_amd  # noqa: F401
    return torch.device("cuda:0")


def _to(dev, a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _mixed_problems(count, seed, n_max=300):
    r = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(r.integers(1, n_max + 1)) if t % 7 else int(r.choice([1, 2, 63, 64, 65, 257]))
        case = "A" if r.random() < 0.5 else "B"
        real = r.standard_normal((n, n)).astype(np.float32)
        real[r.random((n, n)) > r.uniform(0.05, 1)] = 0
        hi = int(r.choice([3, 15, 63, 255, 400]))
        ints = r.integers(0, hi + 1, (n, n)).astype(np.int32)
        ints[r.random((n, n)) > r.uniform(0.05, 1)] = 0
        if t % 11 == 3:
            ints[::2, ::3] *= -1  # negative counts add nothing
        out.append((case, *((real, ints) if case == "A" else (ints, real))))
    return out


def _run_plan(dev, probs):
    import torch
    import paper_1308_2400_amd as afmm
    dprobs = []
    for case, X, Y in probs:
        Xd, Yd = _to(dev, X), _to(dev, Y)
        Zd = torch.full((X.shape[0], X.shape[0]), float("nan"), dtype=torch.float32, device=dev)
        dprobs.append((case, Xd, Yd, Zd))
    return afmm.Plan(dprobs), dprobs


def test_batched_mixed_bitexact_and_counts(dev):
    probs = _mixed_problems(60, 1)
    plan, dprobs = _run_plan(dev, probs)
    plan.launch()
    adds = plan.problem_adds()
    for t, ((case, X, Y), (_, _, _, Zd)) in enumerate(zip(probs, dprobs)):
        Zref, a = oracle.strict_f32(case, X, Y)
        Z = Zd.cpu().numpy()
        assert np.array_equal(Z.view(np.uint32), Zref.view(np.uint32)), (t, case, X.shape)
        assert adds[t] == a == oracle.count(case, X, Y)[0], t
    plan.close()


def test_batched_large_tiles_bitexact(dev):
    """Problems of n >= 512 (the batch's widest tile body) mixed with small ones,
    every element bit for bit: both cases, counts up to 400 (escape path) and
    negative counts."""
    r = np.random.default_rng(17)
    probs = []
    for t, n in enumerate([512, 530, 601, 700, 577, 33, 129]):
        case = "AB"[t % 2]
        real = r.standard_normal((n, n)).astype(np.float32)
        real[r.random((n, n)) > r.uniform(0.1, 1)] = 0
        ints = r.integers(0, [3, 63, 400, 15, 255, 9, 7][t] + 1, (n, n)).astype(np.int32)
        ints[r.random((n, n)) > r.uniform(0.1, 1)] = 0
        if t == 2:
            ints[::3, ::2] *= -1
        probs.append((case, *((real, ints) if case == "A" else (ints, real))))
    plan, dprobs = _run_plan(dev, probs)
    plan.launch()
    adds = plan.problem_adds()
    for t, ((case, X, Y), (*_, Zd)) in enumerate(zip(probs, dprobs)):
        Zref, a = oracle.strict_f32_threaded(case, X, Y)
        Z = Zd.cpu().numpy()
        assert np.array_equal(Z.view(np.uint32), Zref.view(np.uint32)), (t, case, X.shape)
        assert adds[t] == a, t
    plan.close()


def test_batched_split_mode(dev):
    """Split-mode plans: each product equals the single-product split call, and
    the per-problem counts are the exact ones."""
    import torch
    import paper_1308_2400_amd as afmm
    r = np.random.default_rng(5)
    probs = []
    for t, n in enumerate([1, 40, 257, 300, 64]):
        case = "AB"[t % 2]
        real = r.standard_normal((n, n)).astype(np.float32)
        ints = r.integers(0, 257, (n, n)).astype(np.int32)
        probs.append((case, *((real, ints) if case == "A" else (ints, real))))
    dprobs = []
    for case, X, Y in probs:
        Zd = torch.full((X.shape[0], X.shape[0]), float("nan"), dtype=torch.float32, device=dev)
        dprobs.append((case, _to(dev, X), _to(dev, Y), Zd))
    plan = afmm.Plan(dprobs, mode="split")
    for _ in range(2):  # the captured graph, then its replay
        plan.launch()
        adds = plan.problem_adds()
        for t, ((case, X, Y), (_, Xd, Yd, Zd)) in enumerate(zip(probs, dprobs)):
            single = afmm.multiply(case, Xd, Yd, "split")
            assert torch.equal(single.view(torch.int32), Zd.view(torch.int32)), t
            assert oracle.rel_frobenius(Zd.cpu().numpy(), oracle.product_f64(case, X, Y)) <= 1e-6
            assert adds[t] == oracle.count(case, X, Y)[0], t
    plan.close()


def test_batched_alias_across_problems(dev):
    """An output that overlaps another problem's input or output is refused."""
    import ctypes
    import torch
    import paper_1308_2400_amd as afmm
    buf = torch.zeros(4 * 64, dtype=torch.float32, device=dev)
    Y = torch.zeros((8, 8), dtype=torch.int32, device=dev)
    p = lambda x, y, z: afmm.afmm_problem(0, 8, x, y, z)  # noqa: E731
    a, b, c, d = (buf.data_ptr() + 256 * t for t in range(4))
    h = ctypes.c_void_p()
    ok = (afmm.afmm_problem * 2)(p(a, Y.data_ptr(), b), p(a, Y.data_ptr(), c))  # shared X: fine
    assert afmm.afmm_batched_plan_create(ok, 2, 0, ctypes.byref(h)) == 0
    afmm.afmm_batched_plan_destroy(h)
    bad = (afmm.afmm_problem * 2)(p(a, Y.data_ptr(), b), p(c, Y.data_ptr(), a))  # Z_2 = X_1
    assert afmm.afmm_batched_plan_create(bad, 2, 0, ctypes.byref(h)) == 2
    bad = (afmm.afmm_problem * 2)(p(a, Y.data_ptr(), c), p(b, Y.data_ptr(), c + 128))  # Zs overlap
    assert afmm.afmm_batched_plan_create(bad, 2, 0, ctypes.byref(h)) == 2


def test_batched_graph_replays_identical(dev):
    import torch
    probs = _mixed_problems(25, 2, n_max=200)
    plan, dprobs = _run_plan(dev, probs)
    plan.launch()
    torch.cuda.synchronize()
    first = [Zd.clone() for *_, Zd in dprobs]
    for rep in range(3):
        # eager work and a synchronisation between the replays
        for *_, Zd in dprobs:
            Zd.fill_(-1.0)
        junk = torch.randn(1000, device=dev).sum()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for a, (*_, Zd) in zip(first, dprobs):
            assert torch.equal(a.view(torch.int32), Zd.view(torch.int32)), rep
        del junk
    plan.close()


def test_batched_oneshot_matches_plan(dev):
    import ctypes
    import torch
    import paper_1308_2400_amd as afmm
    probs = _mixed_problems(12, 3, n_max=150)
    plan, dprobs = _run_plan(dev, probs)
    plan.launch()
    torch.cuda.synchronize()
    arr = (afmm.afmm_problem * len(dprobs))()
    outs = []
    for t, (case, Xd, Yd, Zd) in enumerate(dprobs):
        Z2 = torch.empty_like(Zd)
        outs.append(Z2)
        arr[t] = afmm.afmm_problem(0 if case == "A" else 1, Xd.shape[0], Xd.data_ptr(),
                                   Yd.data_ptr(), Z2.data_ptr())
    st = afmm.afmm_multiply_batched(arr, len(dprobs), 0,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    for Z2, (*_, Zd) in zip(outs, dprobs):
        assert torch.equal(Z2.view(torch.int32), Zd.view(torch.int32))
    plan.close()


def test_batched_errors(dev):
    import ctypes
    import torch
    import paper_1308_2400_amd as afmm
    X = torch.zeros((8, 8), dtype=torch.float32, device=dev)
    Y = torch.zeros((8, 8), dtype=torch.int32, device=dev)
    Z = torch.zeros((8, 8), dtype=torch.float32, device=dev)
    arr = (afmm.afmm_problem * 1)(afmm.afmm_problem(0, 8, X.data_ptr(), Y.data_ptr(), Z.data_ptr()))
    h = ctypes.c_void_p()
    assert afmm.afmm_batched_plan_create(arr, 1, 2, ctypes.byref(h)) == 1  # no such mode
    assert afmm.afmm_batched_plan_create(arr, 0, 0, ctypes.byref(h)) == 1
    arr[0].Z = X.data_ptr()
    assert afmm.afmm_batched_plan_create(arr, 1, 0, ctypes.byref(h)) == 2  # Z aliases X
    arr[0].n = 0
    assert afmm.afmm_batched_plan_create(arr, 1, 0, ctypes.byref(h)) == 1


def test_batched_512_sampled(dev):
    """The 512-product workload: exact counts for all, sampled rows bit-exact for all."""
    ws = gen.batched_512()
    probs = [(w.case, w.X(), w.Y()) for w in ws]
    plan, dprobs = _run_plan(dev, probs)
    plan.launch()
    adds = plan.problem_adds()
    r = np.random.default_rng(0)
    for t, ((case, X, Y), (*_, Zd)) in enumerate(zip(probs, dprobs)):
        n = X.shape[0]
        assert adds[t] == oracle.count(case, X, Y)[0], t
        rows = sorted(set([0, n - 1, int(r.integers(0, n))]))
        Zref, _ = oracle.strict_f32(case, X[rows], Y, rows=rows, x_rows_only=True)
        Z = Zd.cpu().numpy()[rows]
        assert np.array_equal(Z.view(np.uint32), Zref.view(np.uint32)), (t, case, n)
    plan.close()


def test_batched_shape_thresholds_same_bits(dev):
    """Plans built under other tile-shape thresholds (every problem on the widest
    tiles, or every one on the narrowest) give the built-in plan's bits; bad
    thresholds are refused."""
    import torch
    import paper_1308_2400_amd as afmm
    probs = _mixed_problems(20, 9, n_max=700)
    plan, dprobs = _run_plan(dev, probs)
    plan.launch()
    torch.cuda.synchronize()
    ref = [Zd.clone() for *_, Zd in dprobs]
    plan.close()
    try:
        for pair in ((1, 1), (1 << 20, 1 << 20), (300, 64)):
            afmm.set_batch_shapes(*pair)
            plan, dprobs2 = _run_plan(dev, probs)
            plan.launch()
            torch.cuda.synchronize()
            for t, (a, (*_, Zd)) in enumerate(zip(ref, dprobs2)):
                assert torch.equal(a.view(torch.int32), Zd.view(torch.int32)), (pair, t)
            plan.close()
        assert afmm.afmm_set_batch_shapes(64, 128) == 1
        assert afmm.afmm_set_batch_shapes(64, 0) == 1
    finally:
        afmm.set_batch_shapes()
