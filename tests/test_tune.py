"""Host logic of the autotuner: which measured configuration becomes the table
entry for a size, and how the tuned sizes become size ranges (no GPU needed)."""
from paper_1308_2400_amd import tune


def test_compacted_base_form_stays_out_of_the_table():
    # the compacted-base form (mapping 4) is fastest here but density-specific
    timings = sorted([(0.5, (4, 2, 32, 8, 2, 8)), (0.7, (3, 1, 16, 16, 1, 8)),
                      (0.8, (0, 4, 4, 4, 1, 16)), (2.0, (2, 8, 8, 4, 1, 16))])
    r = tune.summarize("A", 2048, timings, [3, 1, 16, 16, 1, 8])
    assert r["config"] == [3, 1, 16, 16, 1, 8] and r["ms"] == 0.7
    assert r["sparse_real_config"] == [4, 2, 32, 8, 2, 8] and r["sparse_real_ms"] == 0.5
    assert [c for c, _ in r["all"]][0] == [4, 2, 32, 8, 2, 8]  # everything measured is kept


def test_no_compacted_base_measurement():
    r = tune.summarize("B", 256, [(0.1, (0, 2, 1, 4, 1, 16))], [0, 2, 1, 4, 1, 16])
    assert "sparse_real_config" not in r and r["config"] == [0, 2, 1, 4, 1, 16]


def test_table_ranges_meet_at_geometric_midpoints():
    res = [{"case": c, "n": n, "config": [0, n // 256, 1, 4, 1, 16], "ms": 1.0}
           for c in ("A", "B") for n in (256, 1024, 4096)]
    t = tune.to_table(res)
    a = [e for e in t if e["case"] == "A"]
    assert [(e["n_lo"], e["n_hi"]) for e in a] == [(1, 512), (513, 2048), (2049, 1 << 30)]
    assert all(e["tuned_at"] in (256, 1024, 4096) for e in t) and len(t) == 6
    # ranges of one case tile [1, 2^30] without gaps or overlaps
    for c in ("A", "B"):
        es = sorted((e for e in t if e["case"] == c), key=lambda e: e["n_lo"])
        assert es[0]["n_lo"] == 1 and es[-1]["n_hi"] == 1 << 30
        assert all(x["n_hi"] + 1 == y["n_lo"] for x, y in zip(es, es[1:]))


def test_candidates_cover_every_compiled_mapping():
    assert {c[0] for c in tune.CANDIDATES} == {0, 2, 3, 4}
    assert set(tune.TABLE_MAPPINGS) == {0, 2, 3}


def test_batch_shape_pick():
    t = [(26.9, (512, 128)), (26.1, (384, 96)), (27.5, (256, 64))]
    r = tune.pick_batch_shapes(t)
    assert (r["n_wide"], r["n_mid"]) == (384, 96) and r["ms"] == 26.1
    assert [p for p, _ in r["all"]][0] == [384, 96]
    # a tie keeps the built-in pair
    r = tune.pick_batch_shapes([(26.0, (384, 96)), (26.0, (512, 128))])
    assert (r["n_wide"], r["n_mid"]) == (512, 128)


def test_batch_grid_is_ordered_and_holds_the_builtin_pair():
    assert (512, 128) in tune.BATCH_GRID
    assert all(1 <= m <= w for w, m in tune.BATCH_GRID)
