"""The paper's Table 1 grid (Section 2.3.1) on the GPU: cells bit-exact with the
exact addition count; and the empirical-order fit of the benchmark recovering
known exponents from synthetic timings (Section 2.3: the order is estimated
from measured times)."""
import numpy as np
import pytest

import gen
import oracle


@pytest.mark.gpu
@pytest.mark.parametrize("n", [250, 500])
@pytest.mark.parametrize("mu", [1, 21])
@pytest.mark.parametrize("ydist", ["const", "uniform"])
def test_table1_cell_bitexact_and_count(n, mu, ydist):
    import torch
    import paper_1308_2400_amd as afmm
    w = gen.table1(n, mu, ydist)
    X, Y = w.X(), w.Y()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    Z = afmm.multiply("A", Xd, Yd).cpu().numpy()
    Zref, adds = oracle.strict_f32_threaded("A", X, Y)
    assert np.array_equal(Z.view(np.uint32), Zref.view(np.uint32))
    assert afmm.count_adds("A", Xd, Yd) == adds == oracle.count("A", X, Y)[0]


def _synthetic_rows(b_time, t0, rate):
    """Timings of the grid's shape built from a known law: per (mu', reading) the
    time grows as c * n^b_time exactly; the additions as n^3."""
    rows = []
    for mu in (1, 21):
        for yd in ("const", "uniform"):
            for n in (250, 500, 1000, 2000):
                adds = 1e-2 * mu * n ** 3
                rows.append({"n": n, "mu_prime": mu, "y_nonzeros": yd, "adds": adds,
                             "gpu_ms": 0.5 * mu * (n / 250.0) ** b_time})
    return rows


def test_empirical_fit_recovers_exponents():
    import bench
    rows = _synthetic_rows(1.37, 0, 0)
    fit = bench.empirical_fit(rows)
    for key, f in fit["per_mu"].items():
        assert abs(f["time_exponent_in_n"] - 1.37) < 1e-9, key
        assert abs(f["adds_exponent_in_n"] - 3.0) < 1e-9, key


def test_empirical_fit_recovers_rate_and_offset():
    import bench
    rows = []
    for n in (250, 500, 1000, 2000):
        for mu in (1, 21):
            adds = 1e-2 * mu * n ** 3
            rows.append({"n": n, "mu_prime": mu, "y_nonzeros": "const", "adds": adds,
                         "gpu_ms": 0.03 + adds / 5e12 * 1e3})
    fit = bench.empirical_fit(rows)["time_vs_adds"]
    assert abs(fit["t0_ms"] - 0.03) < 1e-9
    assert abs(fit["adds_per_s"] / 5e12 - 1) < 1e-9
    assert fit["r2"] > 1 - 1e-12
