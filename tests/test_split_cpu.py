"""Host logic of the row-split planner (no GPU): split points, the 1.25x
competitive classification and the per-iteration time model."""
import math

import numpy as np
import pytest

from paper_2608_09647_amd import split as S


def test_rows_for_share_rounds_half_away_from_zero():
    assert S.rows_for_share(3, 0.5) == 2            # 1.5 -> 2
    assert S.rows_for_share(5, 0.5) == 3            # 2.5 -> 3
    assert S.rows_for_share(4, 0.5) == 2
    assert S.rows_for_share(16_777_216, 0.5) == 8_388_608
    assert S.rows_for_share(10, 0.0) == 0 and S.rows_for_share(10, 1.0) == 10
    for bad in (-0.1, 1.1):
        with pytest.raises(ValueError):
            S.rows_for_share(10, bad)


def test_rows_for_nnz_share_is_the_smallest_prefix_reaching_the_share():
    rng = np.random.default_rng(3)
    for _ in range(50):
        lens = rng.integers(0, 40, size=rng.integers(1, 60))
        rp = np.concatenate([[0], np.cumsum(lens)])
        for g in (0.0, 0.1, 0.25, 0.5, 0.77, 1.0):
            k = S.rows_for_nnz_share(rp, g)
            # brute force: the first row count whose prefix holds >= g nnz
            want = next(i for i in range(rp.size) if rp[i] >= g * rp[-1])
            assert k == want


def test_competitive_classification():
    flags = S.competitive({"a": 1.0, "b": 1.25, "c": 1.2500001, "d": math.inf, "e": None})
    assert flags == {"a": True, "b": True, "c": False, "d": False, "e": False}
    assert S.competitive({"x": math.nan}) == {"x": False}


def _probe(gpu_rate, cpu_rate, ex, other, nnz, nnz_gpu, iters=30):
    """Timers a split solve with these rates would report."""
    tg, tc = nnz_gpu / gpu_rate, (nnz - nnz_gpu) / cpu_rate
    probe = {"iterations": iters, "nnz_gpu": nnz_gpu, "nnz_cpu": nnz - nnz_gpu,
             "t_gpu": tg * iters, "t_cpu": tc * iters, "t_d2h": 0.6 * ex * iters, "t_h2d": 0.4 * ex * iters}
    return probe, (max(tg, tc) + ex + other) * iters


def test_model_recovers_rates_and_predicts_by_hand():
    nnz = 1_000_000
    probe, secs = _probe(gpu_rate=4e9, cpu_rate=1e9, ex=2e-4, other=5e-5, nnz=nnz, nnz_gpu=500_000)
    m = S.IterationModel.fit(probe, secs, nnz)
    assert m.gpu_rate == pytest.approx(4e9) and m.cpu_rate == pytest.approx(1e9)
    assert m.exchange == pytest.approx(2e-4) and m.other == pytest.approx(5e-5)
    # by hand: 800k on the GPU -> max(2e-4, 2e-4) + exchange + other
    assert m.predict(800_000) == pytest.approx(2e-4 + 2e-4 + 5e-5)
    # the ends exchange nothing
    assert m.predict(0) == pytest.approx(1e-3 + 5e-5)
    assert m.predict(nnz) == pytest.approx(2.5e-4 + 5e-5)


def test_choose_split_minimises_the_model_over_the_candidates():
    n = 1000
    rp = np.arange(0, 10 * (n + 1), 10)                 # 10 entries per row
    nnz = int(rp[-1])
    # 2e-6 s of compute at the balance point, exchange 1e-8 s: g = 0.8 beats
    # the GPU alone (2.5e-6 s)
    probe, secs = _probe(gpu_rate=4e9, cpu_rate=1e9, ex=1e-8, other=0.0, nnz=nnz, nnz_gpu=nnz // 2)
    m = S.IterationModel.fit(probe, secs, nnz)
    res = S.choose_split(m, rp)
    brute = min(S.SHARES, key=lambda g: (m.predict(int(rp[S.rows_for_share(n, g)])), -g))
    assert res["share"] == brute == 0.8                 # balance point of a 4:1 rate ratio
    assert len(res["table"]) == len(S.SHARES)
    # expensive exchange: a GPU-only run wins
    probe, secs = _probe(gpu_rate=4e9, cpu_rate=1e9, ex=1.0, other=0.0, nnz=nnz, nnz_gpu=nnz // 2)
    assert S.choose_split(S.IterationModel.fit(probe, secs, nnz), rp)["share"] == 1.0


def test_choose_config_picks_the_fastest_mode():
    rp = np.arange(0, 5 * 101, 5)
    nnz = int(rp[-1])
    fast = S.IterationModel.fit(*_probe(4e9, 1e9, 1e-6, 0.0, nnz, nnz // 2), nnz)
    slow = S.IterationModel.fit(*_probe(1e9, 1e9, 1e-3, 0.0, nnz, nnz // 2), nnz)
    res = S.choose_config({"whole": slow, "halo": fast}, rp)
    assert res["mode"] == "halo" and set(res["per_mode"]) == {"whole", "halo"}


def test_model_needs_a_split_probe():
    probe, secs = _probe(4e9, 1e9, 0.0, 0.0, 100, 100)
    with pytest.raises(ValueError):
        S.IterationModel.fit(probe, secs, 100)


def test_transfer_bound_scales_only_the_transfer_part():
    # by hand: T = 10, transfers 7 of it, R = 7 -> 3 + 1
    assert S.transfer_bound(10.0, 7.0, 7.0) == pytest.approx(4.0)
    assert S.transfer_bound(10.0, 0.0) == 10.0                  # nothing to scale
    assert S.transfer_bound(10.0, 10.0, 2.0) == pytest.approx(5.0)
    assert S.LINK_RATIO == pytest.approx(900 / 128)
    for bad in ((10.0, 11.0, 2.0), (10.0, -1.0, 2.0), (10.0, 1.0, 0.0)):
        with pytest.raises(ValueError):
            S.transfer_bound(*bad)


def test_transfer_bound_table_reports_a_moved_optimum():
    runs = {"g1.00": {"seconds": 5.0, "t_d2h": 0.0, "t_h2d": 0.0},
            "g0.75": {"seconds": 6.0, "t_d2h": 3.0, "t_h2d": 1.0}}   # transfer-heavy hybrid
    tab = S.transfer_bound_table(runs, ratio=8.0)
    assert tab["bound_seconds"]["g0.75"] == pytest.approx(2.0 + 0.5)
    assert tab["preferred_measured"] == "g1.00" and tab["preferred_bound"] == "g0.75"
    assert tab["preferred_changes"]


def test_planner_constants_match_the_paper():
    """tests/golden/paper_constants.json holds the values the paper prints."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")) as f:
        g = json.load(f)
    assert list(S.SHARES) == g["gpu_shares"]["value"]
    assert S.COMPETITIVE_FACTOR == g["competitive_factor"]["value"]
    lr = g["link_ratio"]
    assert S.LINK_RATIO == lr["numerator_gbs"] / lr["denominator_gbs"]
    assert round(S.LINK_RATIO, lr["digits"]) == lr["value"]
