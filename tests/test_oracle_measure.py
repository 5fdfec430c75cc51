"""Pins for the measurement / selection oracle (oracle/measure.py, oracle/space.py)."""
import csv
import itertools
import os

import numpy as np
import pytest

from oracle import measure, space

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_median_even_and_odd():
    assert measure.median([3, 1, 2]) == 2
    assert measure.median([4, 1, 3, 2]) == 2.5
    assert measure.median([5.0]) == 5.0


def test_energy_from_trace_discards_ramp():
    # 10 Hz sensor; ramp 200 -> 700 W over the first 0.3 s, then 800 W +- symmetric noise
    t = np.arange(0.0, 1.0001, 0.1)
    p = np.array([200, 450, 700, 790, 810, 800, 795, 805, 800, 790, 810], float)
    e, pm, t_run, n = measure.energy_per_run(t, p, 0.0, 1.0, 1000, 0.3)
    assert n == 8 and pm == 800.0
    assert t_run == pytest.approx(1e-3) and e == pytest.approx(0.8)


def test_energy_equals_power_times_time_for_constant_power():
    t = np.linspace(0, 2, 41)
    p = np.full_like(t, 612.5)
    e, pm, t_run, _ = measure.energy_per_run(t, p, 0.0, 2.0, 250, 0.3)
    assert pm == 612.5 and e == pytest.approx(612.5 * 2.0 / 250, rel=1e-15)


def test_flops_and_efficiency_units():
    F = measure.flops_xcorr(4096, 4096, 17, 17)
    assert F == 2 * 4096 * 4096 * 289
    assert measure.gflops(F, 1e-3) == pytest.approx(F / 1e6)
    # GFLOP/s/W == GFLOP/J: 1e9 flop over 2 J -> 0.5
    assert measure.gflops_per_watt(1e9, 2.0) == pytest.approx(0.5)
    assert measure.flops_conv(16, 128, 128, 64, 64, 3, 3) == 2 * 16 * 128 * 128 * 64 * 64 * 9


def test_select_objectives_and_tiebreak():
    rows = [dict(t_run=2.0, e_run=5.0), dict(t_run=1.0, e_run=6.0), dict(t_run=3.0, e_run=4.0),
            dict(t_run=1.0, e_run=6.0), dict(t_run=2.5, e_run=4.0)]
    assert measure.select(rows, "time") == 1          # tie with 3 broken by index
    assert measure.select(rows, "energy") == 4        # tie with 2 broken by time


def test_pareto_front_bruteforce_small():
    rows = [dict(t_run=1, e_run=5), dict(t_run=2, e_run=3), dict(t_run=3, e_run=3),
            dict(t_run=4, e_run=1), dict(t_run=2, e_run=4)]
    assert measure.pareto_front(rows) == [0, 1, 3]


def _table2():
    with open(os.path.join(GOLDEN, "table2_model_steered_gains.csv")) as fh:
        return [r for r in csv.reader(l for l in fh if not l.startswith("#"))]


def test_table2_gains_follow_from_before_after():
    # the printed before/after values are rounded to 3-4 digits; gains agree to 0.6 points
    for r in _table2():
        g = measure.relative_gain_pct(float(r[2]), float(r[3]))
        assert abs(g - float(r[4])) < 0.6, r


def test_table2_summary_mean_and_std():
    # section V.E: mean efficiency gain 42.0 +- 24.1 %, mean performance change -24.3 +- 12.1 %
    rows = _table2()
    m, s = measure.mean_and_sample_std([float(r[4]) for r in rows])
    assert round(m, 1) == 42.0 and round(s, 1) == 24.1
    m, s = measure.mean_and_sample_std([float(r[7]) for r in rows])
    assert round(m, 1) == -24.3 and round(s, 1) == 12.1


def test_clock_space_reduction():
    # 5 of 25 points kept is an 80 % reduction (V100 row of section V.E reports 80.0 %)
    assert measure.clock_space_reduction_pct(5, 25) == pytest.approx(80.0)


# ---- tune space ----

VALUES = dict(block_size_x=[16, 32, 64, 128], block_size_y=[1, 2, 4, 8, 16],
              tile_size_x=list(range(1, 9)), tile_size_y=list(range(1, 9)),
              use_lds_padding=[0, 1], read_path=[0])


def test_space_thread_limit_count():
    sp = space.enumerate_space(VALUES, 17, 17, max_threads=1024, lds_limit=1 << 30)
    assert len(sp) == 2560 - 128  # only bx=128, by=16 (2048 threads) is dropped


def test_space_lds_limit_bruteforce():
    for lim in (65536, 163840):
        sp = space.enumerate_space(VALUES, 17, 17, max_threads=1024, lds_limit=lim)
        n = 0
        for bx, by, tx, ty, pad in itertools.product(VALUES["block_size_x"], VALUES["block_size_y"],
                                                     range(1, 9), range(1, 9), (0, 1)):
            w = bx * tx + 16
            pitch = -(-w // 4) * 4 + 4 * pad
            if bx * by <= 1024 and 4 * pitch * (by * ty + 16) <= lim:
                n += 1
        assert len(sp) == n


def test_space_order_and_direct_dedup():
    vals = dict(VALUES, block_size_x=[32], block_size_y=[4], tile_size_x=[1, 2],
                tile_size_y=[1], read_path=[0, 1])
    sp = space.enumerate_space(vals, 3, 3)
    assert sp == [(32, 4, 1, 1, 0, 0), (32, 4, 1, 1, 0, 1), (32, 4, 1, 1, 1, 0),
                  (32, 4, 2, 1, 0, 0), (32, 4, 2, 1, 0, 1), (32, 4, 2, 1, 1, 0)]


def test_gemm_space_size_times_clocks():
    # section IV: 17,472 GEMM configurations times 7 clocks = 122,304 points
    assert 17472 * 7 == 122304
