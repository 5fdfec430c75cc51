"""Power capping versus clock tuning (section V.C) on a simulated device
(CPU): the same configs searched with the clock or the power cap as the extra
tunable, 7 equidistant points of each knob's range.  Under a cap the device
runs the highest clock whose power fits; the cap range starts well above idle,
so capping cannot reach the low clocks that clock tuning can."""
import numpy as np
import pytest

import paper_2211_07260_amd as gt
from paper_2211_07260_amd import tuner
from oracle import power_model as opm


@pytest.fixture(scope="module", autouse=True)
def host_only():
    gt.init(0, gt.INIT_HOST_ONLY)
    yield
    gt.shutdown()


F_MIN, F_MAX = 500.0, 2400.0
FINE = np.arange(F_MIN, F_MAX + 1e-9, 1.0)


def sim(model, t_at_max):
    """measure_clock(cfg, f) and measure_cap(cfg, watts) of one simulated GPU
    (run time ~ 1/clock, power of Eq. 2/3 scaled per config)."""
    def p_of(f, scale):
        return scale * opm.power(f, model["p_idle"], model["alpha"], model["beta"], model["tau"], 1e12)

    def run(cfg, f_act):
        scale = 1.0 + 0.05 * (sum(cfg) % 7) / 7.0
        t = t_at_max[tuple(cfg)] * F_MAX / f_act
        p = float(min(p_of(f_act, scale), model["p_max"]))
        return {"t_run_s": t, "p_median_w": p, "e_run_j": p * t, "sclk_act_mhz": float(f_act)}

    def measure_clock(cfg, f):
        scale = 1.0 + 0.05 * (sum(cfg) % 7) / 7.0
        ok = FINE[(FINE <= f) & (p_of(FINE, scale) <= model["p_max"])]
        return run(cfg, ok[-1] if len(ok) else F_MIN)

    def measure_cap(cfg, cap):
        scale = 1.0 + 0.05 * (sum(cfg) % 7) / 7.0
        ok = FINE[p_of(FINE, scale) <= min(cap, model["p_max"])]
        return run(cfg, ok[-1] if len(ok) else F_MIN)
    return measure_clock, measure_cap


CFGS = [(16, 16, 4, 2, 1, 0), (32, 8, 4, 4, 0, 0), (16, 16, 8, 5, 0, 0)]
T_AT_MAX = {c: 1.4e-4 * (1 + 0.1 * k) for k, c in enumerate(CFGS)}


def test_equidistant_points():
    assert tuner.equidistant(500.0, 2300.0, 7) == [500.0, 800.0, 1100.0, 1400.0, 1700.0, 2000.0, 2300.0]
    assert tuner.equidistant(700.0, 1400.0, 2) == [700.0, 1400.0]
    assert tuner.equidistant(1.0, 9.0, 1) == [9.0]


def test_cap_rows_respect_the_cap_or_sit_at_the_lowest_clock():
    model = dict(p_idle=300.0, alpha=0.3, beta=1.5e-3, tau=1300.0, p_max=1400.0)
    mc, mp = sim(model, T_AT_MAX)
    caps = tuner.equidistant(700.0, 1400.0, 7)
    rep = tuner.cap_vs_clock(mc, mp, CFGS, tuner.equidistant(F_MIN, F_MAX, 7), caps)
    assert rep["cap"]["points"] == rep["clock"]["points"] == 21
    for r in rep["cap"]["rows"]:
        assert r["p_median_w"] <= r["knob"] + 1e-9 or r["sclk_act_mhz"] == F_MIN
    # a higher cap never runs a lower clock
    for c in CFGS:
        f = [r["sclk_act_mhz"] for r in rep["cap"]["rows"] if tuple(r["config"]) == c]
        assert f == sorted(f)


def test_clock_tuning_reaches_below_the_lowest_cap():
    # energy optimum (P*/f minimal) near 900 MHz, far below the clock the
    # lowest cap (900 W) leaves: clock tuning finds lower energy
    model = dict(p_idle=120.0, alpha=0.25, beta=2.5e-3, tau=800.0, p_max=1400.0)
    mc, mp = sim(model, T_AT_MAX)
    clocks = tuner.equidistant(F_MIN, F_MAX, 7)
    caps = tuner.equidistant(900.0, 1400.0, 7)
    rep = tuner.cap_vs_clock(mc, mp, CFGS, clocks, caps)
    low_cap_clock = min(r["sclk_act_mhz"] for r in rep["cap"]["rows"])
    assert rep["clock"]["best"]["sclk_act_mhz"] < low_cap_clock
    assert rep["energy_cap_over_clock"] > 1.05
    # the best of each search is the energy minimum of its own table
    for key in ("clock", "cap"):
        assert rep[key]["best"]["e_run_j"] == min(r["e_run_j"] for r in rep[key]["rows"])


def test_capping_matches_clock_tuning_when_the_optimum_is_inside_the_cap_range():
    # race-to-idle regime (high idle power, flat voltage): the top clock is
    # optimal and both knobs reach it (top clock / highest cap)
    model = dict(p_idle=600.0, alpha=0.2, beta=1e-5, tau=2300.0, p_max=1400.0)
    mc, mp = sim(model, T_AT_MAX)
    rep = tuner.cap_vs_clock(mc, mp, CFGS, tuner.equidistant(F_MIN, F_MAX, 7), tuner.equidistant(700.0, 1400.0, 7))
    assert rep["clock"]["best"]["sclk_act_mhz"] == F_MAX
    assert rep["cap"]["best"]["sclk_act_mhz"] == F_MAX
    assert rep["energy_cap_over_clock"] == pytest.approx(1.0, rel=1e-12)
