"""Model-steered clock search (section V.D-E) end to end on a simulated
device (CPU): power follows Eq. 2/3 plus noise, run time scales as 1/f.  The
library fits the model to 5 readings, picks the band, and the search loop measures
only band clocks; the result must match the exhaustive clock sweep's energy
optimum closely while measuring at least 5x fewer clock points."""
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


def device(model, t_at_max, f_max, noise, seed):
    """Simulated GPU: power of Eq. 2/3 scaled per config; where that would
    exceed the power limit the clock throttles to the highest clock that fits
    (run time grows accordingly) and power sits at the limit."""
    rng = np.random.default_rng(seed)
    fine = np.arange(100.0, f_max + 1e-9, 1.0)

    def p_of(f, scale):
        return scale * float(opm.power(f, model["p_idle"], model["alpha"], model["beta"], model["tau"], 1e12))

    def measure(cfg, f):
        scale = 1.0 + 0.05 * (sum(cfg) % 7) / 7.0   # configs differ in power draw
        f_act, throttled = f, 0
        if p_of(f, scale) > model["p_max"]:
            ok = [g for g in fine if p_of(g, scale) <= model["p_max"]]
            f_act, throttled = (ok[-1] if ok else fine[0]), 1
        t = t_at_max[tuple(cfg)] * f_max / f_act
        p = min(p_of(f_act, scale), model["p_max"]) + rng.normal(0, noise)
        return {"t_run_s": t, "p_median_w": p, "e_run_j": p * t, "throttled": throttled, "sclk_act_mhz": f_act}
    return measure


@pytest.mark.parametrize("seed", range(4))
def test_steered_matches_exhaustive_with_fewer_points(seed):
    rng = np.random.default_rng(100 + seed)
    model = dict(p_idle=rng.uniform(150, 350), alpha=rng.uniform(0.25, 0.45), beta=rng.uniform(8e-4, 2e-3),
                 tau=rng.uniform(1000, 1500), p_max=1400.0)
    cfgs = [(16, 16, 4, 2, 1, 0), (32, 8, 4, 4, 0, 0), (16, 16, 8, 5, 0, 0)]
    t_at_max = {c: 1.4e-4 * (1 + 0.1 * k) for k, c in enumerate(cfgs)}
    settable = list(np.arange(500.0, 2400.0 + 1e-9, 10.0))
    meas = device(model, t_at_max, 2400.0, 2.0, seed)
    steered = tuner.steered_search(meas, cfgs, settable, p_max=model["p_max"], n_fit=5)
    full = tuner.exhaustive_clock_search(meas, cfgs, settable)
    assert len(steered["fit_points"]) <= 5
    # the paper's accounting (band only) and the strict one (with the fit readings)
    assert full["points_measured"] >= 5 * steered["points_measured_band"]
    assert full["points_measured"] >= 5 * steered["points_measured_total"]
    # energy of the steered optimum within 2 % of the exhaustive optimum
    assert steered["best"]["e_run_j"] <= full["best"]["e_run_j"] * 1.02
    # the band is centred on the library's model optimum and clamped to the settable list
    f_opt = steered["f_opt_mhz"]
    assert all(0.9 * f_opt <= f <= 1.1 * f_opt for f in steered["band_mhz"])


def test_fit_clocks_uniform_and_snapped():
    settable = list(np.arange(500.0, 2400.0 + 1e-9, 25.0))
    fc = tuner.fit_clocks(settable, 5)
    assert fc == [500.0, 975.0, 1450.0, 1925.0, 2400.0]


def test_steered_with_calibrated_model_takes_no_fit_readings():
    # fit once (calibration), then tune with that model: the same band and
    # clock choice as fitting inside the search, without its readings
    model = dict(p_idle=250.0, alpha=0.35, beta=1.2e-3, tau=1250.0, p_max=1400.0)
    cfgs = [(16, 16, 4, 2, 1, 0), (32, 8, 4, 4, 0, 0)]
    t_at_max = {c: 1.4e-4 * (1 + 0.1 * k) for k, c in enumerate(cfgs)}
    settable = list(np.arange(500.0, 2400.0 + 1e-9, 10.0))
    meas = device(model, t_at_max, 2400.0, 0.0, 0)
    fitted = tuner.steered_search(meas, cfgs, settable, p_max=model["p_max"], n_fit=5)
    reused = tuner.steered_search(meas, cfgs, settable, p_max=model["p_max"], model=fitted["model"])
    assert reused["fit_points"] == []
    assert reused["band_mhz"] == fitted["band_mhz"] and reused["f_opt_mhz"] == fitted["f_opt_mhz"]
    assert reused["points_measured_total"] == reused["points_measured_band"] == len(cfgs) * len(reused["band_mhz"])
    assert reused["best"]["clock_mhz"] == fitted["best"]["clock_mhz"]


def test_fit_readings_start_at_top_clock_and_skip_throttled():
    model = dict(p_idle=250.0, alpha=0.45, beta=2e-3, tau=1200.0, p_max=1000.0)  # throttles near the top
    cfgs = [(16, 16, 4, 2, 1, 0)]
    meas = device(model, {cfgs[0]: 1.4e-4}, 2400.0, 0.0, 0)
    settable = list(np.arange(500.0, 2400.0 + 1e-9, 10.0))
    pts, fit = tuner.fit_readings(lambda f: meas(cfgs[0], f), settable, model["p_max"], n_fit=5)
    assert pts[0]["clock_mhz"] == 2400.0 and pts[0]["throttled"]
    assert len(pts) <= 5
    assert all(p["clock_mhz"] <= pts[0]["sclk_act_mhz"] for p in pts[1:])


def test_pick_calibration_needs_a_full_load():
    from paper_2211_07260_amd import tuner
    # a register-only FMA load below the convolution's power is not a stand-in
    assert tuner.pick_calibration({0: 735.0, 1: 1350.0, 2: 895.0}, 1034.0) == 1
    assert tuner.pick_calibration({0: 735.0, 2: 895.0}, 1034.0) is None
    assert tuner.pick_calibration({0: 1100.0, 1: 1100.0}, 1034.0) == 0  # tie: lower kind
    assert tuner.pick_calibration({0: float("nan"), 1: 1040.0}, 1034.0) == 1
