"""The measurement loop with the DVFS knob and the power sensor replaced by
the library's fake backends (the hardware clock is never touched): real
kernel launches and HIP-event timing, synthetic power from a known Eq. 2/3
model at the requested clock.  Checks the median-power energy arithmetic,
the clock bookkeeping, the fit recovering the model from <= 5 readings, and
that without the fake backend a clock request is refused."""
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    yield g


def bufs(f=17, side=1024):
    dev = torch.device("cuda:0")
    img = torch.rand(side + f - 1, side + f - 1, device=dev)
    w = torch.rand(f, f, device=dev)
    return img, w, torch.empty(side, side, device=dev)


MODEL = dict(p_idle=240.0, alpha=0.35, beta=0.0012, tau=1250.0, p_max=5000.0)  # no clipping in range


def test_clock_request_refused_without_permission(gt):
    gt.init(0, 0)
    try:
        img, w, out = bufs()
        with pytest.raises(gt.GreentuneError) as e:
            gt.conv2d_run(gt.xcorr_problem(1024, 1024, 17, 17), (32, 8, 4, 2, 0, 0), img, w, out,
                          clk=gt.clock(gt.CLOCK_SCLK_MHZ, 1500))
        assert e.value.code == gt.GT_E_PERM
        assert gt.dvfs_state() == (False, (0, 0))
    finally:
        gt.shutdown()


def test_fake_measurement_and_steered_fit(gt):
    from paper_2211_07260_amd import tuner
    gt.init(0, gt.INIT_FAKE_SENSOR | gt.INIT_FAKE_DVFS)
    try:
        m = gt.power_model(MODEL["p_idle"], MODEL["alpha"], MODEL["beta"], MODEL["tau"], MODEL["p_max"])
        gt.fake_sensor_model(m, noise_w=0.0)
        img, w, out = bufs()
        prob = gt.xcorr_problem(1024, 1024, 17, 17)
        cfg = (32, 8, 4, 2, 0, 0)
        for f in (800, 1300, 1900):
            r = gt.measure_time_energy(prob, cfg, img, w, out, gt.clock(gt.CLOCK_SCLK_MHZ, f), window_s=0.15,
                                       discard_s=0.03)
            want = gt.power_model_eval(m, f)
            assert r["p_median_w"] == pytest.approx(want, rel=1e-12)
            assert r["e_run_j"] == pytest.approx(want * r["t_run_s"], rel=1e-12)
            assert r["sclk_req_mhz"] == f and r["flags"] == 3 and r["launches"] >= 10
            assert gt.dvfs_state() == (True, (gt.CLOCK_SCLK_MHZ, f))

        def measure(c, f):
            return gt.measure_time_energy(prob, c, img, w, out, gt.clock(gt.CLOCK_SCLK_MHZ, int(f)),
                                          window_s=0.1, discard_s=0.02)
        settable = gt.settable_clocks(100.0)
        rep = tuner.steered_search(measure, [cfg], settable, p_max=MODEL["p_max"], n_fit=5)
        assert len(rep["fit_points"]) <= 5
        fit = rep["model"]
        assert fit["rss"] < 1e-6
        assert fit["alpha"] == pytest.approx(MODEL["alpha"], rel=1e-4)
        assert rep["band_mhz"] and len(rep["band_mhz"]) < len(settable)
    finally:
        gt.shutdown()


def test_fake_dvfs_tuning_methods(gt):
    # the five methods over 2 configs x 4 clocks through the real measurement
    # loop: with the fake power model and run time ~ clock-independent (the
    # clock is not really changed), each pick must still follow its rule
    from paper_2211_07260_amd import tuner
    gt.init(0, gt.INIT_FAKE_SENSOR | gt.INIT_FAKE_DVFS)
    try:
        m = gt.power_model(MODEL["p_idle"], MODEL["alpha"], MODEL["beta"], MODEL["tau"], MODEL["p_max"])
        gt.fake_sensor_model(m, noise_w=0.0)
        img, w, out = bufs(side=512)
        prob = gt.xcorr_problem(512, 512, 17, 17)
        cfgs = [(32, 8, 4, 2, 0, 0), (16, 16, 4, 4, 1, 0)]
        calls = []

        def measure(c, f):
            calls.append((tuple(c), f))
            return gt.measure_time_energy(prob, c, img, w, out, gt.clock(gt.CLOCK_SCLK_MHZ, int(f)),
                                          window_s=0.05, discard_s=0.01)
        rep = tuner.tuning_methods(measure, cfgs, [800.0, 1200.0, 1600.0, 2000.0])
        assert len(calls) == 8
        for name in tuner.METHODS:
            r = rep[name]
            assert r["sclk_req_mhz"] == r["clock_mhz"]
            assert r["p_median_w"] == pytest.approx(gt.power_model_eval(m, r["clock_mhz"]), rel=1e-12)
        best = min(rep["rows"], key=lambda r: (r["e_run_j"], r["t_run_s"]))
        assert rep["global_energy_to_solution"]["e_run_j"] == best["e_run_j"]
    finally:
        gt.shutdown()


def test_fake_dvfs_calibration_with_synthetic_loads(gt):
    # the three synthetic full loads run and report their rates; the power
    # model fitted from <= 5 readings of one of them (fake sensor, exact
    # model) recovers that model, and steering with it takes no more readings
    from paper_2211_07260_amd import tuner
    gt.init(0, gt.INIT_FAKE_SENSOR | gt.INIT_FAKE_DVFS)
    try:
        m = gt.power_model(MODEL["p_idle"], MODEL["alpha"], MODEL["beta"], MODEL["tau"], MODEL["p_max"])
        gt.fake_sensor_model(m, noise_w=0.0)
        buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
        for kind in (gt.LOAD_FP32_FMA, gt.LOAD_BF16_MFMA, gt.LOAD_COPY):
            r = gt.measure_load(kind, buf, gt.clock(gt.CLOCK_SCLK_MHZ, 1500), window_s=0.1, discard_s=0.02)
            assert r["gflops"] > 0 and r["launches"] >= 10
            assert r["p_median_w"] == pytest.approx(gt.power_model_eval(m, 1500), rel=1e-12)
        settable = gt.settable_clocks(100.0)
        cal = tuner.calibrate(gt.LOAD_FP32_FMA, buf, settable, MODEL["p_max"], window_s=0.1, discard_s=0.02)
        assert len(cal["fit_points"]) <= 5
        assert cal["model"]["rss"] < 1e-6
        assert cal["model"]["alpha"] == pytest.approx(MODEL["alpha"], rel=1e-4)
        img, w, out = bufs(side=512)
        prob = gt.xcorr_problem(512, 512, 17, 17)

        def measure(c, f):
            return gt.measure_time_energy(prob, c, img, w, out, gt.clock(gt.CLOCK_SCLK_MHZ, int(f)),
                                          window_s=0.05, discard_s=0.01)
        rep = tuner.steered_search(measure, [(32, 8, 4, 2, 0, 0)], settable, MODEL["p_max"], model=cal["model"])
        assert rep["fit_points"] == [] and rep["band_mhz"]
    finally:
        gt.shutdown()


def test_fake_power_cap_runs_the_highest_clock_that_fits(gt):
    # under a cap the fake firmware runs the highest clock (0.01 MHz grid over
    # 500..2400) whose model power fits; below the lowest clock's power the cap
    # is not met and the clock sits at 500 MHz
    import numpy as np
    from oracle import power_model as opm
    capped = dict(p_idle=240.0, alpha=0.35, beta=1.2e-3, tau=1250.0, p_max=1400.0)
    grid = 500.0 + 0.01 * np.arange(190001)
    p_grid = opm.power(grid, capped["p_idle"], capped["alpha"], capped["beta"], capped["tau"], capped["p_max"])
    gt.init(0, gt.INIT_FAKE_SENSOR | gt.INIT_FAKE_DVFS)
    try:
        m = gt.power_model(capped["p_idle"], capped["alpha"], capped["beta"], capped["tau"], capped["p_max"])
        gt.fake_sensor_model(m, noise_w=0.0)
        lo, hi, cur = gt.power_cap_range()
        assert (lo, hi, cur) == (700.0, 1400.0, 1400.0)
        buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
        for cap in (700, 883, 1050, 1233, 1400, 300):
            r = gt.measure_load(gt.LOAD_FP32_FMA, buf, gt.clock(gt.CLOCK_POWER_CAP_W, cap), window_s=0.1,
                                discard_s=0.02)
            ok = grid[p_grid <= cap]
            want = ok[-1] if len(ok) else 500.0
            assert r["sclk_act_mhz"] == pytest.approx(want, abs=0.011), cap
            assert r["p_median_w"] == pytest.approx(gt.power_model_eval(m, r["sclk_act_mhz"]), rel=1e-12)
            assert r["p_median_w"] <= cap or want == 500.0
        assert gt.power_cap_range()[2] == 300.0
    finally:
        gt.shutdown()


def test_power_cap_range_reads_on_the_device(gt):
    # the real amd-smi power-cap range (readable without privileges)
    gt.init(0, 0)
    try:
        lo, hi, cur = gt.power_cap_range()
        print("power cap range: min %.1f W, max %.1f W, in force %.1f W" % (lo, hi, cur))
        assert cur > 0
        if not (math.isnan(lo) or math.isnan(hi)):
            assert 0 <= lo <= cur <= hi
    finally:
        gt.shutdown()


def test_dvfs_requests_go_through_the_registered_backend(gt):
    # the library changes no device setting: with GT_INIT_ALLOW_DVFS a clock
    # request calls the caller's backend (a recorder here, so nothing changes
    # on the device), repeats are no-ops, and shutdown calls its restore
    calls = []
    gt.set_dvfs_backend(lambda dev, kind, value: calls.append(("apply", dev, kind, value)) or 0,
                        lambda dev: calls.append(("restore", dev)) or 0)
    try:
        gt.init(0, gt.INIT_ALLOW_DVFS)
        buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
        for _ in range(2):
            gt.measure_load(gt.LOAD_COPY, buf, gt.clock(gt.CLOCK_SCLK_MHZ, 1500), window_s=0.05, discard_s=0.01)
        gt.measure_load(gt.LOAD_COPY, buf, gt.clock(gt.CLOCK_POWER_CAP_W, 900), window_s=0.05, discard_s=0.01)
        assert gt.dvfs_state() == (True, (gt.CLOCK_POWER_CAP_W, 900))
        gt.shutdown()
        assert calls == [("apply", 0, gt.CLOCK_SCLK_MHZ, 1500), ("apply", 0, gt.CLOCK_POWER_CAP_W, 900),
                         ("restore", 0)]
    finally:
        gt.shutdown()
        gt.set_dvfs_backend(None)
    # without a backend the request is refused
    gt.init(0, gt.INIT_ALLOW_DVFS)
    try:
        buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
        with pytest.raises(gt.GreentuneError) as e:
            gt.measure_load(gt.LOAD_COPY, buf, gt.clock(gt.CLOCK_SCLK_MHZ, 1500), window_s=0.05, discard_s=0.01)
        assert e.value.code == gt.GT_E_PERM
    finally:
        gt.shutdown()


def test_dvfs_state_file_and_recovery(gt, tmp_path, monkeypatch):
    # the knob in force is recorded before the backend changes it and removed
    # after restore; a record left by a crashed process is restored by the
    # next gt_init (and refused when no backend can restore it)
    monkeypatch.setenv("TMPDIR", str(tmp_path))
    calls = []
    gt.set_dvfs_backend(lambda dev, kind, value: calls.append(("apply", kind, value)) or 0,
                        lambda dev: calls.append(("restore",)) or 0)
    try:
        gt.init(0, gt.INIT_ALLOW_DVFS)
        buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
        gt.measure_load(gt.LOAD_COPY, buf, gt.clock(gt.CLOCK_SCLK_MHZ, 1700), window_s=0.05, discard_s=0.01)
        files = list(tmp_path.glob("greentune-dvfs-*.state"))
        assert len(files) == 1 and files[0].read_text().split() == [str(gt.CLOCK_SCLK_MHZ), "1700"]
        record = files[0].read_text()
        gt.shutdown()
        assert not files[0].exists() and calls == [("apply", gt.CLOCK_SCLK_MHZ, 1700), ("restore",)]
        files[0].write_text(record)          # as a crashed process would have left it
        calls.clear()
        gt.init(0, gt.INIT_ALLOW_DVFS)
        assert calls == [("restore",)] and not files[0].exists()
        gt.shutdown()
        files[0].write_text(record)
    finally:
        gt.shutdown()
        gt.set_dvfs_backend(None)
    with pytest.raises(gt.GreentuneError) as e:
        gt.init(0, gt.INIT_ALLOW_DVFS)
    assert e.value.code == gt.GT_E_STATE
    files[0].unlink()
    gt.init(0, gt.INIT_ALLOW_DVFS)
    gt.shutdown()


def test_measure_load_argument_errors(gt):
    gt.init(0, 0)
    try:
        dev = torch.device("cuda:0")
        small = torch.empty(1 << 18, dtype=torch.float32, device=dev)   # 1 MiB
        for kind in (gt.LOAD_FP32_FMA, gt.LOAD_COPY):
            with pytest.raises(gt.GreentuneError) as e:
                gt.measure_load(kind, small, window_s=0.05, discard_s=0.01)
            assert e.value.code == gt.GT_E_INVAL
        buf = torch.empty(1 << 22, dtype=torch.float32, device=dev)
        with pytest.raises(gt.GreentuneError) as e:
            gt.measure_load(7, buf, window_s=0.05, discard_s=0.01)
        assert e.value.code == gt.GT_E_INVAL
    finally:
        gt.shutdown()


def test_refused_first_knob_change_leaves_no_state_file(gt, tmp_path, monkeypatch):
    monkeypatch.setenv("TMPDIR", str(tmp_path))
    gt.set_dvfs_backend(lambda dev, kind, value: 5, lambda dev: 0)   # apply always refuses
    try:
        gt.init(0, gt.INIT_ALLOW_DVFS)
        buf = torch.empty(1 << 22, dtype=torch.float32, device=torch.device("cuda:0"))
        with pytest.raises(gt.GreentuneError) as e:
            gt.measure_load(gt.LOAD_COPY, buf, gt.clock(gt.CLOCK_SCLK_MHZ, 1500), window_s=0.05, discard_s=0.01)
        assert e.value.code == gt.GT_E_PERM
        assert not list(tmp_path.glob("greentune-dvfs-*.state"))
        assert gt.dvfs_state() == (False, (0, 0))
    finally:
        gt.shutdown()
        gt.set_dvfs_backend(None)


@pytest.mark.parametrize("noise_w", [15.0, 60.0])
def test_noisy_window_energy_matches_oracle(gt, noise_w):
    # the fake sensor adds seeded Gaussian noise, so the kept readings differ
    # and the median and discard bound decide the result; the record must
    # equal the oracle's median-power energy over the same readings
    from oracle import measure as om
    gt.init(0, gt.INIT_FAKE_SENSOR | gt.INIT_FAKE_DVFS)
    try:
        m = gt.power_model(MODEL["p_idle"], MODEL["alpha"], MODEL["beta"], MODEL["tau"], MODEL["p_max"])
        gt.fake_sensor_model(m, noise_w=noise_w, seed=7)
        img, w, out = bufs()
        prob = gt.xcorr_problem(1024, 1024, 17, 17)
        for f, discard in ((1100, 0.05), (2000, 0.12)):
            r = gt.measure_time_energy(prob, (32, 8, 4, 2, 0, 0), img, w, out, gt.clock(gt.CLOCK_SCLK_MHZ, f),
                                       window_s=0.3, discard_s=discard)
            smp, t0, t1 = gt.measure_last_window()
            assert len(smp) == r["n_samples"] and t0 < t1
            ts = [s["t_s"] for s in smp]
            ps = [s["power_w"] for s in smp]
            assert len(set(ps)) > 10  # the noise makes the readings differ
            e_o, p_o, t_o, n_o = om.energy_per_run(ts, ps, t0, t1, r["launches"], discard)
            assert r["p_median_w"] == p_o and r["n_used"] == n_o
            assert r["e_run_j"] == p_o * r["t_run_s"]
            # the host-time window and the HIP-event window agree closely
            assert t_o == pytest.approx(r["t_run_s"], rel=0.05)
            assert r["p_min_w"] == min(p for t, p in zip(ts, ps) if t0 + discard <= t <= t1)
            # every fake reading is a fresh metrics update at the set clock
            assert r["sclk_act_mhz"] == float(f) and not r["throttled"]
    finally:
        gt.shutdown()
