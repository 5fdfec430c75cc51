"""Host-side C-ABI tests (no GPU): the library loads, exports every symbol the
header declares, and its host arithmetic agrees with the oracle."""
import os
import re

import numpy as np
import pytest

import paper_2211_07260_amd as gt
from oracle import measure as om
from oracle import power_model as opm
from oracle import space as osp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*(?:\s+|\s*\*\s*)([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             src, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_symbols_exported():
    names = header_functions()
    assert {"conv2d_run", "tune_space_enumerate", "measure_time_energy", "fit_power_model"} <= set(names)
    lib = gt.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(gt.EXPORTED)


@pytest.fixture(scope="module", autouse=True)
def host_only():
    gt.init(0, gt.INIT_HOST_ONLY)
    yield
    gt.shutdown()


def test_gpu_calls_refused_host_only():
    import torch
    t = torch.zeros(16)  # covers the 4x4 input, 3x3 filter and 2x2 output
    with pytest.raises(gt.GreentuneError) as e:
        gt.conv2d_run(gt.xcorr_problem(2, 2, 3, 3), gt.config(), t, t, t, stream=0)
    assert e.value.code == gt.GT_E_STATE


VALUES = dict(block_size_x=[16, 32, 64, 128], block_size_y=[1, 2, 4, 8, 16],
              tile_size_x=list(range(1, 9)), tile_size_y=list(range(1, 9)),
              use_lds_padding=[0, 1], read_path=[0])


@pytest.mark.parametrize("lds", [65536, 163840])
@pytest.mark.parametrize("f", [3, 17])
def test_enumerate_matches_oracle(lds, f):
    p = gt.xcorr_problem(4096, 4096, f, f)
    got = [c.as_tuple() for c in gt.tune_space_enumerate(p, VALUES, max_threads=1024, lds_limit=lds)]
    want = osp.enumerate_space(VALUES, f, f, max_threads=1024, lds_limit=lds)
    assert got == want


def test_enumerate_with_read_path_and_dedup():
    p = gt.xcorr_problem(4096, 4096, 17, 17)
    vals = dict(VALUES, read_path=[0, 1])
    got = [c.as_tuple() for c in gt.tune_space_enumerate(p, vals, max_threads=1024, lds_limit=163840)]
    want = osp.enumerate_space(vals, 17, 17, max_threads=1024, lds_limit=163840)
    assert got == want
    got2 = gt.tune_space_enumerate(p, vals, max_threads=1024, lds_limit=163840, dedup_direct=False)
    assert len(got2) == len(osp.enumerate_space(vals, 17, 17, 1024, 163840, dedup_direct=False))


def test_enumerate_counts_documented():
    p = gt.xcorr_problem(4096, 4096, 17, 17)
    assert len(gt.tune_space_enumerate(p, VALUES, max_threads=1024, lds_limit=1 << 40)) == 2432


def test_enumerate_capacity_error():
    import ctypes
    p = gt.xcorr_problem(64, 64, 3, 3)
    arrs = [(ctypes.c_int32 * len(VALUES[n]))(*VALUES[n]) for n in gt.CONFIG_FIELDS]
    d = gt.SpaceDesc()
    for k, a in enumerate(arrs):
        d.values[k] = ctypes.cast(a, ctypes.POINTER(ctypes.c_int32))
        d.counts[k] = len(a)
    d.max_threads, d.lds_limit_bytes = 1024, 65536
    out = (gt.ConvConfig * 3)()
    n = ctypes.c_size_t(0)
    rc = gt.lib().tune_space_enumerate(ctypes.byref(p), ctypes.byref(d), out, 3, ctypes.byref(n))
    assert rc == gt.GT_E_CAPACITY and n.value > 3


def test_lds_bytes_matches_oracle():
    p = gt.xcorr_problem(256, 256, 17, 17)
    for c in [(32, 8, 4, 4, 0, 0), (16, 16, 3, 5, 1, 0), (128, 4, 8, 2, 1, 0)]:
        assert gt.lds_bytes(p, c) == osp.lds_bytes(c[0], c[1], c[2], c[3], c[4], 17, 17)
    assert gt.lds_bytes(p, (32, 8, 4, 4, 0, 1)) == 0


def test_flops():
    assert gt.problem_flops(gt.xcorr_problem(4096, 4096, 17, 17)) == om.flops_xcorr(4096, 4096, 17, 17)
    p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 16, 128, 128, 64, 64, 3, 3)
    assert gt.problem_flops(p) == om.flops_conv(16, 128, 128, 64, 64, 3, 3)


def test_energy_from_samples_matches_oracle():
    rng = np.random.default_rng(1)
    for n in (7, 8, 101):
        t = np.sort(rng.uniform(0, 1.2, n))
        p = rng.uniform(300, 900, n)
        e, pm, nu = gt.energy_from_samples(t, p, 0.05, 1.1, 977, 0.3)
        e2, pm2, t_run, nu2 = om.energy_per_run(t, p, 0.05, 1.1, 977, 0.3)
        assert nu == nu2 and pm == pm2 and e == pytest.approx(e2, rel=1e-15)


def test_energy_from_samples_empty_window():
    with pytest.raises(gt.GreentuneError) as e:
        gt.energy_from_samples([0.0, 0.1], [1.0, 2.0], 0.0, 1.0, 10, 0.5)
    assert e.value.code == gt.GT_E_SENSOR


def test_select_matches_oracle():
    rng = np.random.default_rng(2)
    for _ in range(20):
        rows = [dict(t_run_s=float(rng.integers(1, 5)), e_run_j=float(rng.integers(1, 5))) for _ in range(12)]
        orows = [dict(t_run=r["t_run_s"], e_run=r["e_run_j"]) for r in rows]
        for obj in ("time", "energy"):
            assert gt.select(rows, obj) == om.select(orows, obj)


MODELS = [dict(p_idle=180.0, alpha=0.12, beta=0.0012, tau=1350.0, p_max=5000.0),
          dict(p_idle=90.0, alpha=0.08, beta=0.0020, tau=1100.0, p_max=5000.0),
          dict(p_idle=250.0, alpha=0.3, beta=0.0015, tau=1500.0, p_max=1000.0)]


@pytest.mark.parametrize("m", MODELS)
def test_eval_matches_oracle(m):
    pmod = gt.power_model(m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"])
    for f in np.linspace(300, 2500, 57):
        want = float(opm.power(f, m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"]))
        assert gt.power_model_eval(pmod, f) == pytest.approx(want, rel=1e-15)
    lit = gt.power_model(m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"], literal=True)
    for f in (m["tau"] - 1, m["tau"], m["tau"] + 300):
        want = float(opm.power(f, m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"], literal=True))
        assert gt.power_model_eval(lit, f) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("m", MODELS)
def test_throttle_clock_matches_oracle(m):
    pmod = gt.power_model(m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"])
    want = opm.throttle_clock(dict(m))
    got = gt.power_model_throttle_clock(pmod)
    assert got == want or got == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("m", MODELS + [dict(p_idle=0.0, alpha=0.5, beta=0.01, tau=1200.0, p_max=1e9),
                                       dict(p_idle=320.0, alpha=0.37, beta=0.00115, tau=1020.0, p_max=1400.0),
                                       dict(p_idle=300.0, alpha=0.1, beta=0.0, tau=1000.0, p_max=1e9),
                                       dict(p_idle=300.0, alpha=0.55, beta=5e-5, tau=1500.0, p_max=1400.0),
                                       dict(p_idle=300.0, alpha=0.5, beta=0.0, tau=1000.0, p_max=1400.0),
                                       dict(p_idle=300.0, alpha=0.5, beta=0.0, tau=1000.0, p_max=400.0),
                                       dict(p_idle=250.0, alpha=0.4, beta=4e-4, tau=1600.0, p_max=1100.0)])
@pytest.mark.parametrize("step", [100.0, 25.0, 5.0])
def test_band_matches_oracle(m, step):
    settable = list(np.arange(500.0, 2400.0 + 1e-9, step))
    pmod = gt.power_model(m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"])
    f_opt, band = gt.power_model_band(pmod, settable, 0.1)
    om_ = dict(m)
    assert f_opt == opm.optimal_clock(settable, om_)
    assert band == opm.clock_band(settable, f_opt, 0.1)
    f_thr = opm.throttle_clock(om_)
    assert f_opt <= f_thr or f_opt == settable[0]


def test_plateau_model_optimum_below_throttle():
    # a full load at the socket cap: the model reaches P_max at 1918.8 MHz
    # while P*(f)/f would still fall above it; the optimum is a held clock
    pmod = gt.power_model(300.0, 0.55, 5e-5, 1500.0, 1400.0)
    f_thr = gt.power_model_throttle_clock(pmod)
    assert f_thr == pytest.approx(1918.8, abs=0.1)
    f_opt, band = gt.power_model_band(pmod, list(np.arange(500.0, 2400.0 + 1e-9, 5.0)), 0.1)
    assert f_opt == 1915.0 and band[0] == 1725.0 and band[-1] == 2105.0


def _synth(f, m):
    return opm.power(np.asarray(f), m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"])


@pytest.mark.parametrize("m", MODELS[:2])
def test_fit_recovers_noise_free(m):
    f = np.linspace(500.0, 2400.0, 9)
    r = gt.fit_power_model(f, _synth(f, m), m["p_max"])
    assert r.rss < 1e-12
    assert r.p_idle == pytest.approx(m["p_idle"], rel=1e-6)
    assert r.alpha == pytest.approx(m["alpha"], rel=1e-6)
    assert r.beta == pytest.approx(m["beta"], rel=1e-6)
    assert r.tau_mhz == pytest.approx(m["tau"], rel=1e-6)


@pytest.mark.parametrize("seed", range(6))
def test_fit_noisy_matches_oracle_sse(seed):
    rng = np.random.default_rng(seed)
    m = dict(p_idle=rng.uniform(100, 300), alpha=rng.uniform(0.05, 0.3), beta=rng.uniform(0.0005, 0.002),
             tau=rng.uniform(900, 1700), p_max=1e9)
    f = np.linspace(500.0, 2400.0, int(rng.integers(5, 10)))
    p = _synth(f, m) + rng.normal(0, 4.0, f.size)
    r = gt.fit_power_model(f, p, m["p_max"])
    o = opm.fit(f, p, m["p_max"])
    # the product's LM must reach the oracle's global least-squares minimum
    assert r.rss <= o["sse"] * (1 + 1e-6) + 1e-9
    # and report the SSE of the parameters it returns
    assert r.rss == pytest.approx(opm.sse((r.p_idle, r.alpha, r.beta, r.tau_mhz), f, p, m["p_max"]), rel=1e-9)


def test_fit_with_clipping():
    m = dict(p_idle=200.0, alpha=0.2, beta=0.0015, tau=1200.0, p_max=900.0)
    f = np.linspace(500.0, 2400.0, 11)
    p = _synth(f, m)
    r = gt.fit_power_model(f, p, m["p_max"])
    o = opm.fit(f, p, m["p_max"])
    assert r.rss <= o["sse"] * (1 + 1e-6) + 1e-9
    assert r.rss < 1e-8


def test_fit_measured_voltage():
    f = np.array([600.0, 1000.0, 1400.0, 1800.0, 2200.0])
    v = np.array([0.70, 0.70, 0.78, 0.90, 1.05])
    p = 120.0 + 0.3 * f * v * v
    r = gt.fit_power_model(f, p, 1e9, v=v)
    o = opm.fit(f, p, 1e9, v=v)
    assert r.v_measured == 1
    assert r.p_idle == pytest.approx(o["p_idle"], rel=1e-8)
    assert r.alpha == pytest.approx(o["alpha"], rel=1e-8)


def test_fit_rejects_bad_input():
    with pytest.raises(gt.GreentuneError):
        gt.fit_power_model([1000, 2000, 1500], [100, 200, 150], 1000.0)  # too few for Eq. 3
    with pytest.raises(gt.GreentuneError):
        gt.fit_power_model([1000, -5, 1500, 1200], [100, 200, 150, 120], 1000.0)


def test_dvfs_backend_registration_rules():
    # the library changes no device setting itself: knob changes go through a
    # caller-registered backend, which needs an apply function
    import ctypes
    b = gt.DvfsBackend(gt.DVFS_APPLY(), gt.DVFS_RESTORE(), None)
    assert gt.lib().gt_dvfs_set_backend(ctypes.byref(b)) == gt.GT_E_INVAL
    gt.set_dvfs_backend(lambda dev, kind, value: 0, lambda dev: 0)
    gt.set_dvfs_backend(None)


def test_sensor_stale_rule():
    t = [0.0, 0.2, 0.4, 0.6]
    assert gt.sensor_stale(t, [900.0] * 4, 0.5)            # unchanged over 0.6 s
    assert not gt.sensor_stale(t, [900.0, 900.0, 901.0, 900.0], 0.5)
    assert not gt.sensor_stale(t[:3], [900.0] * 3, 0.5)     # spans only 0.4 s
    assert not gt.sensor_stale([0.0], [900.0], 0.0)         # one reading proves nothing
    assert not gt.sensor_stale([], [], 0.5)


@pytest.mark.parametrize("seed", range(8))
def test_pareto_matches_oracle(seed):
    # values drawn from small sets, so exact ties in one or both objectives
    # are common; the library's sort-and-sweep must equal brute force
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    rows = [{"t_run": float(rng.integers(1, 8)), "e_run": float(rng.integers(1, 8))} for _ in range(n)]
    if seed == 0:
        rows = [{"t_run": 2.0, "e_run": 3.0}] * 4  # all identical: all on the front
    want = om.pareto_front(rows)
    got = gt.pareto([{"t_run_s": r["t_run"], "e_run_j": r["e_run"]} for r in rows])
    assert got == want


def test_pareto_empty_and_single():
    assert gt.pareto([]) == []
    assert gt.pareto([{"t_run_s": 1.0, "e_run_j": 1.0}]) == [0]


def _smp(t, sclk, mts, p=1000.0):
    return {"t_s": t, "power_w": p, "energy_j": 0.0, "energy_t_s": mts, "sclk_mhz": sclk, "mclk_mhz": 0.0,
            "volt_v": float("nan"), "temp_c": 50.0, "metrics_t_s": mts}


def test_window_clock_ignores_stale_pre_window_metrics():
    # metrics table refreshed at firmware times 10.0 (idle, 165 MHz), 11.0 and
    # 12.0 (loaded); the sensor re-reads it every few ms.  Kept window 0.5..2.5
    trace = ([_smp(0.01 * k, 165.0, 10.0) for k in range(80)]            # 0.00-0.79: idle table
             + [_smp(0.8 + 0.01 * k, 2100.0, 11.0) for k in range(100)]  # 0.80-1.79: first loaded table
             + [_smp(1.8 + 0.01 * k, 2300.0, 12.0) for k in range(100)])  # 1.80-2.79
    # both loaded updates are first seen inside the window: mean 2200
    f, n = gt.window_clock(trace, 0.5, 2.5)
    assert n == 2 and f == pytest.approx(2200.0, rel=1e-15)
    # a window opening after the first loaded update was seen counts only the
    # second one, though the first is still what the sensor reports at 1.0 s
    f, n = gt.window_clock(trace, 1.0, 2.5)
    assert n == 1 and f == 2300.0
    # a window with no refresh inside: NaN (the 165 MHz reading is never used)
    f, n = gt.window_clock(trace, 0.2, 0.7)
    assert n == 0 and f != f
    # no reading before the window: the first one in it only sets the
    # timestamp in force (it may predate the window)
    f, n = gt.window_clock(trace[30:], 0.0, 1.5)
    assert n == 1 and f == 2100.0


def test_window_clock_skips_invalid_timestamps_and_clocks():
    nan = float("nan")
    trace = [_smp(0.0, 500.0, 1.0), _smp(0.1, 900.0, nan), _smp(0.2, nan, 2.0), _smp(0.3, 1800.0, 3.0),
             _smp(0.4, 1900.0, 3.0)]
    f, n = gt.window_clock(trace, 0.05, 1.0)
    assert n == 1 and f == 1800.0  # 2.0 carries no clock, 3.0 counts once


@pytest.mark.parametrize("seed", range(5))
def test_fit_covariance_matches_oracle(seed):
    # s^2 (J^T J)^-1 at the fitted parameters: the library's (from its own
    # fit) against the oracle's (from the oracle's fit of the same readings)
    rng = np.random.default_rng(100 + seed)
    m = dict(p_idle=rng.uniform(100, 300), alpha=rng.uniform(0.05, 0.3), beta=rng.uniform(0.0005, 0.002),
             tau=rng.uniform(900, 1500), p_max=1e9)
    f = np.linspace(500.0, 2400.0, 7)
    p = _synth(f, m) + rng.normal(0, 3.0, f.size)
    r = gt.fit_power_model(f, p, m["p_max"])
    o = opm.fit(f, p, m["p_max"])
    assert r.rss == pytest.approx(o["sse"], rel=1e-6)
    co = opm.covariance(f, p, o)
    cr = np.array(r.covariance())
    assert np.all(np.isfinite(co)) and np.all(np.isfinite(cr))
    assert np.allclose(cr, co, rtol=2e-3, atol=0), (cr, co)


def test_fit_covariance_measured_voltage_and_undefined():
    f = np.array([600.0, 1000.0, 1400.0, 1800.0, 2200.0])
    v = np.array([0.70, 0.72, 0.80, 0.92, 1.05])
    p = 120.0 + 0.3 * f * v * v + np.array([2.0, -3.0, 1.0, 4.0, -2.5])
    r = gt.fit_power_model(f, p, 1e9, v=v)
    o = opm.fit(f, p, 1e9, v=v)
    cr, co = np.array(r.covariance()), opm.covariance(f, p, o, v=v)
    assert np.allclose(cr[:2, :2], co[:2, :2], rtol=1e-8)
    assert np.all(np.isnan(cr[2:, :])) and np.all(np.isnan(cr[:, 2:]))
    # four readings for four parameters: no degrees of freedom left
    r4 = gt.fit_power_model(f[:4], p[:4] * 0 + _synth(f[:4], dict(p_idle=150, alpha=0.2, beta=1e-3, tau=1100,
                                                                   p_max=1e9)), 1e9)
    assert np.all(np.isnan(np.array(r4.covariance())))


def test_igemm_batch_pack_host():
    # descriptors of the batched multi-channel launch: one per convolution,
    # blocks of 256 output pixels, first-block indices in order
    import ctypes
    lib = gt.lib()
    shape = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, 1, 1, 32, 32, 5, 5)
    sides = [(1, 1), (16, 16), (17, 15), (100, 3), (257, 1)]
    items = (gt.BatchItem * len(sides))()
    for k, (oh, ow) in enumerate(sides):
        items[k] = gt.BatchItem(0x10000 * (k + 1), 0x20000000 + 0x100 * k, 0x30000000, oh, ow, 5, 5)
    nb, tb = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert lib.gt_igemm_batch_pack(ctypes.byref(shape), items, len(sides), None, 0, ctypes.byref(nb),
                                   ctypes.byref(tb)) == gt.GT_E_CAPACITY
    blocks = [-(-oh * ow // 256) for oh, ow in sides]
    assert nb.value == 64 * len(sides) and tb.value == sum(blocks)
    blob = (ctypes.c_uint8 * nb.value)()
    assert lib.gt_igemm_batch_pack(ctypes.byref(shape), items, len(sides), blob, nb.value, ctypes.byref(nb),
                                   ctypes.byref(tb)) == gt.GT_OK
    raw = bytes(blob)
    begin = 0
    for k, (oh, ow) in enumerate(sides):
        rec = raw[64 * k:64 * (k + 1)]
        h, wd, o_h, o_w, ph, pw, m, n = np.frombuffer(rec[24:56], dtype=np.int32)
        assert (h, wd, o_h, o_w, ph, pw, m, n) == (oh, ow, oh, ow, 2, 2, oh * ow, 1)  # same padding
        assert np.frombuffer(rec[56:64], dtype=np.int64)[0] == begin
        begin += blocks[k]
    # rejections: unaligned input, filter mismatch, channels not instantiated, BF16 only
    bad = (gt.BatchItem * 1)(gt.BatchItem(0x10008, 0x20000, 0x30000, 4, 4, 5, 5))
    assert lib.gt_igemm_batch_pack(ctypes.byref(shape), bad, 1, None, 0, ctypes.byref(nb),
                                   ctypes.byref(tb)) == gt.GT_E_INVAL
    bad = (gt.BatchItem * 1)(gt.BatchItem(0x10000, 0x20000, 0x30000, 4, 4, 3, 3))
    assert lib.gt_igemm_batch_pack(ctypes.byref(shape), bad, 1, None, 0, ctypes.byref(nb),
                                   ctypes.byref(tb)) == gt.GT_E_INVAL
    for sh in (gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, 1, 1, 48, 32, 5, 5),
               gt.conv_problem(gt.IGEMM_F32_VALU, 1, 1, 1, 32, 64, 5, 5)):
        assert lib.gt_igemm_batch_pack(ctypes.byref(sh), items, len(sides), None, 0, ctypes.byref(nb),
                                       ctypes.byref(tb)) == gt.GT_E_UNSUPPORTED


def test_binding_refuses_short_or_strided_tensors():
    """The binding checks each tensor against the problem's dense extent
    before a pointer reaches the library (the kernels read and write that
    many bytes from it)."""
    import torch
    p = gt.xcorr_problem(8, 10, 3, 3)
    assert gt.buffer_extents(p) == (10 * 12 * 4, 9 * 4, 8 * 10 * 4)
    img, w, out = torch.zeros(10, 12), torch.zeros(3, 3), torch.zeros(8, 10)
    gt.check_buffers(p, img, w, out)
    with pytest.raises(ValueError, match="output"):
        gt.check_buffers(p, img, w, torch.zeros(8, 9))
    with pytest.raises(ValueError, match="input"):
        gt.check_buffers(p, torch.zeros(20, 24)[1:11, :12], w, out)  # a strided view
    big = torch.zeros(10 * 12 + 5)
    gt.check_buffers(p, big[5:].view(10, 12), w, out)                 # a contiguous view at an offset
    with pytest.raises(ValueError, match="input"):
        gt.check_buffers(p, big[6:], w, out)
    q = gt.Problem(gt.IGEMM_BF16_MFMA, 2, 32, 64, 6, 7, 3, 3, 1, 1)
    assert gt.buffer_extents(q) == (2 * 6 * 7 * 32 * 2, 64 * 9 * 32 * 2, 2 * 6 * 7 * 64 * 4)
    assert gt.buffer_extents(gt.xcorr_problem(0, 4, 3, 3)) is None  # the library rejects it itself
