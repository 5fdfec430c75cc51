"""greentune: energy-aware auto-tuning of a parameterised 2-D convolution on
one MI355X, after "Going green: optimizing GPUs for energy efficiency through
model-steered auto-tuning".

This module is a thin ctypes binding over ``libgreentune.so`` (C ABI in
``include/greentune.h``): it marshals arguments and nothing else.  Every step
of the method runs in the native library and its HIP kernels; torch tensors
only provide device memory and streams.  If the native library is missing the
import fails loudly -- there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# GREENTUNE_LIB selects another build of the same library (the host-sanitizer
# build of the tests); by default the one built in this package directory
LIB_PATH = os.environ.get("GREENTUNE_LIB") or os.path.join(_HERE, "libgreentune.so")

# ---- constants mirrored from include/greentune.h ----
GT_OK, GT_E_INVAL, GT_E_UNSUPPORTED, GT_E_PERM = 0, -1, -2, -3
GT_E_SENSOR, GT_E_HIP, GT_E_NOMEM, GT_E_CAPACITY, GT_E_STATE = -4, -5, -6, -7, -8
XCORR_F32, IGEMM_BF16_MFMA, IGEMM_F32_VALU = 0, 1, 2
CLOCK_DEFAULT, CLOCK_SCLK_MHZ, CLOCK_POWER_CAP_W = 0, 1, 2
SPACE_DEDUP_DIRECT = 1
INIT_FAKE_SENSOR, INIT_FAKE_DVFS, INIT_ALLOW_DVFS, INIT_HOST_ONLY = 1, 2, 4, 8
CONFIG_FIELDS = ("block_size_x", "block_size_y", "tile_size_x", "tile_size_y",
                 "use_lds_padding", "read_path")


class GreentuneError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("greentune error %d: %s" % (code, msg))
        self.code = code


class ConvConfig(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in CONFIG_FIELDS]

    def as_tuple(self):
        return tuple(getattr(self, n) for n in CONFIG_FIELDS)

    def __repr__(self):
        return "ConvConfig(%s)" % ", ".join("%s=%d" % (n, getattr(self, n)) for n in CONFIG_FIELDS)


class Problem(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("kind", "n", "c_in", "c_out", "out_h", "out_w",
                                             "filt_h", "filt_w", "pad_h", "pad_w")]


class Clock(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("value", ctypes.c_int32)]


class SpaceDesc(ctypes.Structure):
    _fields_ = [("values", ctypes.POINTER(ctypes.c_int32) * 6), ("counts", ctypes.c_int32 * 6),
                ("flags", ctypes.c_uint32), ("max_threads", ctypes.c_int32),
                ("lds_limit_bytes", ctypes.c_int64)]


DVFS_APPLY = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32)
DVFS_RESTORE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32)


class DvfsBackend(ctypes.Structure):
    _fields_ = [("apply", DVFS_APPLY), ("restore", DVFS_RESTORE), ("user", ctypes.c_void_p)]


class MeasureOpts(ctypes.Structure):
    _fields_ = [("window_s", ctypes.c_double), ("discard_s", ctypes.c_double),
                ("sample_period_ms", ctypes.c_double), ("min_launches", ctypes.c_int32),
                ("warmup_launches", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


_MEAS_D = ("t_run_s", "p_median_w", "p_min_w", "p_max_w", "e_run_j", "e_run_counter_j", "gflops",
           "gflops_per_w", "sclk_req_mhz", "sclk_act_mhz", "mclk_mhz", "volt_v", "temp_c", "window_s")


class Measurement(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_double) for n in _MEAS_D]
                + [("launches", ctypes.c_int64), ("n_samples", ctypes.c_int64), ("n_used", ctypes.c_int64),
                   ("throttled", ctypes.c_int32), ("flags", ctypes.c_int32)])

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class PowerModel(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("p_idle", "alpha", "beta", "tau_mhz", "p_max", "rss")] + \
               [("cov", ctypes.c_double * 16)] + \
               [(n, ctypes.c_int32) for n in ("v_measured", "literal_eq3", "iters", "status")]

    def covariance(self):
        """4 x 4 covariance of (p_idle, alpha, beta, tau_mhz) as nested lists."""
        return [[self.cov[4 * i + j] for j in range(4)] for i in range(4)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "cov"}
        d["cov"] = self.covariance()
        return d


class BatchItem(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("d_filt", ctypes.c_void_p), ("d_out", ctypes.c_void_p),
                ("out_h", ctypes.c_int32), ("out_w", ctypes.c_int32), ("filt_h", ctypes.c_int32),
                ("filt_w", ctypes.c_int32)]


class SensorSample(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("t_s", "power_w", "energy_j", "energy_t_s", "sclk_mhz",
                                               "mclk_mhz", "volt_v", "temp_c", "metrics_t_s")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as fh:
            maps = fh.read()
    except OSError:
        return set()
    return {ln.split()[-1] for ln in maps.splitlines() if "libamdhip64" in ln}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgreentune.so is not built (run paper_2211_07260_amd/build.py)")
    # torch's HIP runtime must be the one the library binds to: load it first so
    # the library's libamdhip64 dependency resolves to the already-loaded copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are loaded (%s); the library must share torch's" % sorted(rts))
    P, c_int, c_double, c_size = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    vp = ctypes.c_void_p
    sig = {
        "gt_init": ([c_int, ctypes.c_uint32], c_int),
        "gt_shutdown": ([], c_int),
        "gt_last_error": ([], ctypes.c_char_p),
        "gt_version": ([], ctypes.c_char_p),
        "conv2d_run": ([P(Problem), P(ConvConfig), Clock, vp, vp, vp, vp], c_int),
        "conv2d_run_part": ([P(Problem), P(ConvConfig), Clock, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp], c_int),
        "tune_space_enumerate": ([P(Problem), P(SpaceDesc), P(ConvConfig), c_size, P(c_size)], c_int),
        "measure_time_energy": ([P(Problem), P(ConvConfig), Clock, P(MeasureOpts), vp, vp, vp, vp,
                                 P(Measurement)], c_int),
        "measure_load": ([ctypes.c_int32, Clock, P(MeasureOpts), vp, c_size, vp, P(Measurement)], c_int),
        "fit_power_model": ([P(c_double), P(c_double), P(c_double), c_size, c_double, P(PowerModel)], c_int),
        "gt_power_model_eval": ([P(PowerModel), c_double], c_double),
        "gt_power_model_throttle_clock": ([P(PowerModel)], c_double),
        "gt_power_model_band": ([P(PowerModel), P(c_double), c_size, c_double, P(c_double), P(c_double),
                                 c_size, P(c_size)], c_int),
        "gt_energy_from_samples": ([P(c_double), P(c_double), c_size, c_double, c_double, ctypes.c_int64,
                                    c_double, P(c_double), P(c_double), P(c_size)], c_int),
        "gt_select": ([P(Measurement), c_size, c_int, P(c_size)], c_int),
        "gt_pareto": ([P(Measurement), c_size, P(ctypes.c_int32)], c_int),
        "gt_window_clock": ([P(SensorSample), c_size, c_double, c_double, P(c_double), P(c_size)], c_int),
        "gt_measure_last_window": ([P(SensorSample), c_size, P(c_size), P(c_double), P(c_double)], c_int),
        "gt_problem_flops": ([P(Problem)], c_double),
        "gt_conv_lds_bytes": ([P(Problem), P(ConvConfig), P(ctypes.c_int64)], c_int),
        "gt_sensor_read": ([P(SensorSample)], c_int),
        "gt_settable_clocks": ([c_double, P(c_double), c_size, P(c_size)], c_int),
        "gt_dvfs_state": ([P(Clock)], c_int),
        "gt_power_cap_range": ([P(c_double), P(c_double), P(c_double)], c_int),
        "gt_dvfs_set_backend": ([P(DvfsBackend)], c_int),
        "gt_sensor_stale": ([P(c_double), P(c_double), c_size, c_double], c_int),
        "gt_fake_sensor_model": ([P(PowerModel), c_double, ctypes.c_uint64], c_int),
        "gt_roofline_probe": ([vp, c_size, vp, P(c_double), P(c_double)], c_int),
        "gt_mfma_probe": ([vp, c_size, vp, P(c_double), P(c_double)], c_int),
        "gt_batch_pack": ([P(BatchItem), ctypes.c_int32, P(ConvConfig), vp, c_size, P(c_size),
                           P(ctypes.c_int64)], c_int),
        "conv2d_run_batched": ([vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P(ConvConfig),
                                ctypes.c_int32, vp], c_int),
        "conv2d_run_batched_noalloc": ([P(BatchItem), ctypes.c_int32, P(ConvConfig), ctypes.c_int32, vp], c_int),
        "gt_igemm_batch_pack": ([P(Problem), P(BatchItem), ctypes.c_int32, vp, c_size, P(c_size),
                                 P(ctypes.c_int64)], c_int),
        "conv2d_run_igemm_batched": ([P(Problem), vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, vp], c_int),
        "measure_batched_time_energy": ([vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P(ConvConfig),
                                         ctypes.c_int32, c_double, Clock, P(MeasureOpts), vp, P(Measurement)], c_int),
        "gt_graph_begin": ([vp], c_int),
        "gt_graph_end": ([vp, P(vp)], c_int),
        "gt_graph_launch": ([vp, vp], c_int),
        "gt_graph_destroy": ([vp], c_int),
        "gt_sampler_start": ([c_double], c_int),
        "gt_sampler_stop": ([P(SensorSample), c_size, P(c_size)], c_int),
        "gt_sensor_busy": ([c_int], c_int),
        "gt_ffg_centrality": ([P(ConvConfig), P(c_double), c_size, c_double, P(c_double), c_size, P(c_double),
                               P(ctypes.c_int32), P(c_double)], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED = ("gt_init", "gt_shutdown", "gt_last_error", "gt_version", "conv2d_run", "conv2d_run_part",
            "tune_space_enumerate", "measure_time_energy", "measure_load", "fit_power_model", "gt_power_model_eval", "gt_power_model_throttle_clock",
            "gt_power_model_band", "gt_energy_from_samples", "gt_select", "gt_pareto", "gt_window_clock",
            "gt_measure_last_window", "gt_problem_flops",
            "gt_conv_lds_bytes", "gt_sensor_read", "gt_settable_clocks", "gt_dvfs_state", "gt_power_cap_range", "gt_dvfs_set_backend", "gt_sensor_stale",
            "gt_fake_sensor_model", "gt_roofline_probe", "gt_mfma_probe", "gt_batch_pack", "conv2d_run_batched",
            "conv2d_run_batched_noalloc", "measure_batched_time_energy", "gt_igemm_batch_pack",
            "conv2d_run_igemm_batched",
            "gt_graph_begin", "gt_graph_end", "gt_graph_launch", "gt_graph_destroy", "gt_sampler_start",
            "gt_sampler_stop", "gt_sensor_busy", "gt_ffg_centrality")


def lib():
    return _lib


def _check(rc):
    if rc != GT_OK:
        raise GreentuneError(rc, _lib.gt_last_error().decode())
    return rc


def _darr(values):
    vals = [float(v) for v in values]
    return (ctypes.c_double * max(len(vals), 1))(*vals), len(vals)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ---- problems and configs ----

def xcorr_problem(out_h, out_w, fh, fw):
    return Problem(XCORR_F32, 1, 1, 1, out_h, out_w, fh, fw, 0, 0)


def conv_problem(kind, n, h, w, c_in, c_out, fh, fw):
    """Multi-channel conv, stride 1, same padding (output h x w)."""
    return Problem(kind, n, c_in, c_out, h, w, fh, fw, (fh - 1) // 2, (fw - 1) // 2)


def config(block_size_x=32, block_size_y=8, tile_size_x=4, tile_size_y=4, use_lds_padding=0, read_path=0):
    return ConvConfig(block_size_x, block_size_y, tile_size_x, tile_size_y, use_lds_padding, read_path)


def as_config(c):
    if isinstance(c, ConvConfig):
        return c
    if isinstance(c, dict):
        return config(**c)
    return ConvConfig(*c)


def clock(kind=CLOCK_DEFAULT, value=0):
    return Clock(kind, int(value))


# ---- lifecycle ----

def init(device=0, flags=0):
    return _check(_lib.gt_init(device, flags))


def shutdown():
    return _check(_lib.gt_shutdown())


def version():
    return _lib.gt_version().decode()


# ---- the four calls ----

def buffer_extents(problem):
    """Bytes the dense input, filter and output of a problem span (None for
    sizes the library rejects anyway)."""
    p = problem
    if min(p.n, p.c_in, p.c_out, p.out_h, p.out_w, p.filt_h, p.filt_w) < 1 or min(p.pad_h, p.pad_w) < 0:
        return None
    if p.kind == XCORR_F32:
        return ((p.out_h + p.filt_h - 1) * (p.out_w + p.filt_w - 1) * 4, p.filt_h * p.filt_w * 4,
                p.out_h * p.out_w * 4)
    eb = 2 if p.kind == IGEMM_BF16_MFMA else 4
    h, w = p.out_h + p.filt_h - 1 - 2 * p.pad_h, p.out_w + p.filt_w - 1 - 2 * p.pad_w
    if h < 1 or w < 1:
        return None
    return (p.n * h * w * p.c_in * eb, p.c_out * p.filt_h * p.filt_w * p.c_in * eb, p.n * p.out_h * p.out_w * p.c_out * 4)


def check_buffers(problem, inp, filt, out):
    """Refuse tensors that are not contiguous or end before the problem's
    dense extent: the kernels read and write that many bytes from each
    pointer.  (Raw integer pointers are passed through unchecked.)"""
    ext = buffer_extents(problem)
    if ext is None:
        return
    for t, need, name in zip((inp, filt, out), ext, ("input", "filter", "output")):
        if not hasattr(t, "is_contiguous"):
            continue
        if not t.is_contiguous():
            raise ValueError("%s tensor must be contiguous" % name)
        have = t.numel() * t.element_size()
        if have < need:
            raise ValueError("%s tensor holds %d bytes; the problem needs %d" % (name, have, need))


def conv2d_run(problem, cfg, inp, filt, out, clk=None, stream=None):
    check_buffers(problem, inp, filt, out)
    _check(_lib.conv2d_run(ctypes.byref(problem), ctypes.byref(as_config(cfg)), clk or clock(),
                           _ptr(inp), _ptr(filt), _ptr(out), _stream(stream)))


def conv2d_run_part(problem, cfg, part, n_parts, inp, filt, out, clk=None, stream=None):
    """Part `part` of `n_parts` of conv2d_run (contiguous ranges of output
    tiles; bit-identical to the whole run)."""
    check_buffers(problem, inp, filt, out)
    _check(_lib.conv2d_run_part(ctypes.byref(problem), ctypes.byref(as_config(cfg)), clk or clock(), int(part),
                                int(n_parts), _ptr(inp), _ptr(filt), _ptr(out), _stream(stream)))


def tune_space_enumerate(problem, values, max_threads=0, lds_limit=0, dedup_direct=True):
    """values: dict name -> list of ints for the six tunables."""
    arrs = [(ctypes.c_int32 * len(values[n]))(*values[n]) for n in CONFIG_FIELDS]
    d = SpaceDesc()
    for k, a in enumerate(arrs):
        d.values[k] = ctypes.cast(a, ctypes.POINTER(ctypes.c_int32))
        d.counts[k] = len(a)
    d.flags = SPACE_DEDUP_DIRECT if dedup_direct else 0
    d.max_threads = max_threads
    d.lds_limit_bytes = lds_limit
    n = ctypes.c_size_t(0)
    rc = _lib.tune_space_enumerate(ctypes.byref(problem), ctypes.byref(d), None, 0, ctypes.byref(n))
    if rc not in (GT_OK, GT_E_CAPACITY):
        _check(rc)
    out = (ConvConfig * max(n.value, 1))()
    _check(_lib.tune_space_enumerate(ctypes.byref(problem), ctypes.byref(d), out, n.value, ctypes.byref(n)))
    return [out[k] for k in range(n.value)]


def measure_time_energy(problem, cfg, inp, filt, out, clk=None, window_s=1.0, discard_s=0.3,
                        sample_period_ms=1.0, min_launches=10, warmup_launches=3, stream=None, use_graph=False):
    check_buffers(problem, inp, filt, out)
    o = MeasureOpts(window_s, discard_s, sample_period_ms, min_launches, warmup_launches, 1 if use_graph else 0)
    m = Measurement()
    _check(_lib.measure_time_energy(ctypes.byref(problem), ctypes.byref(as_config(cfg)), clk or clock(),
                                    ctypes.byref(o), _ptr(inp), _ptr(filt), _ptr(out), _stream(stream),
                                    ctypes.byref(m)))
    return m.as_dict()


LOAD_FP32_FMA, LOAD_BF16_MFMA, LOAD_COPY = 0, 1, 2


def measure_load(kind, buf, clk=None, window_s=1.0, discard_s=0.3, sample_period_ms=1.0, min_launches=10,
                 warmup_launches=3, stream=None):
    """Time and energy of a synthetic full-load kernel (LOAD_*) at a clock;
    buf: device tensor of >= 4 MiB (overwritten).  'gflops' is GB/s for the
    copy load."""
    o = MeasureOpts(window_s, discard_s, sample_period_ms, min_launches, warmup_launches)
    m = Measurement()
    _check(_lib.measure_load(int(kind), clk or clock(), ctypes.byref(o), _ptr(buf), buf.numel() * buf.element_size(),
                             _stream(stream), ctypes.byref(m)))
    return m.as_dict()


def fit_power_model(f_mhz, p_w, p_max, v=None, literal=False):
    fa, n = _darr(f_mhz)
    pa, n2 = _darr(p_w)
    if n != n2:
        raise ValueError("f and p differ in length")
    va = _darr(v)[0] if v is not None else None
    m = PowerModel()
    m.literal_eq3 = 1 if literal else 0
    _check(_lib.fit_power_model(fa, pa, va, n, float(p_max), ctypes.byref(m)))
    return m


def power_model_eval(model, f_mhz):
    return _lib.gt_power_model_eval(ctypes.byref(model), float(f_mhz))


def power_model_throttle_clock(model):
    return _lib.gt_power_model_throttle_clock(ctypes.byref(model))


def power_model_band(model, settable, rel_half=0.1):
    sa, n = _darr(settable)
    f_opt = ctypes.c_double(0)
    band = (ctypes.c_double * max(n, 1))()
    nb = ctypes.c_size_t(0)
    _check(_lib.gt_power_model_band(ctypes.byref(model), sa, n, rel_half, ctypes.byref(f_opt), band, n,
                                    ctypes.byref(nb)))
    return f_opt.value, [band[k] for k in range(nb.value)]


def energy_from_samples(t_s, p_w, t_start, t_stop, n_runs, discard_s):
    ta, n = _darr(t_s)
    pa, _ = _darr(p_w)
    e, pm, nu = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_size_t(0)
    _check(_lib.gt_energy_from_samples(ta, pa, n, t_start, t_stop, int(n_runs), discard_s,
                                       ctypes.byref(e), ctypes.byref(pm), ctypes.byref(nu)))
    return e.value, pm.value, nu.value


def select(records, objective):
    """records: list of dicts with t_run_s and e_run_j; objective 'time' | 'energy'."""
    arr = (Measurement * len(records))()
    for k, r in enumerate(records):
        arr[k].t_run_s = r["t_run_s"]
        arr[k].e_run_j = r["e_run_j"]
    idx = ctypes.c_size_t(0)
    _check(_lib.gt_select(arr, len(records), {"time": 0, "energy": 1}[objective], ctypes.byref(idx)))
    return idx.value


def pareto(records):
    """Indices of the records not dominated in (t_run_s, e_run_j), both
    minimised (the GFLOP/s versus GFLOP/s/W front), ascending."""
    arr = (Measurement * max(len(records), 1))()
    for k, r in enumerate(records):
        arr[k].t_run_s = r["t_run_s"]
        arr[k].e_run_j = r["e_run_j"]
    flags = (ctypes.c_int32 * max(len(records), 1))()
    _check(_lib.gt_pareto(arr, len(records), flags))
    return [k for k in range(len(records)) if flags[k]]


def _samples(samples):
    arr = (SensorSample * max(len(samples), 1))()
    nan = float("nan")
    for k, d in enumerate(samples):
        for n, _ in SensorSample._fields_:
            setattr(arr[k], n, float(d.get(n, nan)))
    return arr


def window_clock(samples, t_lo, t_hi):
    """(mean graphics clock of the GPU-metrics updates first seen in
    [t_lo, t_hi], number of such updates); NaN when there is none."""
    f, nf = ctypes.c_double(0), ctypes.c_size_t(0)
    _check(_lib.gt_window_clock(_samples(samples), len(samples), float(t_lo), float(t_hi), ctypes.byref(f),
                                ctypes.byref(nf)))
    return f.value, nf.value


def measure_last_window(capacity=1 << 16):
    """(readings, t_start, t_stop) of the most recent measurement window."""
    arr = (SensorSample * capacity)()
    n, t0, t1 = ctypes.c_size_t(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(_lib.gt_measure_last_window(arr, capacity, ctypes.byref(n), ctypes.byref(t0), ctypes.byref(t1)))
    return [arr[k].as_dict() for k in range(n.value)], t0.value, t1.value


def problem_flops(problem):
    return _lib.gt_problem_flops(ctypes.byref(problem))


def lds_bytes(problem, cfg):
    b = ctypes.c_int64(0)
    _check(_lib.gt_conv_lds_bytes(ctypes.byref(problem), ctypes.byref(as_config(cfg)), ctypes.byref(b)))
    return b.value


def sensor_read():
    s = SensorSample()
    _check(_lib.gt_sensor_read(ctypes.byref(s)))
    return s.as_dict()


def settable_clocks(step_mhz=25.0):
    n = ctypes.c_size_t(0)
    rc = _lib.gt_settable_clocks(step_mhz, None, 0, ctypes.byref(n))
    if rc not in (GT_OK, GT_E_CAPACITY):
        _check(rc)
    arr = (ctypes.c_double * max(n.value, 1))()
    _check(_lib.gt_settable_clocks(step_mhz, arr, n.value, ctypes.byref(n)))
    return [arr[k] for k in range(n.value)]


def sensor_stale(t_s, p_w, min_span_s=0.5):
    """True when a power trace spanning >= min_span_s never changes."""
    ta, n = _darr(t_s)
    pa, n2 = _darr(p_w)
    if n != n2:
        raise ValueError("t and p differ in length")
    rc = _lib.gt_sensor_stale(ta, pa, n, float(min_span_s))
    if rc < 0:
        _check(rc)
    return rc == 1


def power_cap_range():
    """(min, max, current) power cap in W (amd-smi, or the fake backend's)."""
    lo, hi, cur = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(_lib.gt_power_cap_range(ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(cur)))
    return lo.value, hi.value, cur.value


_backend_refs = []


def set_dvfs_backend(apply, restore=None):
    """Register the functions that change the device's DVFS knob (the library
    changes no device setting itself): apply(device_ordinal, kind, value) ->
    0 on success, restore(device_ordinal) -> 0.  None unregisters."""
    if apply is None:
        _check(_lib.gt_dvfs_set_backend(None))
        _backend_refs.clear()
        return
    a = DVFS_APPLY(lambda user, dev, kind, value: int(apply(dev, kind, value)))
    r = DVFS_RESTORE(lambda user, dev: int(restore(dev))) if restore else DVFS_RESTORE()
    b = DvfsBackend(a, r, None)
    _check(_lib.gt_dvfs_set_backend(ctypes.byref(b)))
    if not _backend_refs:
        import atexit
        atexit.register(_lib.gt_shutdown)  # restore the knob on a normal exit
        _restore_on_sigterm()
    _backend_refs[:] = [a, r, b]


def _restore_on_sigterm():
    """A terminated tuner restores the DVFS knob too: SIGTERM (the default
    action ends the process without running atexit) first calls
    gt_shutdown, then the handler that was installed before, or the default
    action.  Only from the main thread, where Python allows handlers."""
    import signal
    import threading
    if threading.current_thread() is not threading.main_thread():
        return
    prev = signal.getsignal(signal.SIGTERM)

    def handler(signum, frame):
        _lib.gt_shutdown()
        if callable(prev):
            prev(signum, frame)
        else:
            signal.signal(signum, signal.SIG_DFL)
            os.kill(os.getpid(), signum)
    signal.signal(signal.SIGTERM, handler)


def dvfs_state():
    c = Clock()
    active = _lib.gt_dvfs_state(ctypes.byref(c))
    return bool(active), (c.kind, c.value)


def fake_sensor_model(model, noise_w=0.0, seed=0):
    _check(_lib.gt_fake_sensor_model(ctypes.byref(model), float(noise_w), int(seed)))


def power_model(p_idle, alpha, beta, tau_mhz, p_max, literal=False):
    m = PowerModel()
    m.p_idle, m.alpha, m.beta, m.tau_mhz, m.p_max = p_idle, alpha, beta, tau_mhz, p_max
    m.literal_eq3 = 1 if literal else 0
    return m


def roofline_probe(buf, stream=None):
    """Achievable FP32 FMA TFLOP/s and copy GB/s on this device (buf: device
    tensor of >= 4 MiB, overwritten)."""
    t, g = ctypes.c_double(0), ctypes.c_double(0)
    _check(_lib.gt_roofline_probe(_ptr(buf), buf.numel() * buf.element_size(), _stream(stream),
                                  ctypes.byref(t), ctypes.byref(g)))
    return t.value, g.value


def mfma_probe(buf, stream=None):
    """BF16 16x16x32 MFMA TFLOP/s with one and with two waves per SIMD (buf:
    device tensor of >= 2 KiB per CU, overwritten)."""
    t1, t2 = ctypes.c_double(0), ctypes.c_double(0)
    _check(_lib.gt_mfma_probe(_ptr(buf), buf.numel() * buf.element_size(), _stream(stream),
                              ctypes.byref(t1), ctypes.byref(t2)))
    return t1.value, t2.value


# ---- batching ----

class Batch:
    """A packed batch of single-channel convolutions sharing one filter size
    and config.  convs: list of (d_in, d_filt, d_out, out_h, out_w, f) with
    torch device tensors.  The descriptor blob lives in a device tensor owned
    by this object; its upload is queued on the stream current at
    construction, so run() on that stream, or order the other stream after it
    (e.g. a synchronize) before the first run."""

    def __init__(self, convs, cfg):
        import torch
        self.cfg = as_config(cfg)
        items = (BatchItem * len(convs))()
        for k, (di, dw, do, oh, ow, f) in enumerate(convs):
            check_buffers(xcorr_problem(oh, ow, f, f), di, dw, do)
            items[k] = BatchItem(di.data_ptr(), dw.data_ptr(), do.data_ptr(), oh, ow, f, f)
        self.n = len(convs)
        self.filt = convs[0][5]
        nb, tt = ctypes.c_size_t(0), ctypes.c_int64(0)
        rc = _lib.gt_batch_pack(items, self.n, ctypes.byref(self.cfg), None, 0, ctypes.byref(nb), ctypes.byref(tt))
        if rc not in (GT_OK, GT_E_CAPACITY):
            _check(rc)
        # pinned staging so the upload is asynchronous on the current stream;
        # kept alive with the batch until the copy has certainly run
        self._host = torch.empty(nb.value, dtype=torch.uint8, pin_memory=True)
        _check(_lib.gt_batch_pack(items, self.n, ctypes.byref(self.cfg), ctypes.c_void_p(self._host.data_ptr()),
                                  nb.value, ctypes.byref(nb), ctypes.byref(tt)))
        self.total_tiles = tt.value
        self.blob = self._host.to(convs[0][0].device, non_blocking=True)
        self._keep = convs  # the device buffers must outlive the batch

    def run(self, grid_blocks=0, stream=None):
        _check(_lib.conv2d_run_batched(_ptr(self.blob), self.n, self.total_tiles, self.filt, ctypes.byref(self.cfg),
                                       grid_blocks, _stream(stream)))

    def flops(self):
        return sum(2.0 * oh * ow * f * f for (_, _, _, oh, ow, f) in self._keep)

    def measure(self, clk=None, window_s=1.0, discard_s=0.3, sample_period_ms=1.0, min_launches=10,
                warmup_launches=3, grid_blocks=0, stream=None, use_graph=False):
        """measure_batched_time_energy of this batch: time and energy per
        launch of the whole batch over a window."""
        o = MeasureOpts(window_s, discard_s, sample_period_ms, min_launches, warmup_launches, 1 if use_graph else 0)
        m = Measurement()
        _check(_lib.measure_batched_time_energy(_ptr(self.blob), self.n, self.total_tiles, self.filt,
                                                ctypes.byref(self.cfg), int(grid_blocks), self.flops(),
                                                clk or clock(), ctypes.byref(o), _stream(stream), ctypes.byref(m)))
        return m.as_dict()


class IgemmBatch:
    """A packed batch of multi-channel BF16 convolutions of one shape family
    (c_in, c_out, square filter f, padding pad; one image each).  convs: list
    of (d_in, d_filt, d_out, out_h, out_w) with torch device tensors (NHWC
    BF16 input, KRSC BF16 weights, NHWC FP32 output).  Descriptor upload as
    for Batch."""

    def __init__(self, convs, c_in, c_out, f, pad):
        import torch
        self.shape = conv_problem(IGEMM_BF16_MFMA, 1, 1, 1, c_in, c_out, f, f)
        self.shape.pad_h = self.shape.pad_w = int(pad)
        items = (BatchItem * len(convs))()
        for k, (di, dw, do, oh, ow) in enumerate(convs):
            check_buffers(Problem(IGEMM_BF16_MFMA, 1, c_in, c_out, oh, ow, f, f, int(pad), int(pad)), di, dw, do)
            items[k] = BatchItem(di.data_ptr(), dw.data_ptr(), do.data_ptr(), oh, ow, f, f)
        self.n = len(convs)
        nb, tb = ctypes.c_size_t(0), ctypes.c_int64(0)
        rc = _lib.gt_igemm_batch_pack(ctypes.byref(self.shape), items, self.n, None, 0, ctypes.byref(nb),
                                      ctypes.byref(tb))
        if rc not in (GT_OK, GT_E_CAPACITY):
            _check(rc)
        self._host = torch.empty(nb.value, dtype=torch.uint8, pin_memory=True)
        _check(_lib.gt_igemm_batch_pack(ctypes.byref(self.shape), items, self.n,
                                        ctypes.c_void_p(self._host.data_ptr()), nb.value, ctypes.byref(nb),
                                        ctypes.byref(tb)))
        self.total_blocks = tb.value
        self.blob = self._host.to(convs[0][0].device, non_blocking=True)
        self._keep = convs

    def flops(self):
        c_in, c_out, f = self.shape.c_in, self.shape.c_out, self.shape.filt_h
        return sum(2.0 * oh * ow * c_in * c_out * f * f for (_, _, _, oh, ow) in self._keep)

    def run(self, grid_blocks=0, stream=None):
        _check(_lib.conv2d_run_igemm_batched(ctypes.byref(self.shape), _ptr(self.blob), self.n, self.total_blocks,
                                             int(grid_blocks), _stream(stream)))


BATCH_NOALLOC_MAX_ITEMS = 4096


def conv2d_run_batched_noalloc(convs, cfg, grid_blocks=0, stream=None):
    """The batched launch without a descriptor blob: the library writes the
    descriptors into its own per-GPU device array (at most
    BATCH_NOALLOC_MAX_ITEMS items), so nothing is allocated.  convs as for
    Batch.  Calls that overlap on one GPU race on that array."""
    items = (BatchItem * max(1, len(convs)))()
    for k, (di, dw, do, oh, ow, f) in enumerate(convs):
        check_buffers(xcorr_problem(oh, ow, f, f), di, dw, do)
        items[k] = BatchItem(di.data_ptr(), dw.data_ptr(), do.data_ptr(), oh, ow, f, f)
    _check(_lib.conv2d_run_batched_noalloc(items, len(convs), ctypes.byref(as_config(cfg)), int(grid_blocks),
                                           _stream(stream)))


class Graph:
    """Executable graph of the launches issued by fn() on a side stream."""

    def __init__(self, fn, stream):
        self.stream = stream
        h = ctypes.c_void_p(0)
        _check(_lib.gt_graph_begin(_stream(stream)))
        try:
            fn()
        finally:
            rc = _lib.gt_graph_end(_stream(stream), ctypes.byref(h))
        _check(rc)
        self.handle = h

    def launch(self):
        _check(_lib.gt_graph_launch(self.handle, _stream(self.stream)))

    def close(self):
        if self.handle:
            _check(_lib.gt_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


# ---- background sampler ----

def sampler_start(period_ms=2.0):
    _check(_lib.gt_sampler_start(float(period_ms)))


def sampler_stop(capacity=1 << 20):
    arr = (SensorSample * capacity)()
    n = ctypes.c_size_t(0)
    rc = _lib.gt_sampler_stop(arr, capacity, ctypes.byref(n))
    if rc not in (GT_OK, GT_E_CAPACITY):
        _check(rc)
    return [arr[k].as_dict() for k in range(min(n.value, capacity))]


def sensor_busy(busy):
    _check(_lib.gt_sensor_busy(1 if busy else 0))


# ---- search difficulty ----

def ffg_centrality(configs, fitness, p_values=(1.0, 1.05, 1.1, 1.25, 1.5, 2.0), damping=0.85):
    """PageRank over the fitness flow graph and the proportion of centrality
    per p.  Returns (pagerank list, is_minimum list, proportions list)."""
    n = len(configs)
    cf = (ConvConfig * n)(*[as_config(c) for c in configs])
    fa, _ = _darr(fitness)
    pa, npv = _darr(p_values)
    pr = (ctypes.c_double * n)()
    im = (ctypes.c_int32 * n)()
    prop = (ctypes.c_double * max(npv, 1))()
    _check(_lib.gt_ffg_centrality(cf, fa, n, damping, pa, npv, pr, im, prop))
    return list(pr), list(im), [prop[k] for k in range(npv)]
