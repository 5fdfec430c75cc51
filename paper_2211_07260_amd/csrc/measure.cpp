// measure_time_energy: the observer of sections III.A-III.B.
//
// The kernel is launched back-to-back for a window (1 s by default) while a
// sampler thread polls the power sensor.  Time per launch comes from HIP
// events around the window; energy per launch is the median power of the
// samples taken after the stabilisation discard times that time (the paper's
// E = <P> (t1 - t0) with the median for <P>).  The energy accumulator gives an
// independent average power over an interval inside the kept window, reported
// as e_run_counter_j.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <functional>
#include <thread>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "gt_internal.hpp"

using namespace gt;

namespace {

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// A captured group of launches (use_graph), and the library stream it runs
// on when the caller passed the null stream (which cannot be captured).
struct GraphGroup {
    hipGraphExec_t exec = nullptr;
    hipStream_t own = nullptr;
    ~GraphGroup() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (own) (void)hipStreamDestroy(own);
    }
};

// The readings of the most recent measurement window (gt_measure_last_window).
struct LastWindow {
    std::mutex mu;
    bool valid = false;
    std::vector<gt_sensor_sample> samples;
    double t_start = 0, t_stop = 0;
};

LastWindow &last_window() {
    static LastWindow w;
    return w;
}

void record_last_window(const std::vector<gt_sensor_sample> &samples, double t_start, double t_stop) {
    LastWindow &w = last_window();
    std::lock_guard<std::mutex> lk(w.mu);
    w.samples = samples;
    w.t_start = t_start;
    w.t_stop = t_stop;
    w.valid = true;
}

}  // namespace

namespace gt {

// Marker text of a measurement window: its work per launch (flop, or bytes
// for the copy load) and options.
static std::string gflops_label(double flops, const gt_measure_opts &o) {
    char buf[160];
    snprintf(buf, sizeof buf, "greentune measure window: %.4g G work/launch, %.3g s, discard %.3g s%s", flops * 1e-9,
             o.window_s, o.discard_s, o.use_graph ? ", graph replay" : "");
    return buf;
}

// A kept window at least this long whose power never changes is stale: the
// socket power reading refreshes every few milliseconds under load.
constexpr double kStaleSpanS = 0.5;

// The measurement window shared by measure_time_energy and measure_load:
// warm-up launches, an estimate of the launch time, then launches back to
// back for the window while the sampler records the sensor.
int measure_window(const std::function<int(hipStream_t)> &launch, double flops_per_launch, gt_measure_opts o,
                   hipStream_t s, gt_measurement *rec) {
    if (!(o.window_s > 0)) o.window_s = 1.0;
    if (o.discard_s < 0) o.discard_s = 0.3;
    if (!(o.sample_period_ms > 0)) o.sample_period_ms = 1.0;
    if (o.min_launches <= 0) o.min_launches = 10;
    if (o.warmup_launches < 0) o.warmup_launches = 3;
    if (o.discard_s >= o.window_s)
        return set_error(GT_E_INVAL, "measure: discard %.3f s >= window %.3f s", o.discard_s, o.window_s);
    int rc = sensor_open();
    if (rc) return rc;
    for (int k = 0; k < o.warmup_launches; ++k) {
        rc = launch(s);
        if (rc) return rc;
    }
    EventPair est, win;
    GT_HIP_CHECK(hipEventCreate(&est.a));
    GT_HIP_CHECK(hipEventCreate(&est.b));
    GT_HIP_CHECK(hipEventCreate(&win.a));
    GT_HIP_CHECK(hipEventCreate(&win.b));
    GT_HIP_CHECK(hipEventRecord(est.a, s));
    for (int k = 0; k < 3; ++k) {
        rc = launch(s);
        if (rc) return rc;
    }
    GT_HIP_CHECK(hipEventRecord(est.b, s));
    GT_HIP_CHECK(hipEventSynchronize(est.b));
    float est_ms = 0;
    GT_HIP_CHECK(hipEventElapsedTime(&est_ms, est.a, est.b));
    const double t_est = std::max(1e-7, est_ms * 1e-3 / 3.0);
    int64_t n = std::max<int64_t>(o.min_launches, (int64_t)std::ceil(o.window_s / t_est));

    // use_graph: capture `group` launches once (about 1 ms of work, at most
    // 256) and replay the graph for the window; the caller's null stream is
    // replaced by a library stream after the work queued on it has finished.
    GraphGroup gg;
    int64_t group = 1;
    if (o.use_graph) {
        group = std::min<int64_t>(256, std::max<int64_t>(1, (int64_t)std::ceil(1e-3 / t_est)));
        if (!s) {
            GT_HIP_CHECK(hipStreamSynchronize(s));
            GT_HIP_CHECK(hipStreamCreateWithFlags(&gg.own, hipStreamNonBlocking));
            s = gg.own;
        }
        hipGraph_t g = nullptr;
        GT_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int64_t k = 0; k < group && rc == GT_OK; ++k) rc = launch(s);
        const hipError_t ce = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ce != hipSuccess) return set_error(GT_E_HIP, "measure: graph capture: %s", hipGetErrorString(ce));
        const hipError_t ie = hipGraphInstantiate(&gg.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return set_error(GT_E_HIP, "measure: graph instantiate: %s", hipGetErrorString(ie));
        GT_HIP_CHECK(hipGraphLaunch(gg.exec, s));  // one untimed replay
        n = (n + group - 1) / group * group;
    }
    auto issue = [&](hipStream_t st) -> int {
        if (!gg.exec) return launch(st);
        const hipError_t e = hipGraphLaunch(gg.exec, st);
        return e == hipSuccess ? GT_OK : set_error(GT_E_HIP, "measure: graph launch: %s", hipGetErrorString(e));
    };

    std::vector<gt_sensor_sample> samples;
    samples.reserve((size_t)(o.window_s * 1000.0 / o.sample_period_ms) + 64);
    std::atomic<bool> stop{false};
    std::atomic<int> sensor_err{0};
    sensor_set_busy(true);
    std::thread sampler([&]() {
        const auto period = std::chrono::duration<double>(o.sample_period_ms * 1e-3);
        while (!stop.load()) {
            gt_sensor_sample smp;
            if (sensor_read(&smp) == GT_OK)
                samples.push_back(smp);
            else
                sensor_err.store(1);
            std::this_thread::sleep_for(period);
        }
    });
    // a marker range around the window (rocprofv3 --marker-trace shows it
    // beside the kernels it times); no-op without a profiler
    roctxRangePushA(gflops_label(flops_per_launch, o).c_str());
    const double t_start = now_s();
    hipError_t herr = hipEventRecord(win.a, s);
    int64_t launched = 0;
    for (; launched < n && herr == hipSuccess; launched += group) {
        rc = issue(s);
        if (rc) break;
    }
    if (herr == hipSuccess && rc == GT_OK) herr = hipEventRecord(win.b, s);
    if (herr == hipSuccess && rc == GT_OK) herr = hipEventSynchronize(win.b);
    const double t_stop = now_s();
    roctxRangePop();
    stop.store(true);
    sampler.join();
    sensor_set_busy(false);
    if (rc) return rc;
    if (herr != hipSuccess) return set_error(GT_E_HIP, "measure window: %s", hipGetErrorString(herr));
    float win_ms = 0;
    GT_HIP_CHECK(hipEventElapsedTime(&win_ms, win.a, win.b));

    // Energy per run: the median of the finite power readings after the
    // stabilisation discard (gt_energy_from_samples, the arithmetic the tests
    // pin against the oracle) times the HIP-event time per launch.
    std::vector<double> all_t, all_p;
    all_t.reserve(samples.size());
    all_p.reserve(samples.size());
    for (const gt_sensor_sample &smp : samples)
        if (std::isfinite(smp.power_w)) {
            all_t.push_back(smp.t_s);
            all_p.push_back(smp.power_w);
        }
    double e_host = 0, p_med = 0;
    size_t n_used = 0;
    const double t_lo = t_start + o.discard_s;
    rc = gt_energy_from_samples(all_t.data(), all_p.data(), all_t.size(), t_start, t_stop, launched, o.discard_s,
                                &e_host, &p_med, &n_used);
    if (rc == GT_E_SENSOR)
        return set_error(GT_E_SENSOR, "measure: no power sample in the kept window (%zu samples, sensor errors %d)",
                         samples.size(), sensor_err.load());
    if (rc) return rc;
    std::vector<double> kept_p, kept_t;
    for (size_t k = 0; k < all_t.size(); ++k)
        if (all_t[k] >= t_lo && all_t[k] <= t_stop) {
            kept_t.push_back(all_t[k]);
            kept_p.push_back(all_p[k]);
        }
    record_last_window(samples, t_start, t_stop);
    // a hardware power reading that never changes under load is stale (the
    // fake sensor without noise is constant by design)
    if (!(state().flags & GT_INIT_FAKE_SENSOR) &&
        gt_sensor_stale(kept_t.data(), kept_p.data(), kept_p.size(), kStaleSpanS) == 1)
        return set_error(GT_E_SENSOR, "measure: stale sensor, power unchanged at %.1f W over %.2f s (%zu samples)",
                         kept_p[0], kept_t.back() - kept_t[0], kept_p.size());
    gt_measurement &m = *rec;
    m = gt_measurement();
    m.launches = launched;
    m.window_s = win_ms * 1e-3;
    m.t_run_s = m.window_s / (double)launched;
    m.n_samples = (int64_t)samples.size();
    m.n_used = (int64_t)n_used;
    m.p_median_w = p_med;
    m.p_min_w = *std::min_element(kept_p.begin(), kept_p.end());
    m.p_max_w = *std::max_element(kept_p.begin(), kept_p.end());
    m.e_run_j = m.p_median_w * m.t_run_s;
    // Energy-counter cross-check: the accumulator updates about once per
    // second with a firmware timestamp.  Use the first and last updates
    // observed inside the kept interval; their timestamps bound an interval
    // that lies wholly inside the window.  NaN when fewer than two updates.
    m.e_run_counter_j = NAN;
    {
        const gt_sensor_sample *ua = nullptr, *ub = nullptr;
        for (size_t k = 1; k < samples.size(); ++k) {
            const gt_sensor_sample &a = samples[k - 1], &b = samples[k];
            if (!(b.energy_t_s != a.energy_t_s) || !std::isfinite(b.energy_j)) continue;
            if (a.t_s < t_start + o.discard_s || b.t_s > t_stop) continue;
            if (!ua) ua = &b;
            ub = &b;
        }
        if (ua && ub && ub->energy_t_s > ua->energy_t_s)
            m.e_run_counter_j = (ub->energy_j - ua->energy_j) / (ub->energy_t_s - ua->energy_t_s) * m.t_run_s;
    }
    m.gflops = flops_per_launch / m.t_run_s * 1e-9;
    m.gflops_per_w = flops_per_launch / m.e_run_j * 1e-9;
    m.sclk_req_mhz = dvfs_requested_mhz();
    size_t n_fresh = 0;
    gt_window_clock(samples.data(), samples.size(), t_lo, t_stop, &m.sclk_act_mhz, &n_fresh);
    const gt_sensor_sample &tail = samples.back();
    m.mclk_mhz = tail.mclk_mhz;
    m.volt_v = tail.volt_v;
    m.temp_c = tail.temp_c;
    m.throttled = (m.sclk_req_mhz > 0 && std::isfinite(m.sclk_act_mhz) && m.sclk_act_mhz < 0.98 * m.sclk_req_mhz)
                      ? 1
                      : 0;
    m.flags = ((state().flags & GT_INIT_FAKE_SENSOR) ? 1 : 0) | ((state().flags & GT_INIT_FAKE_DVFS) ? 2 : 0);
    return GT_OK;
}

}  // namespace gt

extern "C" int gt_window_clock(const gt_sensor_sample *samples, size_t n, double t_lo, double t_hi,
                               double *sclk_mhz, size_t *n_fresh) {
    clear_error();
    if ((n && !samples) || !sclk_mhz) return set_error(GT_E_INVAL, "gt_window_clock: null argument");
    double seen = NAN;  // metrics timestamp in force; NaN = not established yet
    bool have_seen = false;
    double sum = 0;
    size_t cnt = 0;
    for (size_t k = 0; k < n; ++k) {
        const gt_sensor_sample &s = samples[k];
        if (s.t_s > t_hi) break;
        const double ts = s.metrics_t_s;
        if (!std::isfinite(ts)) continue;
        if (s.t_s < t_lo || !have_seen) {
            seen = ts;
            have_seen = true;
            continue;
        }
        if (ts == seen) continue;
        seen = ts;
        if (std::isfinite(s.sclk_mhz)) {
            sum += s.sclk_mhz;
            ++cnt;
        }
    }
    *sclk_mhz = cnt ? sum / (double)cnt : NAN;
    if (n_fresh) *n_fresh = cnt;
    return GT_OK;
}

extern "C" int gt_measure_last_window(gt_sensor_sample *out, size_t capacity, size_t *n, double *t_start,
                                      double *t_stop) {
    clear_error();
    if (!n || (capacity && !out)) return set_error(GT_E_INVAL, "gt_measure_last_window: bad argument");
    LastWindow &w = last_window();
    std::lock_guard<std::mutex> lk(w.mu);
    if (!w.valid) return set_error(GT_E_STATE, "gt_measure_last_window: no window measured yet");
    *n = w.samples.size();
    for (size_t k = 0; k < w.samples.size() && k < capacity; ++k) out[k] = w.samples[k];
    if (t_start) *t_start = w.t_start;
    if (t_stop) *t_stop = w.t_stop;
    if (w.samples.size() > capacity)
        return set_error(GT_E_CAPACITY, "gt_measure_last_window: %zu samples, capacity %zu", w.samples.size(),
                         capacity);
    return GT_OK;
}

extern "C" int gt_sensor_stale(const double *t_s, const double *p_w, size_t n, double min_span_s) {
    clear_error();
    if (n && (!t_s || !p_w)) return set_error(GT_E_INVAL, "gt_sensor_stale: null argument");
    if (n < 2 || !(t_s[n - 1] - t_s[0] >= min_span_s)) return 0;
    for (size_t k = 1; k < n; ++k)
        if (p_w[k] != p_w[0]) return 0;
    return 1;
}

extern "C" int measure_time_energy(const gt_problem *problem, const gt_conv_config *config,
                                   gt_clock clock, const gt_measure_opts *opts, const void *d_in,
                                   const void *d_filt, void *d_out, void *hip_stream,
                                   gt_measurement *rec) {
    clear_error();
    if (!problem || !config || !d_in || !d_filt || !d_out || !rec)
        return set_error(GT_E_INVAL, "measure_time_energy: null argument");
    if (!state().inited) return set_error(GT_E_STATE, "measure_time_energy: call gt_init first");
    if (state().flags & GT_INIT_HOST_ONLY)
        return set_error(GT_E_STATE, "measure_time_energy: library initialised host-only");
    const gt_measure_opts o = opts ? *opts : gt_measure_opts{0, -1, 0, 0, -1, 0};
    if (o.window_s > 0 && o.discard_s >= o.window_s)
        return set_error(GT_E_INVAL, "measure_time_energy: discard %.3f s >= window %.3f s", o.discard_s,
                         o.window_s);
    int rc = validate_problem_config(*problem, *config);
    if (rc) return rc;
    rc = dvfs_apply(clock);
    if (rc) return rc;
    return measure_window([&](hipStream_t s) { return launch_problem(*problem, *config, d_in, d_filt, d_out, s); },
                          gt_problem_flops(problem), o, (hipStream_t)hip_stream, rec);
}

extern "C" int measure_load(int32_t kind, gt_clock clock, const gt_measure_opts *opts, void *d_buf, size_t bytes,
                            void *hip_stream, gt_measurement *rec) {
    clear_error();
    if (!d_buf || !rec) return set_error(GT_E_INVAL, "measure_load: null argument");
    if (!state().inited) return set_error(GT_E_STATE, "measure_load: call gt_init first");
    if (state().flags & GT_INIT_HOST_ONLY) return set_error(GT_E_STATE, "measure_load: library initialised host-only");
    double work = 0;
    int rc = load_work(kind, bytes, &work);
    if (rc) return rc;
    rc = dvfs_apply(clock);
    if (rc) return rc;
    const gt_measure_opts o = opts ? *opts : gt_measure_opts{0, -1, 0, 0, -1, 0};
    return measure_window([&](hipStream_t s) { return launch_load(kind, d_buf, bytes, s); }, work, o,
                          (hipStream_t)hip_stream, rec);
}
