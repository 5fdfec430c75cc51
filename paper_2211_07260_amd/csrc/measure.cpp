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
#include <functional>
#include <thread>

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

}  // namespace

namespace gt {

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
    const int64_t n = std::max<int64_t>(o.min_launches, (int64_t)std::ceil(o.window_s / t_est));

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
    const double t_start = now_s();
    hipError_t herr = hipEventRecord(win.a, s);
    int64_t launched = 0;
    for (; launched < n && herr == hipSuccess; ++launched) {
        rc = launch(s);
        if (rc) break;
    }
    if (herr == hipSuccess && rc == GT_OK) herr = hipEventRecord(win.b, s);
    if (herr == hipSuccess && rc == GT_OK) herr = hipEventSynchronize(win.b);
    const double t_stop = now_s();
    stop.store(true);
    sampler.join();
    sensor_set_busy(false);
    if (rc) return rc;
    if (herr != hipSuccess) return set_error(GT_E_HIP, "measure window: %s", hipGetErrorString(herr));
    float win_ms = 0;
    GT_HIP_CHECK(hipEventElapsedTime(&win_ms, win.a, win.b));

    // keep the samples after the stabilisation discard
    std::vector<double> kept_p, kept_t;
    double sclk_sum = 0;
    int sclk_n = 0;
    for (const gt_sensor_sample &smp : samples) {
        if (smp.t_s < t_start + o.discard_s || smp.t_s > t_stop) continue;
        if (!std::isfinite(smp.power_w)) continue;
        kept_p.push_back(smp.power_w);
        kept_t.push_back(smp.t_s);
        if (std::isfinite(smp.sclk_mhz)) {
            sclk_sum += smp.sclk_mhz;
            ++sclk_n;
        }
    }
    if (kept_p.empty())
        return set_error(GT_E_SENSOR, "measure: no power sample in the kept window (%zu samples, sensor errors %d)",
                         samples.size(), sensor_err.load());
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
    m.n_used = (int64_t)kept_p.size();
    m.p_median_w = median_of(kept_p);
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
    m.sclk_act_mhz = sclk_n ? sclk_sum / sclk_n : NAN;
    const gt_sensor_sample &tail = samples.back();
    m.mclk_mhz = tail.mclk_mhz;
    m.volt_v = tail.volt_v;
    m.temp_c = tail.temp_c;
    m.throttled = (m.sclk_req_mhz > 0 && sclk_n && m.sclk_act_mhz < 0.98 * m.sclk_req_mhz) ? 1 : 0;
    m.flags = ((state().flags & GT_INIT_FAKE_SENSOR) ? 1 : 0) | ((state().flags & GT_INIT_FAKE_DVFS) ? 2 : 0);
    return GT_OK;
}

}  // namespace gt

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
    const gt_measure_opts o = opts ? *opts : gt_measure_opts{0, -1, 0, 0, -1};
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
    const gt_measure_opts o = opts ? *opts : gt_measure_opts{0, -1, 0, 0, -1};
    return measure_window([&](hipStream_t s) { return launch_load(kind, d_buf, bytes, s); }, work, o,
                          (hipStream_t)hip_stream, rec);
}
