// Background power sampler: a native thread that reads the sensor at a fixed
// period between gt_sampler_start and gt_sampler_stop, for callers that
// measure a window of their own (serving, sensor characterisation).
#include <atomic>
#include <chrono>
#include <thread>

#include "gt_internal.hpp"

namespace gt {
namespace {

struct Sampler {
    std::mutex mu;
    std::thread th;
    std::atomic<bool> stop{false};
    bool running = false;
    std::vector<gt_sensor_sample> samples;
    int errors = 0;
};

Sampler &sampler() {
    static Sampler s;
    return s;
}

}  // namespace
}  // namespace gt

using namespace gt;

extern "C" {

int gt_sampler_start(double period_ms) {
    clear_error();
    if (!(period_ms > 0)) return set_error(GT_E_INVAL, "gt_sampler_start: period must be positive");
    if (!state().inited) return set_error(GT_E_STATE, "gt_sampler_start: call gt_init first");
    Sampler &S = sampler();
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.running) return set_error(GT_E_STATE, "gt_sampler_start: already running");
    int rc = sensor_open();
    if (rc) return rc;
    S.samples.clear();
    S.samples.reserve(4096);
    S.errors = 0;
    S.stop.store(false);
    S.running = true;
    S.th = std::thread([period_ms]() {
        Sampler &T = sampler();
        const auto period = std::chrono::duration<double>(period_ms * 1e-3);
        while (!T.stop.load()) {
            gt_sensor_sample smp;
            if (sensor_read(&smp) == GT_OK)
                T.samples.push_back(smp);
            else
                ++T.errors;
            std::this_thread::sleep_for(period);
        }
    });
    return GT_OK;
}

int gt_sampler_stop(gt_sensor_sample *out, size_t capacity, size_t *n) {
    clear_error();
    if (!n || (capacity && !out)) return set_error(GT_E_INVAL, "gt_sampler_stop: bad argument");
    Sampler &S = sampler();
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.running) return set_error(GT_E_STATE, "gt_sampler_stop: not running");
    S.stop.store(true);
    S.th.join();
    S.running = false;
    *n = S.samples.size();
    for (size_t k = 0; k < S.samples.size() && k < capacity; ++k) out[k] = S.samples[k];
    if (S.samples.empty()) return set_error(GT_E_SENSOR, "gt_sampler_stop: no sample (%d sensor errors)", S.errors);
    if (S.samples.size() > capacity)
        return set_error(GT_E_CAPACITY, "gt_sampler_stop: %zu samples, capacity %zu", S.samples.size(), capacity);
    return GT_OK;
}

int gt_sensor_busy(int busy) {
    sensor_set_busy(busy != 0);
    return GT_OK;
}

}  // extern "C"
