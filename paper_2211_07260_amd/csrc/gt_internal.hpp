// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/greentune.h"

namespace gt {

int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define GT_HIP_CHECK(expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::gt::set_error(GT_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                   __FILE__, __LINE__);                                      \
    } while (0)

struct DeviceInfo {
    int ordinal = -1;
    int max_threads = 1024;
    int64_t lds_per_block = 65536;
    int cu_count = 0;
    int clock_khz = 0;
    int pci_domain = 0, pci_bus = 0, pci_device = 0;
    char name[256] = {0};
};

struct State {
    std::mutex mu;
    bool inited = false;
    uint32_t flags = 0;
    DeviceInfo dev;
    gt_clock clock{GT_CLOCK_DEFAULT, 0};  // knob currently applied through the library
};
State &state();
bool host_only();

// ---- kernels ----
int validate_xcorr(const gt_problem &p, const gt_conv_config &c, int64_t lds_limit, int max_threads);
int64_t xcorr_lds_bytes(const gt_problem &p, const gt_conv_config &c);
int launch_xcorr_f32(const gt_problem &p, const gt_conv_config &c, const void *in, const void *w,
                     void *out, hipStream_t s);
int validate_igemm(const gt_problem &p, const gt_conv_config &c);
int launch_igemm(const gt_problem &p, const gt_conv_config &c, const void *in, const void *w,
                 void *out, hipStream_t s, int part = 0, int n_parts = 1);
int validate_problem_config(const gt_problem &p, const gt_conv_config &c);
// synthetic full loads (roofline_probe.hip): work per launch, and one launch
int load_work(int kind, size_t bytes, double *work);
int launch_load(int kind, void *buf, size_t bytes, hipStream_t s);
int launch_problem(const gt_problem &p, const gt_conv_config &c, const void *in, const void *w,
                   void *out, hipStream_t s);

// ---- sensor / DVFS ----
int sensor_open();                       // amd-smi or fake, per state().flags
void sensor_close();
int sensor_read(gt_sensor_sample *s);
void sensor_set_busy(bool busy);         // fake sensor: kernel activity in progress
int dvfs_apply(const gt_clock &clk);     // no-op when equal to the current knob
int dvfs_restore();
int dvfs_recover();                       // restore a knob a previous process left set (state file)
std::string dvfs_state_path();            // that process's record of the knob in force
int dvfs_settable(double step_mhz, std::vector<double> &out);
double dvfs_requested_mhz();             // 0 when the clock is at its default

double now_s();                          // host steady clock

// The measurement window of measure_time_energy (measure.cpp): warm-up,
// launches back to back (or graph replays) for the window while the sampler
// runs, time from HIP events, energy by gt_energy_from_samples.
int measure_window(const std::function<int(hipStream_t)> &launch, double flops_per_launch, gt_measure_opts o,
                   hipStream_t s, gt_measurement *rec);

// ---- method arithmetic (host, FP64) ----
double median_of(std::vector<double> v);

}  // namespace gt
