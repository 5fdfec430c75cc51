// C ABI of the library: lifecycle, error reporting, conv2d_run,
// tune_space_enumerate and the host-side helpers of the method.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "gt_internal.hpp"

namespace gt {

static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

State &state() {
    static State s;
    return s;
}

bool host_only() { return (state().flags & GT_INIT_HOST_ONLY) != 0 || !state().inited; }

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

double median_of(std::vector<double> v) {
    const size_t n = v.size();
    if (n == 0) return NAN;
    const size_t m = n / 2;
    std::nth_element(v.begin(), v.begin() + m, v.end());
    const double hi = v[m];
    if (n % 2) return hi;
    const double lo = *std::max_element(v.begin(), v.begin() + m);
    return 0.5 * (lo + hi);
}

int validate_problem_config(const gt_problem &p, const gt_conv_config &c) {
    const State &st = state();
    switch (p.kind) {
        case GT_XCORR_F32:
            return validate_xcorr(p, c, st.dev.lds_per_block, st.dev.max_threads);
        case GT_IGEMM_BF16_MFMA:
        case GT_IGEMM_F32_VALU:
            return validate_igemm(p, c);
        default:
            return set_error(GT_E_INVAL, "unknown problem kind %d", p.kind);
    }
}

int launch_problem(const gt_problem &p, const gt_conv_config &c, const void *in, const void *w,
                   void *out, hipStream_t s) {
    if (p.kind == GT_XCORR_F32) return launch_xcorr_f32(p, c, in, w, out, s);
    return launch_igemm(p, c, in, w, out, s);
}

}  // namespace gt

using namespace gt;

extern "C" {

const char *gt_last_error(void) { return g_err.c_str(); }

const char *gt_version(void) { return "greentune 0.1 (gfx950)"; }

int gt_init(int device_ordinal, uint32_t flags) {
    clear_error();
    State &st = state();
    std::lock_guard<std::mutex> lk(st.mu);
    if (st.inited) {
        if (st.flags == flags && (st.dev.ordinal == device_ordinal || (flags & GT_INIT_HOST_ONLY)))
            return GT_OK;
        return set_error(GT_E_STATE, "already initialised with other arguments; call gt_shutdown first");
    }
    st.flags = flags;
    st.dev = DeviceInfo();
    if (!(flags & GT_INIT_HOST_ONLY)) {
        int n = 0;
        GT_HIP_CHECK(hipGetDeviceCount(&n));
        if (device_ordinal < 0 || device_ordinal >= n)
            return set_error(GT_E_HIP, "device %d not present (%d devices)", device_ordinal, n);
        GT_HIP_CHECK(hipSetDevice(device_ordinal));
        DeviceInfo &d = st.dev;
        d.ordinal = device_ordinal;
        int v = 0;
        GT_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxThreadsPerBlock, device_ordinal));
        d.max_threads = v;
        GT_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device_ordinal));
        d.lds_per_block = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, device_ordinal) ==
                hipSuccess && v > d.lds_per_block)
            d.lds_per_block = v;
        GT_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device_ordinal));
        d.cu_count = v;
        GT_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeClockRate, device_ordinal));
        d.clock_khz = v;
        GT_HIP_CHECK(hipDeviceGetAttribute(&d.pci_domain, hipDeviceAttributePciDomainID, device_ordinal));
        GT_HIP_CHECK(hipDeviceGetAttribute(&d.pci_bus, hipDeviceAttributePciBusId, device_ordinal));
        GT_HIP_CHECK(hipDeviceGetAttribute(&d.pci_device, hipDeviceAttributePciDeviceId, device_ordinal));
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device_ordinal) == hipSuccess)
            snprintf(d.name, sizeof d.name, "%s", prop.gcnArchName);
    }
    st.clock = gt_clock{GT_CLOCK_DEFAULT, 0};
    st.inited = true;
    if ((flags & GT_INIT_ALLOW_DVFS) && !(flags & (GT_INIT_FAKE_DVFS | GT_INIT_HOST_ONLY))) {
        const int rc = dvfs_recover();
        if (rc) {
            st.inited = false;
            return rc;
        }
    }
    return GT_OK;
}

int gt_shutdown(void) {
    clear_error();
    State &st = state();
    std::lock_guard<std::mutex> lk(st.mu);
    if (!st.inited) return GT_OK;
    int rc = dvfs_restore();
    sensor_close();
    st.inited = false;
    st.flags = 0;
    return rc;
}

int conv2d_run(const gt_problem *problem, const gt_conv_config *config, gt_clock clock,
               const void *d_in, const void *d_filt, void *d_out, void *hip_stream) {
    clear_error();
    if (!problem || !config || !d_in || !d_filt || !d_out)
        return set_error(GT_E_INVAL, "conv2d_run: null argument");
    if (!state().inited) return set_error(GT_E_STATE, "conv2d_run: call gt_init first");
    if (state().flags & GT_INIT_HOST_ONLY)
        return set_error(GT_E_STATE, "conv2d_run: library initialised host-only");
    int rc = validate_problem_config(*problem, *config);
    if (rc) return rc;
    rc = dvfs_apply(clock);
    if (rc) return rc;
    return launch_problem(*problem, *config, d_in, d_filt, d_out, (hipStream_t)hip_stream);
}

int conv2d_run_part(const gt_problem *problem, const gt_conv_config *config, gt_clock clock, int32_t part,
                    int32_t n_parts, const void *d_in, const void *d_filt, void *d_out, void *hip_stream) {
    clear_error();
    if (!problem || !config || !d_in || !d_filt || !d_out)
        return set_error(GT_E_INVAL, "conv2d_run_part: null argument");
    if (n_parts < 1 || part < 0 || part >= n_parts)
        return set_error(GT_E_INVAL, "conv2d_run_part: part %d of %d", part, n_parts);
    if (!state().inited) return set_error(GT_E_STATE, "conv2d_run_part: call gt_init first");
    if (state().flags & GT_INIT_HOST_ONLY)
        return set_error(GT_E_STATE, "conv2d_run_part: library initialised host-only");
    int rc = validate_problem_config(*problem, *config);
    if (rc) return rc;
    if (n_parts > 1 && problem->kind != GT_IGEMM_BF16_MFMA)
        return set_error(GT_E_UNSUPPORTED, "conv2d_run_part: parts are for the BF16 implicit GEMM only");
    rc = dvfs_apply(clock);
    if (rc) return rc;
    if (n_parts == 1) return launch_problem(*problem, *config, d_in, d_filt, d_out, (hipStream_t)hip_stream);
    return launch_igemm(*problem, *config, d_in, d_filt, d_out, (hipStream_t)hip_stream, part, n_parts);
}

int tune_space_enumerate(const gt_problem *problem, const gt_space_desc *space,
                         gt_conv_config *out, size_t capacity, size_t *n_total) {
    clear_error();
    if (!problem || !space || !n_total || (capacity && !out))
        return set_error(GT_E_INVAL, "tune_space_enumerate: null argument");
    for (int k = 0; k < 6; ++k)
        if (space->counts[k] < 1 || !space->values[k])
            return set_error(GT_E_INVAL, "tune_space_enumerate: empty value list %d", k);
    const int max_threads = space->max_threads > 0 ? space->max_threads : state().dev.max_threads;
    int64_t lds_limit = space->lds_limit_bytes;
    if (lds_limit <= 0) {
        if (host_only())
            return set_error(GT_E_STATE, "tune_space_enumerate: lds_limit_bytes = 0 needs a device");
        lds_limit = state().dev.lds_per_block;
    }
    const bool dedup = (space->flags & GT_SPACE_DEDUP_DIRECT) != 0;
    size_t n = 0;
    int32_t idx[6] = {0, 0, 0, 0, 0, 0};
    const int32_t *const *V = space->values;
    const int32_t *C = space->counts;
    for (;;) {
        gt_conv_config c{V[0][idx[0]], V[1][idx[1]], V[2][idx[2]],
                         V[3][idx[3]], V[4][idx[4]], V[5][idx[5]]};
        bool ok = (int64_t)c.block_size_x * c.block_size_y <= max_threads;
        if (ok && c.read_path == 0 && problem->kind == GT_XCORR_F32)
            ok = xcorr_lds_bytes(*problem, c) <= lds_limit;
        if (ok && dedup && c.read_path == 1 && c.use_lds_padding != 0) ok = false;
        if (ok) {
            if (n < capacity) out[n] = c;
            ++n;
        }
        int k = 5;
        while (k >= 0 && ++idx[k] == C[k]) idx[k--] = 0;
        if (k < 0) break;
    }
    *n_total = n;
    if (n > capacity)
        return set_error(GT_E_CAPACITY, "tune_space_enumerate: %zu configs, capacity %zu", n, capacity);
    return GT_OK;
}

double gt_problem_flops(const gt_problem *p) {
    if (!p) return NAN;
    return 2.0 * p->n * (double)p->out_h * p->out_w * p->c_out * p->c_in * p->filt_h * p->filt_w;
}

int gt_conv_lds_bytes(const gt_problem *problem, const gt_conv_config *config, int64_t *bytes) {
    clear_error();
    if (!problem || !config || !bytes) return set_error(GT_E_INVAL, "gt_conv_lds_bytes: null argument");
    *bytes = problem->kind == GT_XCORR_F32 ? xcorr_lds_bytes(*problem, *config) : 0;
    return GT_OK;
}

int gt_energy_from_samples(const double *t_s, const double *p_w, size_t n, double t_start,
                           double t_stop, int64_t n_runs, double discard_s, double *e_run_j,
                           double *p_median_w, size_t *n_used) {
    clear_error();
    if ((n && (!t_s || !p_w)) || !e_run_j || n_runs < 1 || !(t_stop > t_start))
        return set_error(GT_E_INVAL, "gt_energy_from_samples: bad argument");
    std::vector<double> kept;
    for (size_t k = 0; k < n; ++k)
        if (t_s[k] >= t_start + discard_s && t_s[k] <= t_stop) kept.push_back(p_w[k]);
    if (n_used) *n_used = kept.size();
    if (kept.empty()) return set_error(GT_E_SENSOR, "gt_energy_from_samples: no sample in the window");
    const double pm = median_of(kept);
    if (p_median_w) *p_median_w = pm;
    *e_run_j = pm * ((t_stop - t_start) / (double)n_runs);
    return GT_OK;
}

int gt_select(const gt_measurement *recs, size_t n, int objective, size_t *index) {
    clear_error();
    if (!recs || !n || !index || (objective != 0 && objective != 1))
        return set_error(GT_E_INVAL, "gt_select: bad argument");
    size_t best = 0;
    for (size_t k = 1; k < n; ++k) {
        const gt_measurement &a = recs[k], &b = recs[best];
        const double a1 = objective ? a.e_run_j : a.t_run_s, b1 = objective ? b.e_run_j : b.t_run_s;
        const double a2 = objective ? a.t_run_s : a.e_run_j, b2 = objective ? b.t_run_s : b.e_run_j;
        if (a1 < b1 || (a1 == b1 && a2 < b2)) best = k;
    }
    *index = best;
    return GT_OK;
}

int gt_pareto(const gt_measurement *recs, size_t n, int32_t *on_front) {
    clear_error();
    if (n && (!recs || !on_front)) return set_error(GT_E_INVAL, "gt_pareto: null argument");
    // sort by (t_run, e_run); a record is dominated exactly when some record
    // before it in that order (a different point) has e_run <= its own, so one
    // sweep keeping the running minimum of e_run over earlier points decides
    std::vector<size_t> ord(n);
    for (size_t k = 0; k < n; ++k) ord[k] = k;
    std::sort(ord.begin(), ord.end(), [recs](size_t a, size_t b) {
        if (recs[a].t_run_s != recs[b].t_run_s) return recs[a].t_run_s < recs[b].t_run_s;
        return recs[a].e_run_j < recs[b].e_run_j;
    });
    double best_e = INFINITY;  // lowest e_run among points strictly before the current group
    size_t k = 0;
    while (k < n) {
        size_t g = k;  // group of records at the same point
        while (g < n && recs[ord[g]].t_run_s == recs[ord[k]].t_run_s && recs[ord[g]].e_run_j == recs[ord[k]].e_run_j)
            ++g;
        const gt_measurement &r = recs[ord[k]];
        const int32_t front = r.e_run_j < best_e ? 1 : 0;
        for (size_t j = k; j < g; ++j) on_front[ord[j]] = front;
        best_e = std::min(best_e, r.e_run_j);
        k = g;
    }
    return GT_OK;
}

}  // extern "C"
