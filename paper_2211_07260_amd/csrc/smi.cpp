// Power sensor and DVFS controller.
//
// The paper reads board power, energy, clocks, voltage and temperature
// through the vendor management library and sets the graphics clock or the
// power limit as tunables (sections III.B and III.C).  On MI355X the roles
// split by refresh rate:
//   - socket power comes from the amdgpu hwmon file power1_input (microwatts),
//     which the firmware refreshes every few milliseconds;
//   - the GPU metrics table read through amd-smi (energy accumulator with its
//     firmware timestamp, per-XCD graphics clocks, memory clock, graphics
//     voltage, hotspot temperature) refreshes about once per second, so it is
//     re-read at most every 50 ms and serves as the slow cross-check.
// The clock knob is the graphics-clock upper limit and the power knob the
// socket power cap.  The library itself changes no device setting: a caller
// with the privileges registers a DVFS backend (gt_dvfs_set_backend) whose
// apply and restore functions change the knob; the library keeps the knob's
// state (repeated settings are no-ops, gt_shutdown restores) and refuses any
// change without GT_INIT_ALLOW_DVFS and a backend (GT_E_PERM).
//
// Fake backends (for tests that must not touch the hardware):
//   GT_INIT_FAKE_DVFS    the knob is only recorded; settable clocks 500..2400 MHz
//   GT_INIT_FAKE_SENSOR  power follows a gt_power_model at the current clock
//                        plus seeded Gaussian noise; idle power between kernels
#include <amd_smi/amdsmi.h>

#include <dirent.h>
#include <stdio.h>
#include <string.h>
#include <fcntl.h>
#include <limits.h>
#include <stdlib.h>
#include <unistd.h>

#include <atomic>
#include <cmath>
#include <string>

#include "gt_internal.hpp"

namespace gt {
namespace {

struct Smi {
    bool open = false;
    amdsmi_processor_handle h = nullptr;
    double energy_res_j = 15.259e-6;
    uint64_t last_energy_raw = 0;
    double energy_wrap_j = 0;
    int hwmon_fd = -1;            // power1_input of this device
    std::string hwmon_dir;        // its hwmon directory
    double metrics_t = -1;        // host time of the cached metrics read
    gt_sensor_sample cached{};    // slow fields of the last metrics read
};

struct Fake {
    gt_power_model model{};
    bool have_model = false;
    double noise_w = 0;
    uint64_t rng = 0x9E3779B97F4A7C15ull;
    double e_j = 0, last_t = -1, last_p = 0;
};

Smi g_smi;
Fake g_fake;
gt_dvfs_backend g_backend{};    // caller-supplied knob setter (none by default)
bool g_backend_changed = false;  // the backend changed a knob since the last restore
std::mutex g_mu;
std::atomic<bool> g_busy{false};

const char *smi_str(amdsmi_status_t s) {
    const char *str = nullptr;
    if (amdsmi_status_code_to_string(s, &str) == AMDSMI_STATUS_SUCCESS && str) return str;
    return "unknown amd-smi status";
}

// Locate /sys/class/drm/cardN/device/hwmon/hwmonM (the one holding
// power1_input) for the PCI address of the HIP device; "" if none.
std::string find_hwmon_dir(const DeviceInfo &d) {
    DIR *drm = opendir("/sys/class/drm");
    if (!drm) return "";
    std::string found;
    while (struct dirent *e = readdir(drm)) {
        if (strncmp(e->d_name, "card", 4) != 0 || strchr(e->d_name, '-')) continue;
        std::string dev = std::string("/sys/class/drm/") + e->d_name + "/device";
        char real[PATH_MAX];
        if (!realpath(dev.c_str(), real)) continue;
        const char *base = strrchr(real, '/');
        unsigned dom = 0, bus = 0, slot = 0, fn = 0;
        if (!base || sscanf(base + 1, "%x:%x:%x.%x", &dom, &bus, &slot, &fn) != 4) continue;
        if ((int)dom != d.pci_domain || (int)bus != d.pci_bus || (int)slot != d.pci_device) continue;
        DIR *hw = opendir((dev + "/hwmon").c_str());
        if (!hw) continue;
        while (struct dirent *h = readdir(hw)) {
            if (strncmp(h->d_name, "hwmon", 5) != 0) continue;
            const std::string dir = dev + "/hwmon/" + h->d_name;
            if (access((dir + "/power1_input").c_str(), R_OK) == 0) {
                found = dir;
                break;
            }
        }
        closedir(hw);
        if (!found.empty()) break;
    }
    closedir(drm);
    return found;
}

// One microwatt value from a hwmon file of this device, in W; NaN if absent.
double read_hwmon_file_w(const std::string &dir, const char *name) {
    if (dir.empty()) return NAN;
    const int fd = open((dir + "/" + name).c_str(), O_RDONLY | O_CLOEXEC);
    if (fd < 0) return NAN;
    char buf[64];
    const ssize_t n = pread(fd, buf, sizeof buf - 1, 0);
    close(fd);
    if (n <= 0) return NAN;
    buf[n] = 0;
    char *end = nullptr;
    const double uw = strtod(buf, &end);
    return end == buf ? NAN : uw * 1e-6;
}

double read_hwmon_w(int fd) {
    char buf[64];
    const ssize_t n = pread(fd, buf, sizeof buf - 1, 0);
    if (n <= 0) return NAN;
    buf[n] = 0;
    char *end = nullptr;
    const double uw = strtod(buf, &end);
    return end == buf ? NAN : uw * 1e-6;
}

int smi_open_locked() {
    if (g_smi.open) return GT_OK;
    const State &st = state();
    if (st.flags & GT_INIT_HOST_ONLY) return set_error(GT_E_STATE, "sensor: host-only mode");
    amdsmi_status_t s = amdsmi_init(AMDSMI_INIT_AMD_GPUS);
    if (s != AMDSMI_STATUS_SUCCESS) return set_error(GT_E_SENSOR, "amdsmi_init: %s", smi_str(s));
    uint32_t ns = 0;
    s = amdsmi_get_socket_handles(&ns, nullptr);
    if (s != AMDSMI_STATUS_SUCCESS || ns == 0)
        return set_error(GT_E_SENSOR, "amd-smi: no sockets (%s)", smi_str(s));
    std::vector<amdsmi_socket_handle> socks(ns);
    amdsmi_get_socket_handles(&ns, socks.data());
    for (uint32_t i = 0; i < ns && !g_smi.open; ++i) {
        uint32_t np = 0;
        if (amdsmi_get_processor_handles(socks[i], &np, nullptr) != AMDSMI_STATUS_SUCCESS) continue;
        std::vector<amdsmi_processor_handle> procs(np);
        amdsmi_get_processor_handles(socks[i], &np, procs.data());
        for (uint32_t j = 0; j < np; ++j) {
            amdsmi_bdf_t bdf;
            if (amdsmi_get_gpu_device_bdf(procs[j], &bdf) != AMDSMI_STATUS_SUCCESS) continue;
            if ((int)bdf.bus_number == st.dev.pci_bus && (int)bdf.device_number == st.dev.pci_device &&
                (int)bdf.domain_number == st.dev.pci_domain) {
                g_smi.h = procs[j];
                g_smi.open = true;
                break;
            }
        }
    }
    if (!g_smi.open)
        return set_error(GT_E_SENSOR, "amd-smi: no processor matches PCI %04x:%02x:%02x",
                         st.dev.pci_domain, st.dev.pci_bus, st.dev.pci_device);
    uint64_t acc = 0, ts = 0;
    float res = 0;
    if (amdsmi_get_energy_count(g_smi.h, &acc, &res, &ts) == AMDSMI_STATUS_SUCCESS && res > 0)
        g_smi.energy_res_j = res * 1e-6;
    g_smi.hwmon_dir = find_hwmon_dir(st.dev);
    g_smi.hwmon_fd = g_smi.hwmon_dir.empty() ? -1
                                             : open((g_smi.hwmon_dir + "/power1_input").c_str(), O_RDONLY | O_CLOEXEC);
    g_smi.metrics_t = -1;
    return GT_OK;
}

// Re-read the slow metrics (about 1 Hz upstream) at most every 50 ms.
int refresh_metrics_locked(double now) {
    if (g_smi.metrics_t >= 0 && now - g_smi.metrics_t < 0.05) return GT_OK;
    amdsmi_gpu_metrics_t m;
    amdsmi_status_t s = amdsmi_get_gpu_metrics_info(g_smi.h, &m);
    if (s != AMDSMI_STATUS_SUCCESS) return set_error(GT_E_SENSOR, "gpu metrics: %s", smi_str(s));
    gt_sensor_sample &c = g_smi.cached;
    const uint16_t NA16 = 0xFFFF;
    c.power_w = m.current_socket_power != NA16 ? (double)m.current_socket_power
                                               : (m.average_socket_power != NA16 ? (double)m.average_socket_power : NAN);
    uint64_t acc = 0, ts = 0;
    float res = 0;
    if (amdsmi_get_energy_count(g_smi.h, &acc, &res, &ts) == AMDSMI_STATUS_SUCCESS) {
        if (acc < g_smi.last_energy_raw) g_smi.energy_wrap_j += (double)g_smi.last_energy_raw * g_smi.energy_res_j;
        g_smi.last_energy_raw = acc;
        c.energy_j = g_smi.energy_wrap_j + (double)acc * g_smi.energy_res_j;
        c.energy_t_s = ts * 1e-9;
    } else {
        c.energy_j = NAN;
        c.energy_t_s = NAN;
    }
    double sum = 0;
    int cnt = 0;
    for (int i = 0; i < AMDSMI_MAX_NUM_GFX_CLKS; ++i)
        if (m.current_gfxclks[i] != NA16 && m.current_gfxclks[i] != 0) {
            sum += m.current_gfxclks[i];
            ++cnt;
        }
    c.sclk_mhz = cnt ? sum / cnt : (m.current_gfxclk != NA16 ? (double)m.current_gfxclk : NAN);
    c.mclk_mhz = m.current_uclk != NA16 ? (double)m.current_uclk : NAN;
    c.volt_v = (m.voltage_gfx != NA16 && m.voltage_gfx != 0) ? m.voltage_gfx * 1e-3 : NAN;
    c.temp_c = m.temperature_hotspot != NA16 ? (double)m.temperature_hotspot : NAN;
    // the firmware's timestamp of this table (10 ns units) tells a refreshed
    // table from a re-read of the same one; the energy accumulator's
    // timestamp stands in when the table carries none
    if (m.firmware_timestamp != 0 && m.firmware_timestamp != UINT64_MAX)
        c.metrics_t_s = (double)m.firmware_timestamp * 1e-8;
    else
        c.metrics_t_s = c.energy_t_s;
    g_smi.metrics_t = now;
    return GT_OK;
}

double gauss(uint64_t &state) {
    auto next = [&state]() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    const double u1 = ((next() >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (next() >> 11) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

constexpr double kFakeDefaultMhz = 2400.0, kFakeMinMhz = 500.0;

// Under a power cap the (fake) firmware runs the highest clock, on a 0.01 MHz
// grid over 500..2400 MHz, whose loaded power P*(f) stays within the cap;
// when even 500 MHz exceeds it, 500 MHz (the cap is then not met).  A scan
// from the top (P* need not be monotone with the literal Eq. 3), memoised
// per (cap, model): the sensor asks at every sample.
double fake_capped_clock(double cap_w) {
    static double memo_cap = -1, memo_f = 0;
    static gt_power_model memo_model{};
    const gt_power_model &m = g_fake.model;
    if (cap_w == memo_cap && memcmp(&m, &memo_model, sizeof m) == 0) return memo_f;
    double f = kFakeMinMhz;
    for (int64_t k = (int64_t)llround((kFakeDefaultMhz - kFakeMinMhz) * 100); k >= 0; --k) {
        const double fk = kFakeMinMhz + 0.01 * (double)k;
        if (gt_power_model_eval(&m, fk) <= cap_w) {
            f = fk;
            break;
        }
    }
    memo_cap = cap_w;
    memo_model = m;
    memo_f = f;
    return f;
}

// Record the knob about to be set (kind and value, one line).
bool write_state_file(const gt_clock &clk) {
    const std::string path = dvfs_state_path();
    FILE *f = fopen(path.c_str(), "w");
    if (!f) return false;
    const bool ok = fprintf(f, "%d %d\n", clk.kind, clk.value) > 0;
    return fclose(f) == 0 && ok;
}

}  // namespace

int sensor_open() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (state().flags & GT_INIT_FAKE_SENSOR) {
        if (!g_fake.have_model) return set_error(GT_E_SENSOR, "fake sensor: call gt_fake_sensor_model");
        return GT_OK;
    }
    return smi_open_locked();
}

void sensor_close() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_smi.open) {
        if (g_smi.hwmon_fd >= 0) close(g_smi.hwmon_fd);
        amdsmi_shut_down();
        g_smi = Smi();
    }
    g_fake.e_j = 0;
    g_fake.last_t = -1;
}

void sensor_set_busy(bool busy) { g_busy.store(busy); }

int sensor_read(gt_sensor_sample *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    const State &st = state();
    out->t_s = now_s();
    if (st.flags & GT_INIT_FAKE_SENSOR) {
        if (!g_fake.have_model) return set_error(GT_E_SENSOR, "fake sensor: no model");
        double f = st.clock.kind == GT_CLOCK_SCLK_MHZ ? st.clock.value : kFakeDefaultMhz;
        if (st.clock.kind == GT_CLOCK_POWER_CAP_W) f = fake_capped_clock(st.clock.value);
        double p = g_busy.load() ? gt_power_model_eval(&g_fake.model, f) : g_fake.model.p_idle;
        p += g_fake.noise_w * gauss(g_fake.rng);
        if (g_fake.last_t >= 0) g_fake.e_j += g_fake.last_p * (out->t_s - g_fake.last_t);
        g_fake.last_t = out->t_s;
        g_fake.last_p = p;
        out->power_w = p;
        out->energy_j = g_fake.e_j;
        out->energy_t_s = out->t_s;
        out->sclk_mhz = f;
        out->mclk_mhz = NAN;
        out->volt_v = NAN;
        out->temp_c = NAN;
        out->metrics_t_s = out->t_s;
        return GT_OK;
    }
    int rc = smi_open_locked();
    if (rc) return rc;
    rc = refresh_metrics_locked(out->t_s);
    if (rc) return rc;
    const double t = out->t_s;
    *out = g_smi.cached;
    out->t_s = t;
    if (g_smi.hwmon_fd >= 0) {
        const double p = read_hwmon_w(g_smi.hwmon_fd);
        if (std::isfinite(p)) out->power_w = p;
    }
    return GT_OK;
}

double dvfs_requested_mhz() {
    const gt_clock &c = state().clock;
    return c.kind == GT_CLOCK_SCLK_MHZ ? (double)c.value : 0.0;
}

int dvfs_apply(const gt_clock &clk) {
    State &st = state();
    if (clk.kind == GT_CLOCK_DEFAULT) return GT_OK;  // never touches DVFS
    if (clk.kind != GT_CLOCK_SCLK_MHZ && clk.kind != GT_CLOCK_POWER_CAP_W)
        return set_error(GT_E_INVAL, "clock kind %d", clk.kind);
    if (clk.value <= 0) return set_error(GT_E_INVAL, "clock value must be positive");
    if (st.clock.kind == clk.kind && st.clock.value == clk.value) return GT_OK;
    if (st.flags & GT_INIT_FAKE_DVFS) {
        st.clock = clk;
        return GT_OK;
    }
    if (!(st.flags & GT_INIT_ALLOW_DVFS))
        return set_error(GT_E_PERM, "DVFS changes are not enabled (gt_init flag GT_INIT_ALLOW_DVFS)");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_backend.apply) return set_error(GT_E_PERM, "DVFS: no backend registered (gt_dvfs_set_backend)");
    // the state file goes first, so that a crash after the change still
    // leaves a record for the next gt_init to restore from
    if (!write_state_file(clk)) return set_error(GT_E_PERM, "DVFS: cannot write %s", dvfs_state_path().c_str());
    const int rc = g_backend.apply(g_backend.user, st.dev.ordinal, clk.kind, clk.value);
    if (rc != 0) {
        if (!g_backend_changed) unlink(dvfs_state_path().c_str());  // nothing of ours is in force
        return set_error(GT_E_PERM, "DVFS: the backend refused %s = %d (status %d)",
                         clk.kind == GT_CLOCK_SCLK_MHZ ? "clock limit" : "power cap", clk.value, rc);
    }
    g_backend_changed = true;
    st.clock = clk;
    return GT_OK;
}

int dvfs_restore() {
    State &st = state();
    if (st.flags & GT_INIT_FAKE_DVFS) {
        st.clock = gt_clock{GT_CLOCK_DEFAULT, 0};
        return GT_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = GT_OK;
    if (g_backend_changed && g_backend.restore) {
        const int s = g_backend.restore(g_backend.user, st.dev.ordinal);
        if (s != 0)
            rc = set_error(GT_E_PERM, "DVFS: the backend's restore failed (status %d)", s);
        else
            unlink(dvfs_state_path().c_str());
    }
    g_backend_changed = false;
    st.clock = gt_clock{GT_CLOCK_DEFAULT, 0};
    return rc;
}

std::string dvfs_state_path() {
    const DeviceInfo &d = state().dev;
    const char *dir = getenv("TMPDIR");
    char name[96];
    snprintf(name, sizeof name, "/greentune-dvfs-%04x-%02x-%02x.state", d.pci_domain, d.pci_bus, d.pci_device);
    return std::string(dir && *dir ? dir : "/tmp") + name;
}

int dvfs_recover() {
    const std::string path = dvfs_state_path();
    if (access(path.c_str(), F_OK) != 0) return GT_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_backend.restore)
        return set_error(GT_E_STATE, "DVFS: %s records a knob left set by an earlier process; register a "
                         "backend with a restore function before gt_init", path.c_str());
    const int s = g_backend.restore(g_backend.user, state().dev.ordinal);
    if (s != 0) return set_error(GT_E_PERM, "DVFS: restoring the knob recorded in %s failed (status %d)",
                                 path.c_str(), s);
    unlink(path.c_str());
    return GT_OK;
}

int dvfs_settable(double step_mhz, std::vector<double> &out) {
    out.clear();
    if (!(step_mhz > 0)) return set_error(GT_E_INVAL, "step must be positive");
    double lo = kFakeMinMhz, hi = kFakeDefaultMhz;
    if (!(state().flags & GT_INIT_FAKE_DVFS)) {
        std::lock_guard<std::mutex> lk(g_mu);
        int rc = smi_open_locked();
        if (rc) return rc;
        amdsmi_clk_info_t ci;
        amdsmi_status_t s = amdsmi_get_clock_info(g_smi.h, AMDSMI_CLK_TYPE_GFX, &ci);
        if (s != AMDSMI_STATUS_SUCCESS) return set_error(GT_E_SENSOR, "clock info: %s", smi_str(s));
        lo = ci.min_clk;
        hi = ci.max_clk;
    }
    for (double f = lo; f <= hi + 1e-9; f += step_mhz) out.push_back(f);
    if (out.empty() || out.back() < hi) out.push_back(hi);
    return GT_OK;
}

}  // namespace gt

using namespace gt;

extern "C" {

int gt_sensor_read(gt_sensor_sample *s) {
    clear_error();
    if (!s) return set_error(GT_E_INVAL, "gt_sensor_read: null argument");
    if (!state().inited) return set_error(GT_E_STATE, "gt_sensor_read: call gt_init first");
    return sensor_read(s);
}

int gt_settable_clocks(double step_mhz, double *mhz, size_t cap, size_t *n) {
    clear_error();
    if (!n || (cap && !mhz)) return set_error(GT_E_INVAL, "gt_settable_clocks: null argument");
    if (!state().inited) return set_error(GT_E_STATE, "gt_settable_clocks: call gt_init first");
    std::vector<double> v;
    int rc = dvfs_settable(step_mhz, v);
    if (rc) return rc;
    *n = v.size();
    for (size_t i = 0; i < v.size() && i < cap; ++i) mhz[i] = v[i];
    if (v.size() > cap) return set_error(GT_E_CAPACITY, "gt_settable_clocks: %zu clocks", v.size());
    return GT_OK;
}

int gt_dvfs_set_backend(const gt_dvfs_backend *backend) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_backend_changed) return set_error(GT_E_STATE, "gt_dvfs_set_backend: restore the knob first (gt_shutdown)");
    if (backend && !backend->apply) return set_error(GT_E_INVAL, "gt_dvfs_set_backend: apply is required");
    g_backend = backend ? *backend : gt_dvfs_backend{};
    return GT_OK;
}

int gt_power_cap_range(double *min_w, double *max_w, double *current_w) {
    clear_error();
    if (!min_w || !max_w || !current_w) return set_error(GT_E_INVAL, "gt_power_cap_range: null argument");
    if (!state().inited) return set_error(GT_E_STATE, "gt_power_cap_range: call gt_init first");
    if (state().flags & GT_INIT_FAKE_DVFS) {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_fake.have_model)
            return set_error(GT_E_SENSOR, "gt_power_cap_range: fake DVFS needs gt_fake_sensor_model");
        // fake range: half the model's P_max up to P_max
        *min_w = 0.5 * g_fake.model.p_max;
        *max_w = g_fake.model.p_max;
        *current_w = state().clock.kind == GT_CLOCK_POWER_CAP_W ? (double)state().clock.value : *max_w;
        return GT_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    int rc = smi_open_locked();
    if (rc) return rc;
    // amd-smi first; fields it leaves at 0 come from the hwmon files
    // power1_cap_min / power1_cap_max / power1_cap; NaN where neither knows
    amdsmi_power_cap_info_t pc{};
    const bool smi_ok = amdsmi_get_power_cap_info(g_smi.h, 0, &pc) == AMDSMI_STATUS_SUCCESS;
    auto pick = [&](uint64_t smi_uw, const char *file) {
        return smi_ok && smi_uw > 0 ? smi_uw * 1e-6 : read_hwmon_file_w(g_smi.hwmon_dir, file);
    };
    *min_w = pick(pc.min_power_cap, "power1_cap_min");
    *max_w = pick(pc.max_power_cap, "power1_cap_max");
    *current_w = pick(pc.power_cap, "power1_cap");
    if (std::isnan(*min_w) && std::isnan(*max_w) && std::isnan(*current_w))
        return set_error(GT_E_SENSOR, "power cap: neither amd-smi nor hwmon reports it");
    return GT_OK;
}

int gt_dvfs_state(gt_clock *current) {
    clear_error();
    if (!current) return set_error(GT_E_INVAL, "gt_dvfs_state: null argument");
    *current = state().clock;
    return current->kind != GT_CLOCK_DEFAULT ? 1 : 0;
}

int gt_fake_sensor_model(const gt_power_model *model, double noise_w, uint64_t seed) {
    clear_error();
    if (!model || noise_w < 0) return set_error(GT_E_INVAL, "gt_fake_sensor_model: bad argument");
    std::lock_guard<std::mutex> lk(g_mu);
    g_fake.model = *model;
    g_fake.have_model = true;
    g_fake.noise_w = noise_w;
    g_fake.rng = seed ^ 0x9E3779B97F4A7C15ull;
    return GT_OK;
}

}  // extern "C"
