/*
 * greentune -- energy-aware auto-tuning of a parameterised 2-D convolution on
 * one MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The method is the one of "Going green: optimizing GPUs for energy
 * efficiency through model-steered auto-tuning" (Schoonhoven, Veenboer,
 * van Werkhoven, Batenburg, 2022):
 *   - every kernel configuration of a restricted tune space is launched and
 *     measured for time and energy (sections III.B, III.C, IV);
 *   - energy is a representative (median) power reading times elapsed time
 *     (section III.A);
 *   - a power-versus-clock model, Eq. 2 with the voltage estimate of Eq. 3,
 *     is fitted by Levenberg-Marquardt least squares to a few power readings
 *     (sections III.A and V.D), and the clock search is cut to +-10 % around
 *     the clock where the model's energy estimate P*(f)/f is lowest.
 *
 * Conventions for every function below:
 *   - returns GT_OK (0) or a negative GT_E_* code; gt_last_error() then gives
 *     a message (thread-local, valid until the next call on that thread);
 *   - the caller owns every buffer.  Device pointers are plain HIP device
 *     addresses (e.g. torch tensor data pointers); hip_stream is a
 *     hipStream_t (NULL = the null stream).  The library keeps no reference
 *     to a caller buffer after the call returns;
 *   - all row-major arrays are dense (pitch = width).
 */
#ifndef GREENTUNE_H
#define GREENTUNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define GT_OK             0
#define GT_E_INVAL       -1  /* bad argument (null pointer, size, enum) */
#define GT_E_UNSUPPORTED -2  /* configuration outside the kernel's limits (threads, LDS, filter width) */
#define GT_E_PERM        -3  /* DVFS change not permitted (or not allowed by gt_init flags) */
#define GT_E_SENSOR      -4  /* no power sensor, or stale readings */
#define GT_E_HIP         -5  /* HIP runtime error */
#define GT_E_NOMEM       -6  /* host allocation failed */
#define GT_E_CAPACITY    -7  /* output array too small; the *n_total style outputs are still written */
#define GT_E_STATE       -8  /* library not initialised, or a GPU call in host-only mode */

/* ---- problem kinds ---- */
#define GT_XCORR_F32        0  /* single-channel FP32 cross-correlation, valid region */
#define GT_IGEMM_BF16_MFMA  1  /* multi-channel NHWC conv, BF16 in, FP32 accumulate, MFMA */
#define GT_IGEMM_F32_VALU   2  /* the same contraction in FP32 on the vector ALUs */

/* A tunable kernel configuration (section IV: thread-block dimensions, work
 * per thread, shared-memory use and read path are the tunable style).
 *   block_size_x/y   workgroup shape in threads; bx*by <= 1024
 *   tile_size_x/y    outputs per thread along x / y (1..8)
 *   use_lds_padding  0/1: pad each LDS row by 4 floats
 *   read_path        0: stage the input halo in LDS; 1: read global memory directly
 * The implicit-GEMM kinds take their kernel from the problem (see
 * conv2d_run), with one tunable: for GT_IGEMM_BF16_MFMA, tile_size_y = 4 or
 * 8 asks for the LDS-staged kernel with that many output rows per workgroup
 * tile where the shape has both (e.g. 3x3 with c_out a multiple of 64: 4
 * rows of two 32-channel groups, the default, or 8 rows of 64 channels;
 * 5x5 with c_in 64: 8 rows of 32 channels, the default, or 4 rows of 64).
 * The fastest instance is the default; it need not be the most
 * energy-efficient one.  Any other value, and the other fields, leave the
 * choice to the library; GT_IGEMM_F32_VALU ignores the config. */
typedef struct {
    int32_t block_size_x, block_size_y, tile_size_x, tile_size_y, use_lds_padding, read_path;
} gt_conv_config;

/* Problem description.
 * GT_XCORR_F32: n = c_in = c_out = 1, pad = 0.  Input (out_h+filt_h-1) x
 *   (out_w+filt_w-1) FP32, filter filt_h x filt_w FP32, output out_h x out_w FP32:
 *   out[y][x] = sum_{i,j} in[y+i][x+j] * w[i][j]   (no filter flip).
 * GT_IGEMM_*: stride 1, zero padding pad_h/pad_w; input NHWC [n][H][W][c_in]
 *   with H = out_h + filt_h - 1 - 2*pad_h (likewise W); weights KRSC
 *   [c_out][filt_h][filt_w][c_in]; output NHWC FP32 [n][out_h][out_w][c_out]:
 *   out[b][y][x][k] = sum_{r,s,c} in[b][y+r-pad_h][x+s-pad_w][c] * wt[k][r][s][c].
 *   Input and weights are BF16 for GT_IGEMM_BF16_MFMA and FP32 for GT_IGEMM_F32_VALU. */
typedef struct {
    int32_t kind;
    int32_t n, c_in, c_out, out_h, out_w, filt_h, filt_w, pad_h, pad_w;
} gt_problem;

/* DVFS knob (section III.C: clock frequency or power limit as tunables). */
#define GT_CLOCK_DEFAULT     0  /* leave DVFS untouched; value ignored */
#define GT_CLOCK_SCLK_MHZ    1  /* upper limit of the graphics clock, MHz */
#define GT_CLOCK_POWER_CAP_W 2  /* socket power cap, W */
typedef struct { int32_t kind; int32_t value; } gt_clock;

/* Tune-space descriptor: one value list per tunable (order as in
 * gt_conv_config).  Enumeration is the Cartesian product in that order, last
 * parameter fastest, filtered by the restrictions (section IV). */
#define GT_SPACE_DEDUP_DIRECT 1u  /* drop read_path=1 with use_lds_padding=1 (same kernel) */
typedef struct {
    const int32_t *values[6];
    int32_t counts[6];
    uint32_t flags;
    int32_t max_threads;      /* 0 = device limit (1024) */
    int64_t lds_limit_bytes;  /* 0 = device's max shared memory per block (needs gt_init) */
} gt_space_desc;

/* Measurement options (section III.B: the kernel is repeated for a window,
 * 1 s by default, because the sensor refreshes slowly and settles late). */
typedef struct {
    double window_s;          /* timed window; <= 0 -> 1.0 */
    double discard_s;         /* leading samples dropped before the median; < 0 -> 0.3 */
    double sample_period_ms;  /* sensor poll period; <= 0 -> 1.0 */
    int32_t min_launches;     /* at least this many launches; <= 0 -> 10 */
    int32_t warmup_launches;  /* untimed launches first; < 0 -> 3 */
    int32_t use_graph;        /* 1: capture a group of launches into a HIP graph once and replay it
                               * for the window (no host launch gaps between short kernels; the
                               * group is as many launches as take about 1 ms, at most 256);
                               * 0: launch one by one */
} gt_measure_opts;

/* One measurement (section III.B observer fields; section III.C metrics). */
typedef struct {
    double t_run_s;           /* mean time per launch over the window (HIP events) */
    double p_median_w;        /* median socket power over the kept samples */
    double p_min_w, p_max_w;
    double e_run_j;           /* p_median_w * t_run_s */
    double e_run_counter_j;   /* energy-counter delta over the window / launches */
    double gflops;            /* flops / t_run / 1e9 */
    double gflops_per_w;      /* flops / e_run / 1e9  (= GFLOP/J) */
    double sclk_req_mhz;      /* requested clock limit (0 = default) */
    double sclk_act_mhz;      /* mean graphics clock of the GPU-metrics updates first seen
                               * inside the kept window (gt_window_clock); NaN if none */
    double mclk_mhz;          /* memory clock */
    double volt_v;            /* graphics voltage, NaN if not reported */
    double temp_c;            /* hotspot temperature at the end of the window */
    double window_s;          /* actual timed window */
    int64_t launches, n_samples, n_used;
    int32_t throttled;        /* actual clock > 2 % below the requested limit (0 when
                               * sclk_act_mhz is NaN) */
    int32_t flags;            /* bit 0: fake sensor, bit 1: fake DVFS */
} gt_measurement;

/* Fitted power model, Eq. 2 with Eq. 3:
 *   P*(f) = min(p_max, p_idle + alpha * f * v(f)^2),
 *   v(f)  = 1 for f < tau, 1 + beta * (f - tau) for f >= tau   (f in MHz).
 * The printed Eq. 3 is discontinuous at tau; literal_eq3 = 1 evaluates it as
 * printed (v = beta * (f - tau) above tau).  With measured voltage
 * (v_measured = 1) beta and tau are unused and v comes from the readings. */
typedef struct {
    double p_idle, alpha, beta, tau_mhz, p_max;
    double rss;               /* residual sum of squares of the fit, W^2 */
    /* Covariance of the fitted parameters, row-major 4 x 4 in the order
     * (p_idle W, alpha W/MHz, beta 1/MHz, tau_mhz MHz): s^2 (J^T J)^-1 at the
     * solution, J the Jacobian of the modelled power over the free parameters
     * (readings clipped at p_max contribute nothing), s^2 = rss / (n - k) for
     * n readings and k free parameters (4, or 2 -- p_idle and alpha -- with
     * measured voltage).  NaN where undefined: parameters not fitted, n <= k,
     * or J^T J singular (e.g. beta = 0 leaves tau without influence). */
    double cov[16];
    int32_t v_measured, literal_eq3, iters, status;  /* status 0 = converged */
} gt_power_model;

/* One sensor reading. */
typedef struct {
    double t_s;               /* host steady clock, seconds */
    double power_w;           /* socket power (hwmon power1_input, refreshed every few ms) */
    double energy_j;          /* energy accumulator (monotone, wraps are unwrapped) */
    double energy_t_s;        /* firmware timestamp of that accumulator value, seconds */
    double sclk_mhz, mclk_mhz, volt_v, temp_c;  /* from the GPU metrics table (about 1 Hz) */
    double metrics_t_s;       /* firmware timestamp of the GPU metrics table those four fields
                               * came from, s (the energy accumulator's timestamp when the table
                               * carries none; NaN if neither); the fake sensor gives t_s */
} gt_sensor_sample;

/* ---- lifecycle ---- */
#define GT_INIT_FAKE_SENSOR 1u  /* synthetic power: P*(f) of gt_fake_sensor_model at the set clock */
#define GT_INIT_FAKE_DVFS   2u  /* clock knob is recorded, hardware untouched */
#define GT_INIT_ALLOW_DVFS  4u  /* permit real DVFS changes through the registered backend */
#define GT_INIT_HOST_ONLY   8u  /* no HIP calls at all (host arithmetic only) */

/* Select the HIP device, open the power sensor (amd-smi) and DVFS controller.
 * Idempotent for the same arguments.  Errors: GT_E_HIP (no such device),
 * GT_E_SENSOR is NOT returned here -- a missing sensor is reported by the
 * first measurement. */
int gt_init(int device_ordinal, uint32_t flags);
/* Restore any DVFS change made through the library, stop the sensor. */
int gt_shutdown(void);
const char *gt_last_error(void);
/* Library version string. */
const char *gt_version(void);

/* ---- the four calls of the method ---- */

/* Launch one convolution asynchronously on hip_stream.
 * problem/config as above; clock: knob applied first (synchronously, only if
 * it differs from the current setting; GT_CLOCK_DEFAULT never touches DVFS).
 * d_in, d_filt, d_out: device pointers laid out as in gt_problem; the
 * caller keeps them valid until the launch has run.  Every index is a 32-bit
 * element offset: inputs of 2^31 elements or more are GT_E_INVAL.
 * Implicit GEMM, BF16 (c_in 32 or 64, c_out a multiple of 32, square
 * filters): filters of 1, 3, 5, 7, 9 (and 17 for c_in 32) with a 16-byte
 * aligned output run the LDS-staged MFMA kernel (workgroups of 4 or 8 output
 * rows x 64 pixels x 32 or 64 output channels, persistent over tiles); other
 * filter sizes and unaligned outputs the global-load MFMA kernel.  FP32
 * (c_in 32 or 64, c_out a multiple of 64): the register-tiled vector kernel.
 * Errors: GT_E_INVAL (null pointer, sizes), GT_E_UNSUPPORTED (config outside
 * the restricted space or filter width not instantiated: single-channel
 * filt_w in {3,5,9,17} with tile sizes 1..8), GT_E_PERM (clock knob
 * refused), GT_E_HIP (launch failure). */
int conv2d_run(const gt_problem *problem, const gt_conv_config *config, gt_clock clock,
               const void *d_in, const void *d_filt, void *d_out, void *hip_stream);

/* One part of a convolution: the work of conv2d_run split into n_parts
 * contiguous ranges of the kernel's output tiles (part k covers tiles
 * [T*k/n, T*(k+1)/n) of T), so that a long convolution can be issued in
 * pieces between which other work runs (the serving form).  Every output
 * element belongs to exactly one part and is computed exactly as by
 * conv2d_run; the parts may run in any order, on any streams, once each.
 * n_parts > 1 is for GT_IGEMM_BF16_MFMA on its LDS-staged kernel (square
 * filter of an instantiated size, c_in 32 or 64, 16-byte aligned output);
 * otherwise GT_E_UNSUPPORTED.  n_parts == 1 is conv2d_run.  GT_E_INVAL for
 * part outside [0, n_parts). */
int conv2d_run_part(const gt_problem *problem, const gt_conv_config *config, gt_clock clock, int32_t part,
                    int32_t n_parts, const void *d_in, const void *d_filt, void *d_out, void *hip_stream);

/* Enumerate the restricted tune space (section IV) into out[0..capacity).
 * *n_total always receives the full count; GT_E_CAPACITY if capacity is too
 * small (call with capacity 0 to size the array). */
int tune_space_enumerate(const gt_problem *problem, const gt_space_desc *space,
                         gt_conv_config *out, size_t capacity, size_t *n_total);

/* Measure time and energy of one (problem, config, clock) point (sections
 * III.A-III.B): apply the clock, run warm-up launches, then launch
 * back-to-back on hip_stream for the window while a sampler thread polls the
 * power sensor; t_run from HIP events, energy = median power of the samples
 * after discard_s times t_run, cross-checked with the energy counter.
 * Blocks until done; exclusive use of the device is assumed.
 * Errors: as conv2d_run, plus GT_E_SENSOR (no usable samples). */
int measure_time_energy(const gt_problem *problem, const gt_conv_config *config, gt_clock clock,
                        const gt_measure_opts *opts, const void *d_in, const void *d_filt,
                        void *d_out, void *hip_stream, gt_measurement *rec);

/* Levenberg-Marquardt least-squares fit of Eq. 2 (+ Eq. 3 unless v_or_null
 * is given) to n readings (f_mhz[i], p_w[i]).  p_max_w is held fixed (the
 * paper takes it from the measured maximum or the TDP).  Host-only, FP64.
 * Bounds: p_idle, alpha, beta >= 0; tau within [min f, max f].  Needs n >= 2
 * with measured voltage, n >= 4 otherwise.  Errors: GT_E_INVAL. */
int fit_power_model(const double *f_mhz, const double *p_w, const double *v_or_null, size_t n,
                     double p_max_w, gt_power_model *out);

/* ---- helpers of the method ---- */

/* P*(f) of a fitted model (Eq. 2/3); NaN on a null model.  For a model
 * fitted with measured voltage, v is taken as 1 (the fit, not the curve, is
 * what that variant provides). */
double gt_power_model_eval(const gt_power_model *model, double f_mhz);
/* Throttling clock: where the unclipped model p_idle + alpha f v(f)^2 reaches
 * p_max (bisection); +inf if it never does below 1e7 MHz. */
double gt_power_model_throttle_clock(const gt_power_model *model);
/* Model-optimal clock: argmin of the energy estimate of section V.D,
 * P*(f)/f, over the settable clocks the device can hold, settable[i] <= f_thr
 * (the paper takes performance as linear in the clock, and fits and searches,
 * only up to where throttling starts: Fig. 8 and section V.D); the lowest
 * settable clock when every one lies above f_thr.  Ties (relative gap
 * <= 1e-12) go to the higher clock.  Then the band: the settable clocks
 * within [(1-rel_half) f_opt, (1+rel_half) f_opt], ascending (rel_half = 0.1
 * in the paper).
 * GT_E_CAPACITY if cap is too small (*n_band still written). */
int gt_power_model_band(const gt_power_model *model, const double *settable, size_t n,
                        double rel_half, double *f_opt, double *band, size_t cap, size_t *n_band);
/* Energy per run from a power trace (section III.A): median of the samples
 * with t_start + discard_s <= t <= t_stop (mean of the middle two for an even
 * count) times (t_stop - t_start) / n_runs.  GT_E_SENSOR if no sample is kept. */
int gt_energy_from_samples(const double *t_s, const double *p_w, size_t n, double t_start,
                           double t_stop, int64_t n_runs, double discard_s, double *e_run_j,
                           double *p_median_w, size_t *n_used);
/* Graphics clock over a window of sensor readings (times ascending): the mean
 * sclk_mhz of the GPU-metrics updates first observed at t_lo <= t_s <= t_hi.
 * An update is a change of metrics_t_s from the reading before; readings
 * before t_lo only establish the timestamp in force when the window opens
 * (with none, the first reading in the window does), so a clock reported
 * before the window is never counted.  The first observation of an update
 * lags it by at most the sensor's metrics re-read period (50 ms) plus the
 * poll period.  *sclk_mhz = NaN and *n_fresh = 0 when no update is seen.
 * Errors: GT_E_INVAL. */
int gt_window_clock(const gt_sensor_sample *samples, size_t n, double t_lo, double t_hi, double *sclk_mhz,
                    size_t *n_fresh);
/* The readings of the most recent measure_time_energy / measure_load window
 * in this process (every reading the sampler took, the stabilisation prefix
 * included), oldest first, and the window's host-time bounds: energy per run
 * is gt_energy_from_samples over them with t_start, t_stop, the launch count
 * and discard_s (readings with a non-finite power left out), with
 * (t_stop - t_start) / launches replaced by the HIP-event time per launch.
 * GT_E_STATE if no window has been measured; GT_E_CAPACITY as elsewhere. */
int gt_measure_last_window(gt_sensor_sample *out, size_t capacity, size_t *n, double *t_start, double *t_stop);
/* Objective selection over a measurement table (section V.A):
 * objective 0 = time (race-to-idle): min t_run, then e_run, then index;
 * objective 1 = energy: min e_run, then t_run, then index. */
int gt_select(const gt_measurement *recs, size_t n, int objective, size_t *index);
/* Pareto front of a measurement table (section V.A, the GFLOP/s versus
 * GFLOP/s/W front): on_front[k] = 1 when no record j has t_run <= and
 * e_run <= those of record k with at least one strictly lower, else 0.
 * Records with equal (t_run, e_run) are all on the front or all off it.
 * Errors: GT_E_INVAL. */
int gt_pareto(const gt_measurement *recs, size_t n, int32_t *on_front);
/* Algorithmic flop count: 2 per filter tap per output (padded taps counted). */
double gt_problem_flops(const gt_problem *problem);
/* LDS bytes the config's workgroup allocates (0 for read_path 1 and for the
 * implicit-GEMM kinds' fixed tiles, which report their own static size). */
int gt_conv_lds_bytes(const gt_problem *problem, const gt_conv_config *config, int64_t *bytes);

/* ---- sensor and DVFS ---- */

/* One reading of the power sensor (amd-smi GPU metrics, or the fake sensor). */
int gt_sensor_read(gt_sensor_sample *s);
/* Background sampler: a native thread reads the sensor every period_ms
 * from gt_sampler_start until gt_sampler_stop, which joins it and copies up
 * to capacity samples (oldest first) into out; *n receives the total.
 * GT_E_CAPACITY if capacity < *n (the first capacity samples are written);
 * GT_E_SENSOR if no reading succeeded; GT_E_STATE if not started / already
 * running.  One sampler per process. */
int gt_sampler_start(double period_ms);
int gt_sampler_stop(gt_sensor_sample *out, size_t capacity, size_t *n);
/* Tell the fake sensor whether kernels are running (it reports idle power
 * otherwise); no effect on the hardware sensor. */
int gt_sensor_busy(int busy);

/* Settable graphics-clock list in MHz, ascending (DVFS range of the device,
 * at step_mhz spacing; the fake DVFS backend reports 500..2400).
 * GT_E_CAPACITY if cap is too small (*n still written). */
int gt_settable_clocks(double step_mhz, double *mhz, size_t cap, size_t *n);
/* Stale-sensor test on a power trace (times ascending, s; readings, W):
 * 1 when the trace spans at least min_span_s and every reading equals the
 * first, else 0 (negative error code on bad arguments).  measure_time_energy
 * and measure_load apply it to the kept window of the hardware sensor with a
 * 0.5 s span and fail with GT_E_SENSOR on a stale reading. */
int gt_sensor_stale(const double *t_s, const double *p_w, size_t n, double min_span_s);

/* DVFS backend: the library changes no device setting itself.  A caller
 * with the privileges to change the graphics-clock limit or the socket power
 * cap (the two knobs of sections III.C and V.C) registers functions that do
 * it; with GT_INIT_ALLOW_DVFS, a measurement's clock argument then calls
 * apply(user, device_ordinal, kind, value) (kind GT_CLOCK_SCLK_MHZ or
 * GT_CLOCK_POWER_CAP_W; value in MHz or W; 0 = success) whenever the knob
 * changes, and gt_shutdown calls restore(user, device_ordinal) (may be
 * NULL) to return the device to its defaults.  The structure is copied;
 * NULL unregisters.  GT_E_STATE while a knob set through the backend is
 * still in force.  Without a backend, DVFS requests fail with GT_E_PERM.
 * Before each apply the library records the knob in a state file
 * ($TMPDIR or /tmp, greentune-dvfs-<pci domain>-<bus>-<device>.state),
 * removed after a successful restore; gt_init with GT_INIT_ALLOW_DVFS finds
 * a file a crashed process left and calls restore first (GT_E_STATE if no
 * backend with a restore function is registered then). */
typedef struct {
    int (*apply)(void *user, int32_t device_ordinal, int32_t kind, int32_t value);
    int (*restore)(void *user, int32_t device_ordinal);
    void *user;
} gt_dvfs_backend;
int gt_dvfs_set_backend(const gt_dvfs_backend *backend);

/* Power-cap range of the device in W (amd-smi: minimum and maximum settable
 * cap, and the cap in force), the range a power-cap sweep samples (the
 * comparison of power capping with clock tuning, section V.C).  With
 * GT_INIT_FAKE_DVFS: 0.5 * P_max .. P_max of the gt_fake_sensor_model model,
 * and under a fake cap the fake sensor reports the highest clock (0.01 MHz
 * grid, 500..2400 MHz) whose model power fits within the cap, or 500 MHz.
 * A field amd-smi reports as 0 is read from the hwmon files power1_cap_min,
 * power1_cap_max, power1_cap; NaN where neither reports it (GT_E_SENSOR if
 * none of the three is known). */
int gt_power_cap_range(double *min_w, double *max_w, double *current_w);
/* Current DVFS state: 1 if a knob set through the library is active. */
int gt_dvfs_state(gt_clock *current);
/* Synthetic power for GT_INIT_FAKE_SENSOR: readings follow the model at the
 * clock the (fake or real) DVFS controller reports, plus zero-mean noise of
 * the given standard deviation (deterministic, seeded).  Idle power applies
 * when no kernel is running in the window. */
int gt_fake_sensor_model(const gt_power_model *model, double noise_w, uint64_t seed);

/* ---- batching: many convolutions in one persistent launch ---- */

/* One single-channel FP32 cross-correlation of a batch (layouts as for
 * GT_XCORR_F32; all device pointers). */
typedef struct {
    const void *d_in, *d_filt;
    void *d_out;
    int32_t out_h, out_w, filt_h, filt_w;
} gt_batch_item;

/* Pack n_items convolutions into a device-ready descriptor blob (48 bytes per
 * item) written to host_blob[0..capacity); the caller copies it to device
 * memory (8-byte aligned) and passes that copy to conv2d_run_batched.  All
 * items must share one square filter size (3, 5, 9 or 17); cfg must use the
 * LDS read path with tile sizes in {1, 2, 4, 8}.  *blob_bytes and
 * *total_tiles (workgroup tiles over all items) are always written;
 * GT_E_CAPACITY if capacity < *blob_bytes. */
int gt_batch_pack(const gt_batch_item *items, int32_t n_items, const gt_conv_config *cfg, void *host_blob,
                  size_t capacity, size_t *blob_bytes, int64_t *total_tiles);

/* One persistent launch over every tile of a packed batch: grid_blocks
 * workgroups (0 = resident capacity of the device) stride over the tile
 * list.  Each output equals, bit for bit, what conv2d_run with the same
 * config writes.  Launch only (no allocation, no memset), so it may be
 * captured in a graph.  Errors: GT_E_INVAL, GT_E_UNSUPPORTED, GT_E_HIP. */
int conv2d_run_batched(const void *d_blob, int32_t n_items, int64_t total_tiles, int32_t filt,
                       const gt_conv_config *cfg, int32_t grid_blocks, void *hip_stream);

/* measure_time_energy for a packed batch (sections III.A-III.B applied to
 * the batched launch, for the per-size autotuner's energy objective): the
 * launch of conv2d_run_batched with these arguments is repeated for the
 * window.  flops_per_launch: the batch's algorithmic flops (the sum of
 * gt_problem_flops over its items), from which rec->gflops and
 * rec->gflops_per_w are derived.  Errors: as conv2d_run_batched and
 * measure_time_energy. */
int measure_batched_time_energy(const void *d_blob, int32_t n_items, int64_t total_tiles, int32_t filt,
                                const gt_conv_config *cfg, int32_t grid_blocks, double flops_per_launch,
                                gt_clock clock, const gt_measure_opts *opts, void *hip_stream, gt_measurement *rec);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): conv2d_run_batched
 * without the caller's descriptor blob.  Takes the items as in gt_batch_pack
 * (host array, read during the call only) and runs the same persistent
 * kernel, so every output is bit for bit that of conv2d_run_batched with the
 * same items, config and grid.  The descriptors go to a device array the
 * library holds for the life of the process, one per GPU, of
 * GT_BATCH_NOALLOC_MAX_ITEMS 48-byte records (192 KiB); they are written
 * there by small kernels on hip_stream ahead of the launch (the descriptors
 * travel as kernel arguments), so the call allocates nothing, on the device
 * or the host, and returns without waiting.  Every call on a GPU shares that
 * array: calls on one stream are ordered, but calls that overlap on one GPU
 * (on different streams, or from several threads) race and give undefined
 * results.  Errors: GT_E_INVAL (n_items outside 1..GT_BATCH_NOALLOC_MAX_ITEMS,
 * bad items), GT_E_UNSUPPORTED (config), GT_E_STATE (no device), GT_E_HIP. */
#define GT_BATCH_NOALLOC_MAX_ITEMS 4096
int conv2d_run_batched_noalloc(const gt_batch_item *items, int32_t n_items, const gt_conv_config *cfg,
                               int32_t grid_blocks, void *hip_stream);

/* Batching for multi-channel BF16 convolutions (the MFMA kind): many
 * convolutions of one shape family -- shared c_in, c_out, square filter and
 * padding, given by `shape` (its n, out_h, out_w are ignored) -- each of
 * one image (n = 1) of its own size, in one persistent launch.  items: as
 * for gt_batch_pack (d_in NHWC BF16 [H][W][c_in], d_filt KRSC BF16, d_out
 * NHWC FP32 [out_h][out_w][c_out], H = out_h + filt - 1 - 2 pad), input and
 * weights 16-byte aligned.  Packs 64-byte descriptors into host_blob, which
 * the caller copies to device memory (8-byte aligned) for
 * conv2d_run_igemm_batched; *blob_bytes and *total_blocks (workgroup blocks of
 * 256 output pixels over all items) are always written, GT_E_CAPACITY if
 * capacity is too small.  The launch runs the global-load MFMA kernel on
 * every block (grid_blocks workgroups along the pixels, 0 = about the
 * resident capacity); each output equals bit for bit what that kernel writes
 * for the convolution alone (conv2d_run takes the LDS-staged kernel where it
 * applies, which sums in another order; both agree within FP32 rounding).
 * Launch only: no allocation, no memset.  Errors: GT_E_INVAL,
 * GT_E_UNSUPPORTED (kind other than GT_IGEMM_BF16_MFMA, non-square filter,
 * c_in not 32 or 64, c_out not a multiple of 32), GT_E_STATE, GT_E_HIP. */
int gt_igemm_batch_pack(const gt_problem *shape, const gt_batch_item *items, int32_t n_items, void *host_blob,
                        size_t capacity, size_t *blob_bytes, int64_t *total_blocks);
int conv2d_run_igemm_batched(const gt_problem *shape, const void *d_blob, int32_t n_items, int64_t total_blocks,
                             int32_t grid_blocks, void *hip_stream);

/* Graph capture of the launches issued on hip_stream between begin and end
 * (hipStreamBeginCapture / EndCapture / Instantiate).  *graph_exec is an
 * opaque executable graph owned by the caller until gt_graph_destroy. */
int gt_graph_begin(void *hip_stream);
int gt_graph_end(void *hip_stream, void **graph_exec);
int gt_graph_launch(void *graph_exec, void *hip_stream);
int gt_graph_destroy(void *graph_exec);

/* ---- search difficulty (section V.B) ---- */

/* Fitness flow graph of a measured tune space: neighbours differ in exactly
 * one tunable, edges point to strictly better (lower) fitness.  PageRank with
 * the given damping (0.85 usual), uniform teleportation, rank of nodes without
 * out-edges spread uniformly.  Writes pagerank[n] and is_minimum[n] when non-
 * null, and for each p_values[k] the proportion of centrality: PageRank mass of
 * the minima with fitness <= p * min(fitness) over the mass of all minima.
 * Host-only.  Errors: GT_E_INVAL. */
int gt_ffg_centrality(const gt_conv_config *cfgs, const double *fitness, size_t n, double damping,
                      const double *p_values, size_t n_p, double *pagerank, int32_t *is_minimum,
                      double *proportion);

/* ---- synthetic full loads (per-GPU power calibration) ---- */

#define GT_LOAD_FP32_FMA   0  /* FP32 FMA chains, the convolution's instruction form, all CUs */
#define GT_LOAD_BF16_MFMA  1  /* BF16 16x16x32 MFMA chains, two waves per SIMD */
#define GT_LOAD_COPY       2  /* device copy through HBM */

/* Measure time and energy of a synthetic kernel that fully loads one unit of
 * the GPU, at a clock, with the same window, sampler and statistics as
 * measure_time_energy.  Such readings calibrate the power model once per GPU
 * and serve every kernel tuned on it (the paper's procedure, section V.D).
 * d_buf: caller-owned device scratch of `bytes` (overwritten): >= 4 MiB
 * covers every kind.  rec->gflops holds the load's rate: GFLOP/s for the
 * FMA and MFMA loads, GB/s of read + written bytes for the copy.
 * Errors: as measure_time_energy; GT_E_INVAL for an unknown kind or a
 * small buffer. */
int measure_load(int32_t kind, gt_clock clock, const gt_measure_opts *opts, void *d_buf, size_t bytes,
                 void *hip_stream, gt_measurement *rec);

/* ---- roofline probes ---- */

/* Measure the achievable FP32 vector FMA rate (FMA with one SGPR operand, the
 * form the convolution issues; packed FP32 is not used) and the device copy
 * bandwidth (read + write bytes), on hip_stream.  d_buf: caller-owned device
 * scratch of `bytes` >= 4 MiB (overwritten).  Blocks until done.
 * Errors: GT_E_INVAL (buffer), GT_E_STATE (no device), GT_E_HIP. */
int gt_roofline_probe(void *d_buf, size_t bytes, void *hip_stream, double *fp32_fma_tflops,
                      double *copy_gbs);

/* Measure the issue rate of v_mfma_f32_16x16x32_bf16 (independent chains, no
 * memory traffic) with one and with two waves per SIMD (one or two 256-thread
 * workgroups per CU), in TFLOP/s, on hip_stream.  d_buf: caller-owned device
 * scratch of `bytes` >= 2 KiB per CU (overwritten).  Blocks until done.
 * Errors: GT_E_INVAL (buffer), GT_E_STATE (no device), GT_E_HIP. */
int gt_mfma_probe(void *d_buf, size_t bytes, void *hip_stream, double *tflops_1wave, double *tflops_2wave);

#ifdef __cplusplus
}
#endif
#endif /* GREENTUNE_H */
