// Multi-channel convolution as an implicit GEMM (no im2col buffer).
//
//   out[b][y][x][k] = sum_{r,s,c} in[b][y+r-ph][x+s-pw][c] * wt[k][r][s][c]
//
// with NHWC activations, KRSC weights and an NHWC FP32 output.  Seen as a
// GEMM, M = batch*out_h*out_w output pixels, N = c_out, and the reduction runs
// over (r, s, c).  Two kernels:
//
// * BF16 on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate).  A fragment
//   lane l holds A[m = l%16][k = 8*(l/16) .. +8]: with NHWC input that is 16
//   contiguous bytes of one pixel's channels, and the KRSC weight fragment
//   B[k = 8*(l/16) .. +8][n = l%16] is likewise 16 contiguous bytes, so both
//   operands are loaded straight from memory with one 16-byte load per lane
//   and no transposition.  A wave owns 4 M-tiles (64 pixels) x NT N-tiles
//   (16*NT output channels); the fragments of the next (r, s, c-block) step
//   are loaded while the current step's MFMAs issue.  Zero padding is a
//   masked load (the address is clamped in bounds, the value replaced by 0).
//
// * FP32 on the vector ALUs, the comparison path.  Lanes are output channels
//   (64 per wave) and a wave owns P pixels, so an input value is the same for
//   the whole wave: it is read with scalar loads into SGPRs and each FMA is
//   v_fmac acc, s_x, v_w with the weights in VGPRs (read through L1/L2).
#include <hip/hip_runtime.h>

#include "gt_internal.hpp"

namespace gt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct IgemmArgs {
    const void *in;
    const void *w;
    float *out;
    int32_t n, h, wd, c_in, c_out, out_h, out_w, ph, pw;
    int32_t m_total;  // n * out_h * out_w
};

constexpr int kMfmaWaves = 4, kMT = 4;  // waves per workgroup, 16-pixel M-tiles per wave

template <int R, int S, int C, int NT>
__global__ __launch_bounds__(256) void igemm_bf16_mfma_kernel(IgemmArgs a) {
    constexpr int KC = C / 32;         // 32-channel reduction blocks per (r, s)
    constexpr int STEPS = R * S * KC;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m_wave = (blockIdx.x * kMfmaWaves + wave) * (16 * kMT);
    const int n_blk = blockIdx.y * (16 * NT);
    const unsigned short *in = static_cast<const unsigned short *>(a.in);
    const unsigned short *wt = static_cast<const unsigned short *>(a.w);

    // this lane's A pixels (row li of each M-tile)
    int pb[kMT], py[kMT], px[kMT];
    bool pv[kMT];
#pragma unroll
    for (int t = 0; t < kMT; ++t) {
        int m = m_wave + t * 16 + li;
        pv[t] = m < a.m_total;
        m = pv[t] ? m : 0;
        px[t] = m % a.out_w;
        const int q = m / a.out_w;
        py[t] = q % a.out_h;
        pb[t] = q / a.out_h;
    }

    auto load_step = [&](int step, u32x4 (&A)[kMT], u32x4 (&B)[NT]) {
        const int kc = step % KC, rs = step / KC;
        const int s = rs % S, r = rs / S;
        const int c0 = kc * 32 + lg * 8;
#pragma unroll
        for (int t = 0; t < kMT; ++t) {
            const int yy = py[t] + r - a.ph, xx = px[t] + s - a.pw;
            const bool ok = pv[t] && yy >= 0 && yy < a.h && xx >= 0 && xx < a.wd;
            const size_t off = ok ? (((size_t)pb[t] * a.h + yy) * a.wd + xx) * C + c0 : 0;
            const u32x4 v = *reinterpret_cast<const u32x4 *>(in + off);
            A[t] = ok ? v : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = n_blk + j * 16 + li;
            B[j] = *reinterpret_cast<const u32x4 *>(wt + (((size_t)co * R + r) * S + s) * C + c0);
        }
    };

    f32x4 acc[kMT][NT];
#pragma unroll
    for (int t = 0; t < kMT; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    u32x4 A0[kMT], B0[NT], A1[kMT], B1[NT];
    load_step(0, A0, B0);
#pragma unroll
    for (int step = 0; step < STEPS; step += 2) {
        if (step + 1 < STEPS) load_step(step + 1, A1, B1);
#pragma unroll
        for (int t = 0; t < kMT; ++t)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, A0[t]), __builtin_bit_cast(bf16x8, B0[j]), acc[t][j], 0, 0, 0);
        if (step + 1 < STEPS) {
            if (step + 2 < STEPS) load_step(step + 2, A0, B0);
#pragma unroll
            for (int t = 0; t < kMT; ++t)
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, A1[t]), __builtin_bit_cast(bf16x8, B1[j]), acc[t][j], 0, 0,
                        0);
        }
    }

    // D[m = 4*lg + e][n = li]: for fixed e, 16 lanes store 16 consecutive channels
#pragma unroll
    for (int t = 0; t < kMT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m_wave + t * 16 + lg * 4 + e;
            if (m < a.m_total) {
                float *dst = a.out + (size_t)m * a.c_out + n_blk + li;
#pragma unroll
                for (int j = 0; j < NT; ++j) dst[j * 16] = acc[t][j][e];
            }
        }
}

// Same tile and fragment layout with the filter size a runtime value: the
// (r, s, c-block) walk is a loop with scalar counters instead of a fully
// unrolled sequence, for filter sizes without a dedicated instance.
template <int C, int NT>
__global__ __launch_bounds__(256) void igemm_bf16_mfma_any_kernel(IgemmArgs a, int R, int S) {
    constexpr int KC = C / 32;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int m_wave = (blockIdx.x * kMfmaWaves + wave) * (16 * kMT);
    const int n_blk = blockIdx.y * (16 * NT);
    const unsigned short *in = static_cast<const unsigned short *>(a.in);
    const unsigned short *wt = static_cast<const unsigned short *>(a.w);

    int pb[kMT], py[kMT], px[kMT];
    bool pv[kMT];
#pragma unroll
    for (int t = 0; t < kMT; ++t) {
        int m = m_wave + t * 16 + li;
        pv[t] = m < a.m_total;
        m = pv[t] ? m : 0;
        px[t] = m % a.out_w;
        const int q = m / a.out_w;
        py[t] = q % a.out_h;
        pb[t] = q / a.out_h;
    }
    auto load = [&](int r, int s, int kc, u32x4 (&A)[kMT], u32x4 (&B)[NT]) {
        const int c0 = kc * 32 + lg * 8;
#pragma unroll
        for (int t = 0; t < kMT; ++t) {
            const int yy = py[t] + r - a.ph, xx = px[t] + s - a.pw;
            const bool ok = pv[t] && yy >= 0 && yy < a.h && xx >= 0 && xx < a.wd;
            const size_t off = ok ? (((size_t)pb[t] * a.h + yy) * a.wd + xx) * C + c0 : 0;
            const u32x4 v = *reinterpret_cast<const u32x4 *>(in + off);
            A[t] = ok ? v : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = n_blk + j * 16 + li;
            B[j] = *reinterpret_cast<const u32x4 *>(wt + (((size_t)co * R + r) * S + s) * C + c0);
        }
    };
    auto next = [&](int &r, int &s, int &kc) {
        if (++kc == KC) {
            kc = 0;
            if (++s == S) {
                s = 0;
                ++r;
            }
        }
    };
    f32x4 acc[kMT][NT];
#pragma unroll
    for (int t = 0; t < kMT; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int steps = R * S * KC;
    int r = 0, s = 0, kc = 0;
    u32x4 A0[kMT], B0[NT], A1[kMT], B1[NT];
    load(r, s, kc, A0, B0);
    next(r, s, kc);
    for (int step = 0; step < steps; step += 2) {
        const bool more = step + 1 < steps;
        if (more) {
            load(r, s, kc, A1, B1);
            next(r, s, kc);
        }
#pragma unroll
        for (int t = 0; t < kMT; ++t)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, A0[t]), __builtin_bit_cast(bf16x8, B0[j]), acc[t][j], 0, 0, 0);
        if (more) {
            if (step + 2 < steps) {
                load(r, s, kc, A0, B0);
                next(r, s, kc);
            }
#pragma unroll
            for (int t = 0; t < kMT; ++t)
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, A1[t]), __builtin_bit_cast(bf16x8, B1[j]), acc[t][j], 0, 0,
                        0);
        }
    }
#pragma unroll
    for (int t = 0; t < kMT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m_wave + t * 16 + lg * 4 + e;
            if (m < a.m_total) {
                float *dst = a.out + (size_t)m * a.c_out + n_blk + li;
#pragma unroll
                for (int j = 0; j < NT; ++j) dst[j * 16] = acc[t][j][e];
            }
        }
}

// LDS-staged variant.  A workgroup owns a TH-row x 64-column output tile
// (one row per wave, four 16-pixel M-tiles per wave) for 16*NT output
// channels.  Its input halo, (TH+R-1) x (64+S-1) pixels x C channels, is
// staged in LDS once (zero where the filter overhangs the image), so each
// input byte crosses L2 once per workgroup instead of once per filter tap.
// LDS holds pixel-major 16-byte channel chunks; chunk q of halo column hx is
// stored at slot q ^ swz(hx), which spreads the 16 lanes of an A-fragment read
// (16 consecutive pixels, same chunk) over distinct banks.  Weights (B) are
// staged in LDS too when they fit (same swizzle over output channels), else
// read from L2 as 16-byte fragments; the (s, c-block) walk of one filter row
// is unrolled with fragments loaded ahead of their MFMAs.
constexpr int kLdsTW = 64;

template <int C>
__device__ __forceinline__ int lds_swz(int hx) {
    if constexpr (C == 64)
        return (hx >> 1) & 7;
    else
        return (hx >> 2) & 3;
}

// Where the workgroup's weights live.
enum WeightMode { kWeightsL2 = 0, kWeightsLds = 1, kWeightsLdsByRow = 2 };

// Workgroup shape and LDS use of the staged kernel for (C, NT, F), within
// 160 KiB: eight output rows with all weights in LDS if that fits; else four
// rows with all weights, or with one filter row of weights double-buffered
// (the next row's weights load while the current row computes); else four
// rows with the weights read from L2.
template <int C, int NT, int F>
struct LdsPlan {
    static constexpr int kLimit = 163840;
    static constexpr int halo(int th) { return (th + F - 1) * (kLdsTW + F - 1) * C * 2; }
    static constexpr int wbytes = 16 * NT * F * F * C * 2;
    static constexpr int wrow = 16 * NT * F * C * 2;
    static constexpr int TH = (halo(8) + wbytes <= kLimit) ? 8 : 4;
    static constexpr int WM = halo(TH) + wbytes <= kLimit       ? kWeightsLds
                              : halo(TH) + 2 * wrow <= kLimit ? kWeightsLdsByRow
                                                              : kWeightsL2;
    static constexpr int bytes = halo(TH) + (WM == kWeightsLds ? wbytes : WM == kWeightsLdsByRow ? 2 * wrow : 0);
};

// TH output rows (= waves) per workgroup; WM: weight placement (WeightMode).
template <int C, int NT, int R, int S, int TH, int WM>
__global__ __launch_bounds__(TH * 64) void igemm_bf16_lds_kernel(IgemmArgs a) {
    constexpr bool WL = WM == kWeightsLds, WROW = WM == kWeightsLdsByRow;
    constexpr int CH = C / 8, KC = C / 32;
    constexpr int HW = kLdsTW + S - 1, HH = TH + R - 1;
    constexpr int NCHUNK = HH * HW * CH;
    constexpr int NTHR = TH * 64;
    constexpr int HALO_BYTES = HH * HW * C * 2;
    constexpr int WCHUNK = 16 * NT * R * S * CH;     // this workgroup's weight chunks
    constexpr int RCHUNK = 16 * NT * S * CH;         // ... of one filter row
    constexpr int WROW_BYTES = 16 * NT * S * C * 2;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *wlds = lds + HALO_BYTES;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int tiles_x = (a.out_w + kLdsTW - 1) / kLdsTW, tiles_y = (a.out_h + TH - 1) / TH;
    int t = blockIdx.x;
    const int txi = t % tiles_x;
    t /= tiles_x;
    const int tyi = t % tiles_y, b = t / tiles_y;
    const int x0 = txi * kLdsTW, y0 = tyi * TH;
    const int n_blk = blockIdx.y * (16 * NT);
    const unsigned short *in = static_cast<const unsigned short *>(a.in);
    const unsigned short *wt = static_cast<const unsigned short *>(a.w);

    // Stage the halo: chunk k = (pixel p = k / CH, channel chunk q = k % CH).
    // All of a thread's chunk loads are issued before any LDS store, so the
    // staging costs about one memory latency; chunks outside the image read a
    // valid address and are replaced by zeros.
    {
        constexpr int ITERS = (NCHUNK + NTHR - 1) / NTHR;
        u32x4 v[ITERS];
        int off[ITERS];
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int p = k / CH, q = k - p * CH;
            const int hy = p / HW, hx = p - hy * HW;
            const int y = y0 - a.ph + hy, x = x0 - a.pw + hx;
            const bool inside = k < NCHUNK && y >= 0 && y < a.h && x >= 0 && x < a.wd;
            const size_t src = inside ? (((size_t)b * a.h + y) * a.wd + x) * C + q * 8 : 0;
            const u32x4 t = *reinterpret_cast<const u32x4 *>(in + src);
            v[it] = inside ? t : u32x4{0u, 0u, 0u, 0u};
            off[it] = k < NCHUNK ? p * (C * 2) + 16 * (q ^ lds_swz<C>(hx)) : -1;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int it = 0; it < ITERS; ++it)
            if (off[it] >= 0) *reinterpret_cast<u32x4 *>(lds + off[it]) = v[it];
    }
    if constexpr (WL) {
        // weights of output channels n_blk .. n_blk + 16*NT: chunk k = (channel
        // cl, tap rs, chunk q); chunk q of channel cl at slot q ^ swz(cl), so a
        // B-fragment read (16 consecutive channels, same chunk) is bank-free
        constexpr int ITERS = (WCHUNK + NTHR - 1) / NTHR;
        u32x4 v[ITERS];
        int off[ITERS];
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (R * S * CH), rem = k - cl * (R * S * CH);
            const int rs = rem / CH, q = rem - rs * CH;
            const bool ok = k < WCHUNK;
            v[it] = *reinterpret_cast<const u32x4 *>(
                wt + (ok ? (((size_t)(n_blk + cl) * R * S + rs) * C + q * 8) : 0));
            off[it] = ok ? (cl * R * S + rs) * (C * 2) + 16 * (q ^ lds_swz<C>(cl)) : -1;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int it = 0; it < ITERS; ++it)
            if (off[it] >= 0) *reinterpret_cast<u32x4 *>(wlds + off[it]) = v[it];
    }
    // one filter row of weights (row-buffered mode): chunk k = (channel cl,
    // tap s, chunk q) of row r, stored at (cl*S + s) with the same swizzle
    constexpr int RITERS = (RCHUNK + NTHR - 1) / NTHR;
    auto wrow_load = [&](int r, u32x4 (&v)[RITERS]) {
#pragma unroll
        for (int it = 0; it < RITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (S * CH), rem = k - cl * (S * CH);
            const int sx = rem / CH, q = rem - sx * CH;
            v[it] = *reinterpret_cast<const u32x4 *>(
                wt + (k < RCHUNK ? (((size_t)(n_blk + cl) * R + r) * S + sx) * C + q * 8 : 0));
        }
    };
    auto wrow_store = [&](int buf, const u32x4 (&v)[RITERS]) {
#pragma unroll
        for (int it = 0; it < RITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (S * CH), rem = k - cl * (S * CH);
            const int sx = rem / CH, q = rem - sx * CH;
            if (k < RCHUNK)
                *reinterpret_cast<u32x4 *>(wlds + buf * WROW_BYTES + (cl * S + sx) * (C * 2) +
                                           16 * (q ^ lds_swz<C>(cl))) = v[it];
        }
    };
    if constexpr (WROW) {
        u32x4 v[RITERS];
        wrow_load(0, v);
        wrow_store(0, v);
    }
    __syncthreads();

    f32x4 acc[kMT][NT];
#pragma unroll
    for (int m = 0; m < kMT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // One filter row: its S * KC steps are unrolled with weight fragments
    // loaded two steps ahead (they come from L2) and activation fragments one
    // step ahead (from LDS).
    auto filter_row = [&](int r) {
        constexpr int NS = S * KC;
        const unsigned char *row = lds + (wave + r) * HW * (C * 2);
        u32x4 Bq[NS][NT], Aq[NS][kMT];
        auto ld_b = [&](int k) {
            const int s = k / KC, kc = k - s * KC;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int cl = j * 16 + li;
                if constexpr (WL) {
                    const int q = kc * 4 + lg;
                    Bq[k][j] = *reinterpret_cast<const u32x4 *>(wlds + (cl * R * S + r * S + s) * (C * 2) +
                                                                16 * (q ^ lds_swz<C>(cl)));
                } else if constexpr (WROW) {
                    const int q = kc * 4 + lg;
                    Bq[k][j] = *reinterpret_cast<const u32x4 *>(wlds + (r & 1) * WROW_BYTES + (cl * S + s) * (C * 2) +
                                                                16 * (q ^ lds_swz<C>(cl)));
                } else {
                    Bq[k][j] = *reinterpret_cast<const u32x4 *>(
                        wt + (((size_t)(n_blk + cl) * R + r) * S + s) * C + kc * 32 + lg * 8);
                }
            }
        };
        auto ld_a = [&](int k) {
            const int s = k / KC, kc = k - s * KC;
            const int q = kc * 4 + lg;
#pragma unroll
            for (int m = 0; m < kMT; ++m) {
                const int hx = m * 16 + li + s;
                Aq[k][m] = *reinterpret_cast<const u32x4 *>(row + hx * (C * 2) + 16 * (q ^ lds_swz<C>(hx)));
            }
        };
        ld_b(0);
        if (NS > 1) ld_b(1);
        ld_a(0);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (k + 2 < NS) ld_b(k + 2);
            if (k + 1 < NS) ld_a(k + 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < kMT; ++m)
#pragma unroll
                for (int j = 0; j < NT; ++j)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, Aq[k][m]), __builtin_bit_cast(bf16x8, Bq[k][j]), acc[m][j], 0,
                        0, 0);
        }
    };
    if constexpr (WROW) {
        // next row's weights load from L2 while this row computes; the barrier
        // after the store keeps the two buffers' readers and writer apart
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u32x4 v[RITERS];
            if (r + 1 < R) wrow_load(r + 1, v);
            filter_row(r);
            if (r + 1 < R) wrow_store((r + 1) & 1, v);
            __syncthreads();
        }
    } else if constexpr (R <= 7) {  // small filters: the whole walk unrolled (no loop-carried accumulator copies)
#pragma unroll
        for (int r = 0; r < R; ++r) filter_row(r);
    } else {
#pragma unroll 1
        for (int r = 0; r < R; ++r) filter_row(r);
    }

    // D[m = 4*lg + e][n = li] of M-tile m: pixel (y0 + wave, x0 + 16*m + 4*lg + e)
    const int y = y0 + wave;
    if (y < a.out_h) {
#pragma unroll
        for (int m = 0; m < kMT; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = x0 + m * 16 + lg * 4 + e;
                if (x < a.out_w) {
                    float *dst = a.out + (((size_t)b * a.out_h + y) * a.out_w + x) * a.c_out + n_blk + li;
#pragma unroll
                    for (int j = 0; j < NT; ++j) dst[j * 16] = acc[m][j][e];
                }
            }
    }
}

constexpr int kValuP = 8, kValuWaves = 4;  // pixels per wave, waves per workgroup

// A wave computes kValuP consecutive output pixels of one output row (all
// 64 output channels of its channel block, one per lane).  The input row
// pointer and the row check are wave-uniform; in interior tiles every pixel
// of a filter tap is valid and its 8-channel input chunk is one scalar load
// at a compile-time offset from the row pointer.
template <int R, int S, int C>
__global__ __launch_bounds__(256) void igemm_f32_valu_kernel(IgemmArgs a) {
    typedef const __attribute__((address_space(4))) float cfloat;
    const float *__restrict__ wt = static_cast<const float *>(a.w);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tiles_x = (a.out_w + kValuP - 1) / kValuP;
    const int tile = blockIdx.x * kValuWaves + wave;
    const int row = tile / tiles_x;                      // b * out_h + y
    const int x0 = (tile - row * tiles_x) * kValuP;
    const int co = blockIdx.y * 64 + lane;
    if (row >= a.n * a.out_h) return;  // wave-uniform: past the last row
    const int b = row / a.out_h, y = row - b * a.out_h;

    float acc[kValuP];
#pragma unroll
    for (int p = 0; p < kValuP; ++p) acc[p] = 0.f;

    for (int r = 0; r < R; ++r) {
        const int yy = y + r - a.ph;
        if (yy < 0 || yy >= a.h) continue;  // zero padding rows
        cfloat *rowp = (cfloat *)a.in + ((size_t)b * a.h + yy) * a.wd * C;
#pragma unroll 1
        for (int s = 0; s < S; ++s) {
            const int xs = x0 + s - a.pw;  // input column of pixel 0
            const float *wrs = wt + (((size_t)co * R + r) * S + s) * C;
            const bool all = xs >= 0 && xs + kValuP <= a.wd;
#pragma unroll 1
            for (int c = 0; c < C; c += 8) {  // one 8-channel chunk: 8 pixels x 8 inputs in SGPRs
                float wv[8];
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const float4 v = *reinterpret_cast<const float4 *>(wrs + c + 4 * k);
                    wv[4 * k] = v.x;
                    wv[4 * k + 1] = v.y;
                    wv[4 * k + 2] = v.z;
                    wv[4 * k + 3] = v.w;
                }
                if (all) {
                    cfloat *px = rowp + (size_t)xs * C + c;
#pragma unroll
                    for (int p = 0; p < kValuP; ++p)
#pragma unroll
                        for (int k = 0; k < 8; ++k) acc[p] = __builtin_fmaf(px[p * C + k], wv[k], acc[p]);
                } else {
#pragma unroll
                    for (int p = 0; p < kValuP; ++p) {
                        const int xx = xs + p;
                        if (xx >= 0 && xx < a.wd) {
                            cfloat *px = rowp + (size_t)xx * C + c;
#pragma unroll
                            for (int k = 0; k < 8; ++k) acc[p] = __builtin_fmaf(px[k], wv[k], acc[p]);
                        }
                    }
                }
            }
        }
    }
    float *dst = a.out + (size_t)row * a.out_w * a.c_out + co;
#pragma unroll
    for (int p = 0; p < kValuP; ++p)
        if (x0 + p < a.out_w) dst[(size_t)(x0 + p) * a.c_out] = acc[p];
}

namespace {

template <int R, int S>
const void *pick_mfma(int c, int nt) {
    if (c == 64 && nt == 4) return (const void *)&igemm_bf16_mfma_kernel<R, S, 64, 4>;
    if (c == 64 && nt == 2) return (const void *)&igemm_bf16_mfma_kernel<R, S, 64, 2>;
    if (c == 32 && nt == 4) return (const void *)&igemm_bf16_mfma_kernel<R, S, 32, 4>;
    if (c == 32 && nt == 2) return (const void *)&igemm_bf16_mfma_kernel<R, S, 32, 2>;
    return nullptr;
}

const void *mfma_any_for(int c, int nt) {
    if (c == 64 && nt == 4) return (const void *)&igemm_bf16_mfma_any_kernel<64, 4>;
    if (c == 64 && nt == 2) return (const void *)&igemm_bf16_mfma_any_kernel<64, 2>;
    if (c == 32 && nt == 4) return (const void *)&igemm_bf16_mfma_any_kernel<32, 4>;
    if (c == 32 && nt == 2) return (const void *)&igemm_bf16_mfma_any_kernel<32, 2>;
    return nullptr;
}

// Dedicated fully unrolled instances for filter sizes 1, 3, 5, 7; the
// runtime-size kernel for the others.  *generic tells which one was chosen.
const void *mfma_kernel_for(int f, int c, int c_out, bool *generic = nullptr) {
    const int nt = (c_out % 64 == 0) ? 4 : 2;
    const void *fn = nullptr;
    switch (f) {
        case 1: fn = pick_mfma<1, 1>(c, nt); break;
        case 3: fn = pick_mfma<3, 3>(c, nt); break;
        case 5: fn = pick_mfma<5, 5>(c, nt); break;
        case 7: fn = pick_mfma<7, 7>(c, nt); break;
        default: break;
    }
    if (generic) *generic = fn == nullptr;
    return fn ? fn : mfma_any_for(c, nt);
}

template <int R, int S>
const void *pick_valu(int c) {
    if (c == 64) return (const void *)&igemm_f32_valu_kernel<R, S, 64>;
    if (c == 32) return (const void *)&igemm_f32_valu_kernel<R, S, 32>;
    return nullptr;
}

const void *valu_kernel_for(int f, int c) {
    switch (f) {
        case 1: return pick_valu<1, 1>(c);
        case 3: return pick_valu<3, 3>(c);
        case 5: return pick_valu<5, 5>(c);
        case 7: return pick_valu<7, 7>(c);
        default: return nullptr;
    }
}

struct LdsEntry {
    int c, nt, f;
    const void *fn;
    int lds, th;
};
#define GT_L(C, NT, F)                                                                                     \
    {C, NT, F, (const void *)&igemm_bf16_lds_kernel<C, NT, F, F, LdsPlan<C, NT, F>::TH, LdsPlan<C, NT, F>::WM>, \
     LdsPlan<C, NT, F>::bytes, LdsPlan<C, NT, F>::TH}
const LdsEntry kLdsTable[] = {
    GT_L(64, 4, 1), GT_L(64, 4, 3), GT_L(64, 4, 5), GT_L(64, 4, 7), GT_L(64, 4, 9),
    GT_L(64, 2, 1), GT_L(64, 2, 3), GT_L(64, 2, 5), GT_L(64, 2, 7), GT_L(64, 2, 9),
    GT_L(32, 4, 1), GT_L(32, 4, 3), GT_L(32, 4, 5), GT_L(32, 4, 7), GT_L(32, 4, 9), GT_L(32, 4, 17),
    GT_L(32, 2, 1), GT_L(32, 2, 3), GT_L(32, 2, 5), GT_L(32, 2, 7), GT_L(32, 2, 9), GT_L(32, 2, 17),
};
#undef GT_L

// The LDS-staged kernel for (c_in, c_out, f) when instantiated and its halo
// fits the device's LDS; null otherwise.
const LdsEntry *lds_kernel_for(int f, int c, int c_out) {
    const int nt = (c_out % 64 == 0) ? 4 : 2;
    for (const LdsEntry &e : kLdsTable)
        if (e.c == c && e.nt == nt && e.f == f && e.lds <= state().dev.lds_per_block) return &e;
    return nullptr;
}

}  // namespace

int validate_igemm(const gt_problem &p, const gt_conv_config &) {
    if (p.n < 1 || p.c_in < 1 || p.c_out < 1 || p.out_h < 1 || p.out_w < 1 || p.filt_h < 1 || p.filt_w < 1 ||
        p.pad_h < 0 || p.pad_w < 0)
        return set_error(GT_E_INVAL, "igemm: sizes must be positive and padding non-negative");
    const int64_t h = (int64_t)p.out_h + p.filt_h - 1 - 2 * p.pad_h;
    const int64_t w = (int64_t)p.out_w + p.filt_w - 1 - 2 * p.pad_w;
    if (h < 1 || w < 1) return set_error(GT_E_INVAL, "igemm: padding larger than the input allows");
    if ((int64_t)p.n * h * w * p.c_in >= (int64_t)1 << 31 || (int64_t)p.n * p.out_h * p.out_w >= (int64_t)1 << 31)
        return set_error(GT_E_INVAL, "igemm: problem too large for 32-bit pixel indexing");
    if (p.filt_h != p.filt_w) return set_error(GT_E_UNSUPPORTED, "igemm: square filters only");
    if (p.kind == GT_IGEMM_BF16_MFMA) {
        if (p.c_out % 32 != 0) return set_error(GT_E_UNSUPPORTED, "igemm bf16: c_out must be a multiple of 32");
        if (!mfma_kernel_for(p.filt_h, p.c_in, p.c_out))
            return set_error(GT_E_UNSUPPORTED, "igemm bf16: c_in %d not instantiated (32 or 64)", p.c_in);
    } else {
        if (p.c_out % 64 != 0) return set_error(GT_E_UNSUPPORTED, "igemm f32: c_out must be a multiple of 64");
        if (!valu_kernel_for(p.filt_h, p.c_in))
            return set_error(GT_E_UNSUPPORTED, "igemm f32: c_in %d / filter %d not instantiated (c_in 32 or 64; "
                             "filter 1, 3, 5, 7)", p.c_in, p.filt_h);
    }
    return GT_OK;
}

int launch_igemm(const gt_problem &p, const gt_conv_config &, const void *in, const void *w, void *out,
                 hipStream_t s) {
    if ((((uintptr_t)in) | ((uintptr_t)w)) & 15)
        return set_error(GT_E_INVAL, "igemm: input and weights must be 16-byte aligned");
    IgemmArgs a;
    a.in = in;
    a.w = w;
    a.out = static_cast<float *>(out);
    a.n = p.n;
    a.h = p.out_h + p.filt_h - 1 - 2 * p.pad_h;
    a.wd = p.out_w + p.filt_w - 1 - 2 * p.pad_w;
    a.c_in = p.c_in;
    a.c_out = p.c_out;
    a.out_h = p.out_h;
    a.out_w = p.out_w;
    a.ph = p.pad_h;
    a.pw = p.pad_w;
    a.m_total = p.n * p.out_h * p.out_w;
    void *args[] = {&a};
    if (p.kind == GT_IGEMM_BF16_MFMA && p.filt_h == p.filt_w) {
        if (const LdsEntry *e = lds_kernel_for(p.filt_h, p.c_in, p.c_out)) {
            const int64_t tiles = (int64_t)p.n * ((p.out_h + e->th - 1) / e->th) * ((p.out_w + kLdsTW - 1) / kLdsTW);
            if (e->lds > 65536)
                GT_HIP_CHECK(hipFuncSetAttribute(e->fn, hipFuncAttributeMaxDynamicSharedMemorySize, e->lds));
            dim3 grid((unsigned)tiles, (unsigned)(p.c_out / (16 * e->nt)));
            GT_HIP_CHECK(hipLaunchKernel(e->fn, grid, dim3(64 * e->th), args, (size_t)e->lds, s));
            return GT_OK;
        }
    }
    if (p.kind == GT_IGEMM_BF16_MFMA) {
        const int nt = (p.c_out % 64 == 0) ? 4 : 2;
        const int per_wg = kMfmaWaves * kMT * 16;
        dim3 grid((unsigned)((a.m_total + per_wg - 1) / per_wg), (unsigned)(p.c_out / (16 * nt)));
        bool generic = false;
        const void *fn = mfma_kernel_for(p.filt_h, p.c_in, p.c_out, &generic);
        if (generic) {
            int R = p.filt_h, S = p.filt_w;
            void *gargs[] = {&a, &R, &S};
            GT_HIP_CHECK(hipLaunchKernel(fn, grid, dim3(256), gargs, 0, s));
        } else {
            GT_HIP_CHECK(hipLaunchKernel(fn, grid, dim3(256), args, 0, s));
        }
    } else {
        const int64_t tiles = (int64_t)p.n * p.out_h * ((p.out_w + kValuP - 1) / kValuP);
        dim3 grid((unsigned)((tiles + kValuWaves - 1) / kValuWaves), (unsigned)(p.c_out / 64));
        GT_HIP_CHECK(hipLaunchKernel(valu_kernel_for(p.filt_h, p.c_in), grid, dim3(256), args, 0, s));
    }
    return GT_OK;
}

}  // namespace gt
