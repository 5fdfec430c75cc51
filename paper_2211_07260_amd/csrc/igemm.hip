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

#include <algorithm>
#include <atomic>

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
// (one row per wave) for 16*NT output channels.  Its input halo,
// (TH+R-1) x (64+S-1) pixels x C channels, sits in LDS (zero where the filter
// overhangs the image), so each input byte crosses L2 about once per strip
// instead of once per filter tap, and the weights sit in LDS too when they
// fit.
//
// A wave's 64 pixels form kMT = 4 M-tiles, interleaved: row i of M-tile m is
// pixel 4*i + m.  For filter tap s, M-tile m then needs pixels 4*i + m + s,
// which is the fragment F(m + s) with lane i holding pixel 4*i + t; so one
// filter row and 32-channel block reads kMT + S - 1 activation fragments from
// LDS instead of kMT * S.
//
// LDS layout.  Every 32-channel block is a plane of 64-byte pixel records,
// and chunk c (8 channels) of a record at position pos sits at 16-byte slot
// c ^ ((pos >> 2) & 3); 16 consecutive positions then cover all 64 banks once,
// and every fragment read below is 16 consecutive positions of one chunk.
// Halo rows store pixel hx at position (hx & 3) * HW4 + (hx >> 2), so F(t)
// is 16 consecutive positions.  Weights are stored [r][s][c-block][channel],
// so a B fragment (16 consecutive output channels) is 16 consecutive records.
constexpr int kLdsTW = 64;
constexpr int kRec = 64;  // bytes of one record: 32 BF16 channels

__device__ __forceinline__ int rec_slot(int c, int pos) { return c ^ ((pos >> 2) & 3); }

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
    static constexpr int HW4 = (kLdsTW + F - 1 + 3) / 4;
    static constexpr int halo(int th) { return (th + F - 1) * 4 * HW4 * C * 2; }
    static constexpr int wbytes = 16 * NT * F * F * C * 2;
    static constexpr int wrow = 16 * NT * F * C * 2;
    static constexpr int TH = (halo(8) + wbytes <= kLimit) ? 8 : 4;
    static constexpr int WM = halo(TH) + wbytes <= kLimit       ? kWeightsLds
                              : halo(TH) + 2 * wrow <= kLimit ? kWeightsLdsByRow
                                                              : kWeightsL2;
    static constexpr int bytes = halo(TH) + (WM == kWeightsLds ? wbytes : WM == kWeightsLdsByRow ? 2 * wrow : 0);
};

// Rows hy0 .. hy0+ROWS-1 of a tile's input halo: chunk k = (pixel p = k / CH,
// channel chunk q = k % CH).  LDS holds the halo as a ring of HH pixel rows:
// halo row hy of the tile whose first output row is y0 lives in ring slot
// (y0 + hy) % HH, so the next tile down the same strip finds its first R-1
// rows in place.
template <int C, int HW, int HH, int NTHR, int ROWS>
struct HaloRows {
    static constexpr int CH = C / 8, KC = C / 32, HW4 = (HW + 3) / 4;
    static constexpr int ROWB = 4 * HW4 * kRec, PLANE = HH * ROWB;
    static constexpr int NCHUNK = ROWS * HW * CH, ITERS = (NCHUNK + NTHR - 1) / NTHR;
    // every load of a thread is issued before any is used; chunks outside the
    // image read a valid address and are replaced by zeros
    __device__ static void load(const IgemmArgs &a, int b, int y0, int x0, int hy0, u32x4 (&v)[ITERS]) {
        const unsigned short *in = static_cast<const unsigned short *>(a.in);
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int p = k / CH, q = k - p * CH;
            const int hy = hy0 + p / HW, hx = p % HW;
            const int y = y0 - a.ph + hy, x = x0 - a.pw + hx;
            const bool inside = k < NCHUNK && y >= 0 && y < a.h && x >= 0 && x < a.wd;
            const size_t src = inside ? (((size_t)b * a.h + y) * a.wd + x) * C + q * 8 : 0;
            const u32x4 t = *reinterpret_cast<const u32x4 *>(in + src);
            v[it] = inside ? t : u32x4{0u, 0u, 0u, 0u};
        }
    }
    __device__ static void store(unsigned char *halo, int y0, int hy0, const u32x4 (&v)[ITERS]) {
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int p = k / CH, q = k - p * CH;
            const int slot = (y0 + hy0 + p / HW) % HH, hx = p % HW;
            const int pos = (hx & 3) * HW4 + (hx >> 2);
            if (k < NCHUNK)
                *reinterpret_cast<u32x4 *>(halo + (q >> 2) * PLANE + slot * ROWB + pos * kRec +
                                           16 * rec_slot(q & 3, pos)) = v[it];
        }
    }
};

// Persistent: the grid holds about as many workgroups as are resident at
// once, and workgroup g runs tiles_per_wg consecutive tiles, ordered down a
// 64-column strip of one image.  A tile's successor in the strip needs only
// TH new halo rows (the ring keeps the other R-1); they are loaded into
// registers while the tile computes and written to LDS once every wave is
// done with the rows they replace.
// TH output rows (= waves) per workgroup; WM: weight placement (WeightMode).
template <int C, int NT, int R, int S, int TH, int WM>
__global__ __launch_bounds__(TH * 64) void igemm_bf16_lds_kernel(IgemmArgs a, int tiles_per_wg) {
    constexpr bool WL = WM == kWeightsLds, WROW = WM == kWeightsLdsByRow;
    constexpr int CH = C / 8, KC = C / 32;
    constexpr int HW = kLdsTW + S - 1, HH = TH + R - 1;
    constexpr int NTHR = TH * 64;
    typedef HaloRows<C, HW, HH, NTHR, HH> Full;
    typedef HaloRows<C, HW, HH, NTHR, TH> Next;
    constexpr int HW4 = Full::HW4, ROWB = Full::ROWB, PLANE = Full::PLANE;
    constexpr int TAPB = 16 * NT * kRec;  // one (tap, c-block) of the workgroup's weights
    constexpr int WROW_BYTES = S * KC * TAPB;
    constexpr int WCHUNK = 16 * NT * R * S * CH;  // this workgroup's weight chunks
    constexpr int RCHUNK = 16 * NT * S * CH;      // ... of one filter row
    // weight loads from L2 would wait behind the prefetch (loads complete in
    // order), so that mode loads the next rows after the tile instead
    constexpr bool PREFETCH = WM != kWeightsL2;
    constexpr int BD = WM == kWeightsL2 ? 2 : 1;  // weight fragments are loaded BD steps ahead
    // weights first (offset 0), then the halo planes
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *wlds = lds;
    unsigned char *halo = lds + (WL ? R * S * KC * TAPB : WROW ? 2 * WROW_BYTES : 0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int tiles_x = (a.out_w + kLdsTW - 1) / kLdsTW, tiles_y = (a.out_h + TH - 1) / TH;
    const int n_tiles = a.n * tiles_x * tiles_y;
    // Workgroups are dispatched round-robin over the 8 XCDs; when the grid is
    // a multiple of 8, XCD x gets the x-th eighth of the workgroup indices, so
    // neighbouring runs of tiles share an L2.
    int g = blockIdx.x;
    if ((gridDim.x & 7) == 0) g = (g & 7) * (gridDim.x >> 3) + (g >> 3);
    const int t_begin = g * tiles_per_wg;
    const int t_end = min(n_tiles, t_begin + tiles_per_wg);
    if (t_begin >= t_end) return;  // uniform over the workgroup
    const int n_blk = blockIdx.y * (16 * NT);
    const unsigned short *wt = static_cast<const unsigned short *>(a.w);

    // tile t -> (image b, column strip, row block), row block fastest
    auto tile_origin = [&](int t, int &b, int &y0, int &x0) {
        const int tyi = t % tiles_y;
        t /= tiles_y;
        const int txi = t % tiles_x;
        b = t / tiles_x;
        y0 = tyi * TH;
        x0 = txi * kLdsTW;
    };
    // weight chunk q of (channel cl, tap) -> LDS offset within a [tap][c-block][channel] block
    auto wofs = [&](int tap, int cl, int q) {
        return ((tap * KC + (q >> 2)) * (16 * NT) + cl) * kRec + 16 * rec_slot(q & 3, cl);
    };
    // one filter row of weights (row-buffered mode): chunk k = (channel cl,
    // tap s, chunk q) of row r
    constexpr int RITERS = (RCHUNK + NTHR - 1) / NTHR;
    auto wrow_load = [&](int r, u32x4(&v)[RITERS]) {
#pragma unroll
        for (int it = 0; it < RITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (S * CH), rem = k - cl * (S * CH);
            const int sx = rem / CH, q = rem - sx * CH;
            v[it] = *reinterpret_cast<const u32x4 *>(
                wt + (k < RCHUNK ? (((size_t)(n_blk + cl) * R + r) * S + sx) * C + q * 8 : 0));
        }
    };
    auto wrow_store = [&](int buf, const u32x4(&v)[RITERS]) {
#pragma unroll
        for (int it = 0; it < RITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (S * CH), rem = k - cl * (S * CH);
            const int sx = rem / CH, q = rem - sx * CH;
            if (k < RCHUNK) *reinterpret_cast<u32x4 *>(wlds + buf * WROW_BYTES + wofs(sx, cl, q)) = v[it];
        }
    };

    {
        int b, y0, x0;
        tile_origin(t_begin, b, y0, x0);
        u32x4 v[Full::ITERS];
        Full::load(a, b, y0, x0, 0, v);
        Full::store(halo, y0, 0, v);
    }
    if constexpr (WL) {
        // all weights of output channels n_blk .. n_blk + 16*NT, staged once:
        // chunk k = (channel cl, tap rs, chunk q)
        constexpr int ITERS = (WCHUNK + NTHR - 1) / NTHR;
        u32x4 v[ITERS];
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (R * S * CH), rem = k - cl * (R * S * CH);
            const int rs = rem / CH, q = rem - rs * CH;
            v[it] = *reinterpret_cast<const u32x4 *>(
                wt + (k < WCHUNK ? (((size_t)(n_blk + cl) * R * S + rs) * C + q * 8) : 0));
        }
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (R * S * CH), rem = k - cl * (R * S * CH);
            const int rs = rem / CH, q = rem - rs * CH;
            if (k < WCHUNK) *reinterpret_cast<u32x4 *>(wlds + wofs(rs, cl, q)) = v[it];
        }
    }
    int wb = 0;  // row-buffered mode: the LDS buffer holding the current filter row
    if constexpr (WROW) {
        u32x4 v[RITERS];
        wrow_load(0, v);
        wrow_store(0, v);
    }
    __syncthreads();

    // this lane's byte offsets: F(t) within a halo row (t < kMT + S - 1), and
    // its B-fragment record within a (tap, c-block) weight block
    int aofs[kMT + S - 1];
#pragma unroll
    for (int t = 0; t < kMT + S - 1; ++t) {
        const int pos = (t & 3) * HW4 + (t >> 2) + li;
        aofs[t] = pos * kRec + 16 * rec_slot(lg, pos);
    }
    const int bofs = li * kRec + 16 * rec_slot(lg, li);

    for (int t = t_begin; t < t_end; ++t) {
        const bool more = t + 1 < t_end;                   // uniform over the workgroup
        const bool down = more && (t + 1) % tiles_y != 0;  // the next tile is the one below
        int b, y0, x0;
        tile_origin(t, b, y0, x0);
        // the next tile's TH new rows: its halo rows R-1 .. R+TH-2
        u32x4 nh[Next::ITERS];
        if constexpr (PREFETCH)
            if (down) Next::load(a, b, y0 + TH, x0, R - 1, nh);
        // opaque per tile, so weight loads from L2 are not hoisted out of the tile loop
        const unsigned short *wtt = wt;
        asm volatile("" : "+s"(wtt));

        f32x4 acc[kMT][NT];
#pragma unroll
        for (int m = 0; m < kMT; ++m)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};

        // One filter row: steps k = (c-block kc, tap s), s fastest.  Step k
        // uses F(s) .. F(s+kMT-1) of block kc and the weights of (r, s, kc);
        // the activation fragments a step newly needs are loaded one step
        // ahead, the weight fragments BD steps ahead.
        auto filter_row = [&](int r) {
            constexpr int NS = KC * S;
            const unsigned char *arow = halo + ((y0 + wave + r) % HH) * ROWB;
            u32x4 Af[KC][kMT + S - 1], Bq[NS][NT];
            auto ld_b = [&](int k) {
                const int kc = k / S, s = k - kc * S;
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    if constexpr (WL) {
                        Bq[k][j] = *reinterpret_cast<const u32x4 *>(wlds + ((r * S + s) * KC + kc) * TAPB + j * 16 * kRec + bofs);
                    } else if constexpr (WROW) {
                        Bq[k][j] = *reinterpret_cast<const u32x4 *>(wlds + wb * WROW_BYTES + (s * KC + kc) * TAPB + j * 16 * kRec + bofs);
                    } else {
                        Bq[k][j] = *reinterpret_cast<const u32x4 *>(
                            wtt + (((size_t)(n_blk + j * 16 + li) * R + r) * S + s) * C + kc * 32 + lg * 8);
                    }
                }
            };
            auto ld_f = [&](int kc, int f) {
                Af[kc][f] = *reinterpret_cast<const u32x4 *>(arow + kc * PLANE + aofs[f]);
            };
            auto ld_a = [&](int k) {  // the activation fragments step k needs first
                const int kc = k / S, s = k - kc * S;
                if (s == 0) {
#pragma unroll
                    for (int f = 0; f < kMT; ++f) ld_f(kc, f);
                } else {
                    ld_f(kc, s + kMT - 1);
                }
            };
#pragma unroll
            for (int k = 0; k < BD && k < NS; ++k) ld_b(k);
            ld_a(0);
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                if (k + BD < NS) ld_b(k + BD);
                if (k + 1 < NS) ld_a(k + 1);
                __builtin_amdgcn_sched_barrier(0);
                const int kc = k / S, s = k - kc * S;
#pragma unroll
                for (int m = 0; m < kMT; ++m)
#pragma unroll
                    for (int j = 0; j < NT; ++j)
                        acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, Af[kc][s + m]), __builtin_bit_cast(bf16x8, Bq[k][j]),
                            acc[m][j], 0, 0, 0);
            }
        };
        if constexpr (WROW) {
            // the next filter row's weights (row 0 of the next tile after the
            // last row) load from L2 while this row computes; the barrier
            // after the store keeps the two buffers' readers and writer apart
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool nxt = r + 1 < R || more;
                u32x4 v[RITERS];
                if (nxt) wrow_load(r + 1 < R ? r + 1 : 0, v);
                filter_row(r);
                if (nxt) wrow_store(wb ^ 1, v);
                if (r + 1 < R) __syncthreads();
                wb ^= 1;
            }
        } else if constexpr (R <= 7) {  // small filters: the whole walk unrolled (no loop-carried accumulator copies)
#pragma unroll
            for (int r = 0; r < R; ++r) filter_row(r);
        } else {
#pragma unroll 1
            for (int r = 0; r < R; ++r) filter_row(r);
        }

        // D[i = 4*lg + e][n = li] of M-tile m: output pixel x0 + 4*i + m
        const int y = y0 + wave;
        if (y < a.out_h) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int m = 0; m < kMT; ++m) {
                    const int x = x0 + 16 * lg + 4 * e + m;
                    if (x < a.out_w) {
                        float *dst = a.out + (((size_t)b * a.out_h + y) * a.out_w + x) * a.c_out + n_blk + li;
#pragma unroll
                        for (int j = 0; j < NT; ++j) dst[j * 16] = acc[m][j][e];
                    }
                }
        }
        if (more) {
            __syncthreads();  // every wave is done with this tile's halo rows
            if (down) {
                if constexpr (!PREFETCH) Next::load(a, b, y0 + TH, x0, R - 1, nh);
                Next::store(halo, y0 + TH, R - 1, nh);
            } else {  // a new strip: the whole halo
                int b1, y1, x1;
                tile_origin(t + 1, b1, y1, x1);
                u32x4 v[Full::ITERS];
                Full::load(a, b1, y1, x1, 0, v);
                Full::store(halo, y1, 0, v);
            }
            __syncthreads();
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
constexpr size_t kLdsTableSize = sizeof(kLdsTable) / sizeof(kLdsTable[0]);
std::atomic<int> g_lds_occupancy[kLdsTableSize];  // resident workgroups per CU, 0 = not yet queried

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
            const int gy = p.c_out / (16 * e->nt);
            const size_t idx = (size_t)(e - kLdsTable);
            int occ = g_lds_occupancy[idx].load(std::memory_order_relaxed);
            if (occ == 0) {
                if (e->lds > 65536)
                    GT_HIP_CHECK(hipFuncSetAttribute(e->fn, hipFuncAttributeMaxDynamicSharedMemorySize, e->lds));
                GT_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, e->fn, 64 * e->th, (size_t)e->lds));
                occ = std::max(1, occ);
                g_lds_occupancy[idx].store(occ, std::memory_order_relaxed);
            }
            // persistent grid: about one resident wave of workgroups, each
            // taking an equal run of tiles; rounded up to a multiple of 8 for
            // the XCD-aware order (surplus workgroups find no tiles and exit)
            const int64_t resident = std::max<int64_t>(1, (int64_t)std::max(1, state().dev.cu_count) * occ / gy);
            const int64_t m = std::min(tiles, resident);
            const int64_t per = (tiles + m - 1) / m;
            int64_t gx = (tiles + per - 1) / per;
            if (gx >= 8) gx = (gx + 7) / 8 * 8;
            if (per > INT32_MAX || gx * per >= ((int64_t)1 << 31))
                return set_error(GT_E_INVAL, "igemm: too many tiles");
            int tiles_per_wg = (int)per;
            void *largs[] = {&a, &tiles_per_wg};
            dim3 grid((unsigned)gx, (unsigned)gy);
            GT_HIP_CHECK(hipLaunchKernel(e->fn, grid, dim3(64 * e->th), largs, (size_t)e->lds, s));
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
