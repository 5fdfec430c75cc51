// Multi-channel convolution as an implicit GEMM (no im2col buffer).
//
//   out[b][y][x][k] = sum_{r,s,c} in[b][y+r-ph][x+s-pw][c] * wt[k][r][s][c]
//
// with NHWC activations, KRSC weights and an NHWC FP32 output.  Seen as a
// GEMM, M = batch*out_h*out_w output pixels, N = c_out, and the reduction runs
// over (r, s, c).  The kernels:
//
// * BF16 on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate).  A fragment
//   lane l holds A[m = l%16][k = 8*(l/16) .. +8]: with NHWC input that is 16
//   contiguous bytes of one pixel's channels, and the KRSC weight fragment
//   B[k = 8*(l/16) .. +8][n = l%16] is likewise 16 contiguous bytes, so both
//   operands are loaded with one 16-byte load per lane and no transposition.
//   The main kernel (igemm_bf16_lds_kernel, below) stages the input halo and
//   the weights in LDS and runs persistent workgroups; a global-load kernel
//   (a wave owns 4 M-tiles (64 pixels) x NT N-tiles, the next step's
//   fragments loaded while the current step's MFMAs issue, zero padding as a
//   masked load) serves the shapes the LDS kernel does not cover.
//
// * FP32 on the vector ALUs, the comparison path: a register-tiled implicit
//   GEMM (each thread 4 pixels x 4 output channels) over LDS-staged,
//   channel-major slices of the input and the weights.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <vector>

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

// One wave's 64 output pixels m_wave .. m_wave+63 (pixels past a.m_total
// are skipped) x 16*NT output channels from n_blk.
template <int R, int S, int C, int NT>
__device__ __forceinline__ void mfma_global_tile(const IgemmArgs &a, int m_wave, int n_blk) {
    constexpr int KC = C / 32;         // 32-channel reduction blocks per (r, s)
    constexpr int STEPS = R * S * KC;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
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
__device__ __forceinline__ void mfma_global_tile_any(const IgemmArgs &a, int R, int S, int m_wave, int n_blk) {
    constexpr int KC = C / 32;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
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

template <int R, int S, int C, int NT>
__global__ __launch_bounds__(256) void igemm_bf16_mfma_kernel(IgemmArgs a) {
    mfma_global_tile<R, S, C, NT>(a, (blockIdx.x * kMfmaWaves + (threadIdx.x >> 6)) * (16 * kMT),
                                  blockIdx.y * (16 * NT));
}

template <int C, int NT>
__global__ __launch_bounds__(256) void igemm_bf16_mfma_any_kernel(IgemmArgs a, int R, int S) {
    mfma_global_tile_any<C, NT>(a, R, S, (blockIdx.x * kMfmaWaves + (threadIdx.x >> 6)) * (16 * kMT),
                                blockIdx.y * (16 * NT));
}

// Many multi-channel convolutions in one persistent launch (the batching
// form for BF16 requests): one descriptor per convolution (n images of one
// shape; all share C, c_out, the filter size and the padding), each
// convolution's pixels cut into blocks of one workgroup (4 waves x 64
// pixels).  A grid of about the resident capacity strides over the blocks of
// all convolutions; blockIdx.y picks the output-channel block as in the
// single launch.  Each block runs the global-load tile above, so a
// convolution's output is bit for bit that of the global-load kernel.
struct IgemmBatchDesc {
    const void *in;
    const void *w;
    float *out;
    int32_t h, wd, out_h, out_w;
    int32_t ph, pw, m_total, n;
    int64_t block_begin;  // first block of this convolution in the batch
};
static_assert(sizeof(IgemmBatchDesc) == 64, "descriptor layout");

// RS > 0: filter RS x RS unrolled; RS == 0: the runtime size rs
template <int RS, int C, int NT>
__global__ __launch_bounds__(256) void igemm_bf16_mfma_batched_kernel(const IgemmBatchDesc *__restrict__ desc,
                                                                      int n_desc, int64_t total_blocks, int c_out,
                                                                      int rs) {
    typedef const __attribute__((address_space(4))) IgemmBatchDesc cdesc;
    cdesc *d = (cdesc *)desc;
    for (int64_t item = blockIdx.x; item < total_blocks; item += gridDim.x) {
        // the convolution holding this block: last descriptor with block_begin <= item
        int lo = 0, hi = n_desc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].block_begin <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        IgemmArgs a;
        a.in = d[lo].in;
        a.w = d[lo].w;
        a.out = d[lo].out;
        a.n = d[lo].n;
        a.h = d[lo].h;
        a.wd = d[lo].wd;
        a.c_in = C;
        a.c_out = c_out;
        a.out_h = d[lo].out_h;
        a.out_w = d[lo].out_w;
        a.ph = d[lo].ph;
        a.pw = d[lo].pw;
        a.m_total = d[lo].m_total;
        const int local = (int)(item - d[lo].block_begin);
        const int m_wave = (local * kMfmaWaves + (threadIdx.x >> 6)) * (16 * kMT);
        if constexpr (RS > 0)
            mfma_global_tile<RS, RS, C, NT>(a, m_wave, blockIdx.y * (16 * NT));
        else
            mfma_global_tile_any<C, NT>(a, rs, rs, m_wave, blockIdx.y * (16 * NT));
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
// c ^ ((pos >> 1) & 3).  Every fragment read below is 16 consecutive records
// of one chunk; with this swizzle such a read is free of bank conflicts for
// any starting record (measured with the SQ_LDS_BANK_CONFLICT counter on
// gfx950, where swizzles by pos & 3 or (pos >> 2) & 3 cost about 4 conflict
// cycles per read).
// Halo rows store pixel hx at position (hx & 3) * HW4 + (hx >> 2), so F(t)
// is 16 consecutive positions.  Weights are stored [r][s][c-block][channel],
// so a B fragment (16 consecutive output channels) is 16 consecutive records.
constexpr int kLdsTW = 64;
constexpr int kRec = 64;  // bytes of one record: 32 BF16 channels

__device__ __forceinline__ int rec_slot(int c, int pos) { return c ^ ((pos >> 1) & 3); }

// Where the workgroup's weights live.
// (A slab is one filter row of weights for one 32-channel block, or for
// all of them; the next slab loads from L2 while the current one computes.)
enum WeightMode { kWeightsL2 = 0, kWeightsLds = 1, kWeightsLdsBySlab = 2, kWeightsLdsByRow = 3 };
// Added to a slab mode: the halo streams through TH+1 rows instead of being
// kept whole as a ring.
constexpr int kHaloStream = 4;

// Workgroup shape and LDS use of the staged kernel for (C, NT, F), within
// 160 KiB.  Eight output rows (eight waves, two per SIMD: one wave alone
// issues a 16x16x32 MFMA only every other slot) are preferred: with all
// weights in LDS (and the halo as a ring), else with weight slabs
// double-buffered (and the halo streamed through TH+1 rows) when the slab's
// fragments fit two waves' registers; a slab is one filter row for all
// 32-channel blocks, or for one.  Otherwise the same choices with four rows;
// last, four rows with the weights read from L2.
template <int C, int NT, int F>
struct LdsPlan {
    static constexpr int kLimit = 163840;
    static constexpr int HW4 = (kLdsTW + F - 1 + 3) / 4;
    static constexpr int rowb = 4 * HW4 * C * 2;        // one halo row, all channels
    static constexpr int ring(int th) { return (th + F - 1) * rowb; }
    static constexpr int strm(int th) { return (th + 1) * rowb; }
    static constexpr int wbytes = 16 * NT * F * F * C * 2;
    static constexpr int slab = 16 * NT * F * kRec;  // one filter row, one 32-channel block
    static constexpr int rslab = slab * (C / 32);    // one filter row, all blocks
    // slab state (fragments, slab and halo rows in flight) within two waves'
    // registers (from the compiled kernels' register counts)
    static constexpr bool regs8 = NT * (F + 3) * (C / 32) <= 40;
    static constexpr int pick() {
        if (ring(8) + wbytes <= kLimit) return 8 * 16 + kWeightsLds;
        if (regs8 && strm(8) + 2 * rslab <= kLimit) return 8 * 16 + kWeightsLdsByRow + kHaloStream;
        if (regs8 && strm(8) + 2 * slab <= kLimit) return 8 * 16 + kWeightsLdsBySlab + kHaloStream;
        if (ring(4) + wbytes <= kLimit) return 4 * 16 + kWeightsLds;
        if (ring(4) + 2 * rslab <= kLimit) return 4 * 16 + kWeightsLdsByRow;
        if (strm(4) + 2 * rslab <= kLimit) return 4 * 16 + kWeightsLdsByRow + kHaloStream;
        if (ring(4) + 2 * slab <= kLimit) return 4 * 16 + kWeightsLdsBySlab;
        if (strm(4) + 2 * slab <= kLimit) return 4 * 16 + kWeightsLdsBySlab + kHaloStream;
        return 4 * 16 + kWeightsL2;
    }
    static constexpr int TH = pick() / 16, WM = pick() % 16;
    static constexpr int halo = WM & kHaloStream ? strm(TH) : ring(TH);
    static constexpr int bytes = halo + ((WM & 3) == kWeightsLds         ? wbytes
                                         : (WM & 3) == kWeightsLdsByRow  ? 2 * rslab
                                         : (WM & 3) == kWeightsLdsBySlab ? 2 * slab
                                                                         : 0);
    static constexpr int threads = 64 * TH;
};

// Rows hy0 .. hy0+ROWS-1 of a tile's input halo: chunk k = (pixel p = k / CH,
// channel chunk q = k % CH).  LDS holds halo rows in a ring of NSLOT slots:
// halo row hy of a tile lives in slot (base + hy) % NSLOT.  With NSLOT =
// TH+R-1 (the whole halo) and base = the tile's first output row, the next
// tile down the same strip finds its first R-1 rows in place; with NSLOT =
// TH+1 and base 0 the rows stream through a window (slab modes).
template <int C, int HW, int NSLOT, int NTHR, int ROWS>
struct HaloRows {
    static constexpr int CH = C / 8, KC = C / 32, HW4 = (HW + 3) / 4;
    static constexpr int ROWB = 4 * HW4 * kRec, PLANE = NSLOT * ROWB;
    static constexpr int NCHUNK = ROWS * HW * CH, ITERS = (NCHUNK + NTHR - 1) / NTHR;
    static_assert(ITERS <= 32, "one mask bit per chunk");
    // Every load of a thread is issued before any is used.  Chunks outside the
    // image read a valid address and have their bit of *outside set; store()
    // writes zeros for them.  (Zeroing here would make the thread wait for
    // the loads, which are meant to stay in flight while a tile computes.)
    __device__ static void load(const IgemmArgs &a, int b, int y0, int x0, int hy0, u32x4 (&v)[ITERS],
                                uint32_t &outside) {
        const unsigned short *in = static_cast<const unsigned short *>(a.in);
        outside = 0;
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int p = k / CH, q = k - p * CH;
            const int hy = hy0 + p / HW, hx = p % HW;
            const int y = y0 - a.ph + hy, x = x0 - a.pw + hx;
            const bool inside = k < NCHUNK && y >= 0 && y < a.h && x >= 0 && x < a.wd;
            const size_t src = inside ? (((size_t)b * a.h + y) * a.wd + x) * C + q * 8 : 0;
            v[it] = *reinterpret_cast<const u32x4 *>(in + src);
            outside |= inside ? 0u : 1u << it;
        }
    }
    __device__ static void store(unsigned char *halo, int y0, int hy0, const u32x4 (&v)[ITERS], uint32_t outside) {
#pragma unroll
        for (int it = 0; it < ITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int p = k / CH, q = k - p * CH;
            const int slot = (y0 + hy0 + p / HW) % NSLOT, hx = p % HW;
            const int pos = (hx & 3) * HW4 + (hx >> 2);
            if (k < NCHUNK)
                *reinterpret_cast<u32x4 *>(halo + (q >> 2) * PLANE + slot * ROWB + pos * kRec +
                                           16 * rec_slot(q & 3, pos)) =
                    (outside >> it) & 1 ? u32x4{0u, 0u, 0u, 0u} : v[it];
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
// G: channel groups per workgroup (G * TH waves; wave w computes output row
// w % TH for the group's 16*NT channels w / TH, all groups sharing the halo).
template <int C, int NT, int R, int S, int TH, int WM, int G = 1>
__global__ __launch_bounds__(TH * G * 64) void igemm_bf16_lds_kernel(IgemmArgs a, int tiles_per_wg, int tile_lo,
                                                                     int tile_hi) {
    constexpr int WP = WM & 3;  // weight placement
    constexpr bool WL = WP == kWeightsLds, WSLAB = WP == kWeightsLdsBySlab || WP == kWeightsLdsByRow;
    constexpr bool STREAM = (WM & kHaloStream) != 0;
    constexpr int NKC = WP == kWeightsLdsBySlab ? 1 : C / 32;  // c-blocks per pass (and per slab)
    constexpr int CH = C / 8, KC = C / 32;
    constexpr int HW = kLdsTW + S - 1, HH = TH + R - 1;
    // A streamed halo passes through TH+1 row slots: filter row r reads rows
    // r .. r+TH-1, and row r+TH loads into the slot row r-1 has freed.
    // Otherwise the whole halo is kept as a ring shared with the next tile
    // down the strip.
    constexpr int NSLOT = STREAM ? TH + 1 : HH;
    constexpr int NTHR = TH * G * 64;
    constexpr int NTG = NT * G;  // 16-channel N-tiles of the workgroup
    typedef HaloRows<C, HW, NSLOT, NTHR, HH> Full;
    typedef HaloRows<C, HW, NSLOT, NTHR, TH> Next;
    typedef HaloRows<C, HW, NSLOT, NTHR, 1> One;
    // ring slab modes: ring row i is free once filter row i is done; rows
    // i < R-1 are refilled during filter row i+1, the rest after the tile
    constexpr int PROG = R - 1 < TH ? R - 1 : TH;
    constexpr int ENDR = TH - PROG;
    typedef HaloRows<C, HW, NSLOT, NTHR, (ENDR > 0 ? ENDR : 1)> EndRows;
    constexpr int HW4 = Full::HW4, ROWB = Full::ROWB, PLANE = Full::PLANE;
    constexpr int TAPB = 16 * NTG * kRec;  // one (tap, c-block) of the workgroup's weights
    constexpr int SLAB_BYTES = S * NKC * TAPB;     // one slab of weights
    constexpr int WCHUNK = 16 * NTG * R * S * CH;  // this workgroup's weight chunks
    constexpr int SCHUNK = 16 * NTG * S * NKC * 4; // ... of one slab
    // Ring modes: the next tile's TH new halo rows replace rows this tile has
    // finished with; with all weights in LDS they are prefetched into
    // registers while the tile computes and stored after it; with weights
    // from L2 (each weight load would wait behind a prefetch: loads complete
    // in order) they load after the tile.  Slab modes: each filter row loads
    // the halo row the next one needs, and the last filter row prefetches
    // the next tile's first TH rows.
    constexpr bool PREFETCH = WL;
    constexpr int BD = WM == kWeightsL2 ? 2 : 1;  // weight fragments are loaded BD steps ahead
    // weights first (offset 0), then the halo planes
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned char *wlds = lds;
    unsigned char *halo = lds + (WL ? R * S * KC * TAPB : WSLAB ? 2 * SLAB_BYTES : 0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = wave % TH, n_w = (wave / TH) * (16 * NT);  // this wave's output row and channel offset
    const int li = lane & 15, lg = lane >> 4;
    const int tiles_x = (a.out_w + kLdsTW - 1) / kLdsTW, tiles_y = (a.out_h + TH - 1) / TH;
    // This launch covers tiles [tile_lo, tile_hi) of the a.n * tiles_x *
    // tiles_y tiles (all of them, or one part of a convolution run in parts).
    // Workgroups are dispatched round-robin over the 8 XCDs; when the grid is
    // a multiple of 8, XCD x gets the x-th eighth of the workgroup indices, so
    // neighbouring runs of tiles share an L2.
    int g = blockIdx.x;
    if ((gridDim.x & 7) == 0) g = (g & 7) * (gridDim.x >> 3) + (g >> 3);
    const int t_begin = tile_lo + g * tiles_per_wg;
    const int t_end = min(tile_hi, t_begin + tiles_per_wg);
    if (t_begin >= t_end) return;  // uniform over the workgroup
    const int n_blk = blockIdx.y * (16 * NTG);
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
        return ((tap * KC + (q >> 2)) * (16 * NTG) + cl) * kRec + 16 * rec_slot(q & 3, cl);
    };
    // one slab of weights (slab modes): slab z = filter row r = z * NKC / KC,
    // c-blocks kc0 = z * NKC % KC .. kc0 + NKC - 1; chunk k = (channel cl,
    // tap s, chunk c of the slab's blocks), stored at (s, block, cl) like the
    // all-in-LDS layout
    constexpr int SITERS = (SCHUNK + NTHR - 1) / NTHR;
    auto wslab_load = [&](int z, u32x4(&v)[SITERS]) {
        const int r = z * NKC / KC, kc0 = z * NKC - r * KC;
#pragma unroll
        for (int it = 0; it < SITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (S * NKC * 4), rem = k - cl * (S * NKC * 4);
            const int sx = rem / (NKC * 4), c = rem - sx * (NKC * 4);
            v[it] = *reinterpret_cast<const u32x4 *>(
                wt + (k < SCHUNK ? (((size_t)(n_blk + cl) * R + r) * S + sx) * C + kc0 * 32 + c * 8 : 0));
        }
    };
    auto wslab_store = [&](int buf, const u32x4(&v)[SITERS]) {
#pragma unroll
        for (int it = 0; it < SITERS; ++it) {
            const int k = threadIdx.x + it * NTHR;
            const int cl = k / (S * NKC * 4), rem = k - cl * (S * NKC * 4);
            const int sx = rem / (NKC * 4), c = rem - sx * (NKC * 4);
            if (k < SCHUNK)
                *reinterpret_cast<u32x4 *>(wlds + buf * SLAB_BYTES + ((sx * NKC + (c >> 2)) * (16 * NTG) + cl) * kRec +
                                           16 * rec_slot(c & 3, cl)) = v[it];
        }
    };

    {
        int b, y0, x0;
        tile_origin(t_begin, b, y0, x0);
        if constexpr (STREAM) {
            u32x4 v[Next::ITERS];
            uint32_t vo;
            Next::load(a, b, y0, x0, 0, v, vo);
            Next::store(halo, 0, 0, v, vo);
        } else {
            u32x4 v[Full::ITERS];
            uint32_t vo;
            Full::load(a, b, y0, x0, 0, v, vo);
            Full::store(halo, y0, 0, v, vo);
        }
    }
    if constexpr (WL) {
        // all weights of output channels n_blk .. n_blk + 16*NTG, staged once:
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
    int wb = 0;  // slab mode: the LDS buffer holding the current slab
    if constexpr (WSLAB) {
        u32x4 v[SITERS];
        wslab_load(0, v);
        wslab_store(0, v);
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

    // The reduction of a tile runs as NZ passes: a pass is one filter row
    // (all c-blocks), or in slab mode one slab (one c-block of a row).
    constexpr int NZ = R * KC / NKC;     // passes per tile
    constexpr int NS = NKC * S;          // steps per pass
    constexpr bool UNROLLED = WSLAB || R <= 7;
    // Deferred output stores: with the passes unrolled, the weights in LDS
    // and four-row tiles (one wave per SIMD, or two with two channel groups
    // of 32 channels: registers to spare either way), a tile's results stay in
    // registers and are stored during the next tile's first passes, instead
    // of every workgroup storing at once at its tile end while the matrix
    // cores idle.  (With weights read from L2, each weight load would wait
    // behind the stores: loads and stores share one in-order counter.)
    constexpr bool DEFER = UNROLLED && WP != kWeightsL2 && TH == 4 && NZ <= 10 && S <= 5;
    constexpr int NQ = kMT * NT / 2;          // store pairs per lane and tile
    constexpr int ZS = NZ < 4 ? NZ : 4;        // passes they are spread over
    constexpr int QPZ = (NQ + ZS - 1) / ZS;    // ... per pass
    constexpr int QPS = (QPZ + NS - 1) / NS;   // ... per step
    // with deferred stores, the next tile's halo rows are prefetched halfway
    // through pass PF_Z (else at the tile start)
    constexpr int PF_Z = NZ >= 2 ? NZ - 2 : 0;
    f32x4 sv[kMT][NT];
    bool pending = false;  // sv holds a tile's results still to be stored (wave-uniform)
    // Full-line stores: a lane holds 4 channels (16 bytes) of one pixel per
    // N-tile, so one store instruction would write half of each 128-byte line
    // (16 channels of 16 pixels).  Adjacent lanes (pixels 4*li and 4*li + 4
    // of an M-tile) swap one N-tile of a pair (j, j+1) through DPP; then the
    // pair's first store writes 32 channels (one whole line) of the even
    // lane's pixel for 8 pixels, and the second those of the odd lane's pixel.
    float *sv_dst = a.out;    // even lane's pixel, this lane's channel slot
    int sv_xl0 = 0, sv_xl1 = 0;  // M-tiles m < sv_xl0 (sv_xl1) of the even (odd) lane's pixel are inside the row
    const bool odd = li & 1;
    auto store_q = [&](int q) {
        const int m = q / (NT / 2), j = 2 * (q - m * (NT / 2));
        const f32x4 send = odd ? sv[m][j] : sv[m][j + 1];
        f32x4 recv;
        // quad_perm [1,0,3,2]: swap with the adjacent lane.  Each element goes
        // through a scalar first: hipcc's __builtin_bit_cast of a vector
        // element (send[e]) reads element 0 whatever e is.
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float se = send[e];
            recv[e] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(se), 0xB1, 0xF, 0xF, true));
        }
        const f32x4 first = odd ? recv : sv[m][j], second = odd ? sv[m][j + 1] : recv;
        float *dst = sv_dst + (size_t)m * a.c_out + 16 * j;
        if (m < sv_xl0) __builtin_nontemporal_store(first, reinterpret_cast<f32x4 *>(dst));
        if (m < sv_xl1) __builtin_nontemporal_store(second, reinterpret_cast<f32x4 *>(dst + 4 * (size_t)a.c_out));
    };

    for (int t = t_begin; t < t_end; ++t) {
        const bool more = t + 1 < t_end;                   // uniform over the workgroup
        const bool down = more && (t + 1) % tiles_y != 0;  // the next tile is the one below
        int b, y0, x0;
        tile_origin(t, b, y0, x0);
        // the next tile's TH new rows: its halo rows R-1 .. R+TH-2
        u32x4 nh[Next::ITERS];
        uint32_t nho = 0;
        if constexpr (PREFETCH && !DEFER)
            if (down) Next::load(a, b, y0 + TH, x0, R - 1, nh, nho);
        // opaque per tile, so weight loads from L2 are not hoisted out of the tile loop
        const unsigned short *wtt = wt;
        asm volatile("" : "+s"(wtt));

        f32x4 acc[kMT][NT];
#pragma unroll
        for (int m = 0; m < kMT; ++m)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};

        // work slotted between the steps of unrolled passes: deferred stores
        // of the previous tile and the halo prefetch
        auto hook = [&](int z, int k) {
            if constexpr (DEFER) {
                if (pending) {
#pragma unroll
                    for (int i = 0; i < QPS; ++i) {
                        const int q = z * QPZ + k * QPS + i;
                        if (z < ZS && k * QPS + i < QPZ && q < NQ) store_q(q);
                    }
                }
                if constexpr (PREFETCH)
                    if (z == PF_Z && k == NS / 2 && down) Next::load(a, b, y0 + TH, x0, R - 1, nh, nho);
            }
        };

        // Pass z = (filter row r, first c-block kc0): steps k = (c-block
        // kc0 + k / S, tap k % S).  Step k uses F(s) .. F(s+kMT-1) of its
        // c-block and the weights of (r, s, c-block); the activation
        // fragments a step newly needs are loaded one step ahead, the weight
        // fragments BD steps ahead.  mid() runs halfway.
        auto pass = [&](int z, auto &&mid) {
            const int r = z * NKC / KC, kc0 = z * NKC - r * KC;
            const unsigned char *arow = halo + ((STREAM ? row + r : y0 + row + r) % NSLOT) * ROWB;
            u32x4 Af[NKC][kMT + S - 1], Bq[NS][NT];
            auto ld_b = [&](int k) {
                const int kk = k / S, s = k - kk * S, kc = kc0 + kk;
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    if constexpr (WL) {
                        Bq[k][j] = *reinterpret_cast<const u32x4 *>(wlds + ((r * S + s) * KC + kc) * TAPB + n_w * kRec + j * 16 * kRec + bofs);
                    } else if constexpr (WSLAB) {
                        Bq[k][j] = *reinterpret_cast<const u32x4 *>(wlds + wb * SLAB_BYTES + (s * NKC + kk) * TAPB + n_w * kRec + j * 16 * kRec + bofs);
                    } else {
                        Bq[k][j] = *reinterpret_cast<const u32x4 *>(
                            wtt + (((size_t)(n_blk + n_w + j * 16 + li) * R + r) * S + s) * C + kc * 32 + lg * 8);
                    }
                }
            };
            auto ld_f = [&](int kk, int f) {
                Af[kk][f] = *reinterpret_cast<const u32x4 *>(arow + (kc0 + kk) * PLANE + aofs[f]);
            };
            auto ld_a = [&](int k) {  // the activation fragments step k needs first
                const int kk = k / S, s = k - kk * S;
                if (s == 0) {
#pragma unroll
                    for (int f = 0; f < kMT; ++f) ld_f(kk, f);
                } else {
                    ld_f(kk, s + kMT - 1);
                }
            };
#pragma unroll
            for (int k = 0; k < BD && k < NS; ++k) ld_b(k);
            ld_a(0);
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                if (k == NS / 2) mid();  // the caller's LDS stores, while earlier MFMAs drain
                hook(z, k);
                if (k + BD < NS) ld_b(k + BD);
                if (k + 1 < NS) ld_a(k + 1);
                __builtin_amdgcn_sched_barrier(0);
                const int kk = k / S, s = k - kk * S;
                // weights as the MFMA's A operand and activations as B, so the
                // accumulator holds D[channel][pixel]: a lane's 4 results are 4
                // consecutive channels of one pixel (one 16-byte store)
#pragma unroll
                for (int m = 0; m < kMT; ++m)
#pragma unroll
                    for (int j = 0; j < NT; ++j)
                        acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, Bq[k][j]), __builtin_bit_cast(bf16x8, Af[kk][s + m]),
                            acc[m][j], 0, 0, 0);
            }
        };
        auto nothing = [] {};
        u32x4 pv[One::ITERS], ev[EndRows::ITERS];  // slab modes: halo rows in flight
        uint32_t po = 0, eo = 0;
        if constexpr (WSLAB) {
            // the next slab (slab 0 of the next tile after the last) loads
            // from L2 while this one computes and is stored halfway through
            // it; the barrier after each slab keeps the two buffers' readers
            // and writer apart
            // LAST: a pass of the last filter row (which prefetches the next
            // tile's first TH rows; a compile-time flag keeps those registers
            // out of the other passes)
            auto slab = [&](int z, auto last) {
                const bool nxt = z + 1 < NZ || more;
                const int r = z * NKC / KC;
                const bool first = z * NKC - r * KC == 0;  // the first pass of filter row r
                bool row_in = false;
                if constexpr (STREAM) {
                    row_in = first && r + TH < HH;  // this tile's halo row r+TH loads now
                    if (row_in) One::load(a, b, y0, x0, r + TH, pv, po);
                    if constexpr (decltype(last)::value) {
                        if (first && more) {  // the next tile's first TH rows
                            int b1, y1, x1;
                            tile_origin(t + 1, b1, y1, x1);
                            Next::load(a, b1, y1, x1, 0, nh, nho);
                        }
                    }
                } else if (first && down) {  // ring: refill the rows filter row r-1 freed
                    if (r >= 1 && r - 1 < PROG) One::store(halo, y0 + TH, R - 1 + (r - 1), pv, po);
                    if (r < PROG) One::load(a, b, y0 + TH, x0, R - 1 + r, pv, po);
                    if constexpr (ENDR > 0 && decltype(last)::value)
                        EndRows::load(a, b, y0 + TH, x0, R - 1 + PROG, ev, eo);
                }
                u32x4 v[SITERS];
                if (nxt) wslab_load(z + 1 < NZ ? z + 1 : 0, v);
                pass(z, [&] {
                    // row r+TH goes to the slot of row r-1, which no wave reads
                    // in filter row r (they read rows r .. r+TH-1)
                    if (row_in) One::store(halo, 0, r + TH, pv, po);
                    if (nxt) wslab_store(wb ^ 1, v);
                });
                if (z + 1 < NZ) __syncthreads();
                wb ^= 1;
            };
            constexpr int ZPR = KC / NKC;  // passes per filter row
            if constexpr (DEFER) {  // the deferred-store slots need compile-time pass indices
#pragma unroll
                for (int z = 0; z < NZ - ZPR; ++z) slab(z, std::false_type{});
            } else {  // two waves per SIMD: keep the code (and its registers) to one pass
#pragma unroll 1
                for (int z = 0; z < NZ - ZPR; ++z) slab(z, std::false_type{});
            }
#pragma unroll
            for (int z = NZ - ZPR; z < NZ; ++z) slab(z, std::true_type{});
        } else if constexpr (R <= 7) {  // small filters: the whole walk unrolled (no loop-carried accumulator copies)
#pragma unroll
            for (int z = 0; z < NZ; ++z) pass(z, nothing);
        } else {
#pragma unroll 1
            for (int z = 0; z < NZ; ++z) pass(z, nothing);
        }

        // D[i = 4*lg + e][n = li] of tiles (m, j): output channel n_blk +
        // 16*j + 4*lg + e of pixel x0 + 4*li + m; stored in pairs (see
        // store_q): the even lane of a pair writes channels 16*j + 4*lg of
        // both pixels, the odd lane channels 16*(j+1) + 4*lg
        const int y = y0 + row;
        pending = y < a.out_h;
        const int xe = x0 + 4 * (li & ~1);
        sv_dst = a.out + (((size_t)b * a.out_h + y) * a.out_w + xe) * a.c_out + n_blk + n_w + 16 * (li & 1) + 4 * lg;
        sv_xl0 = min(kMT, a.out_w - xe);
        sv_xl1 = min(kMT, a.out_w - (xe + 4));
#pragma unroll
        for (int m = 0; m < kMT; ++m)
#pragma unroll
            for (int j = 0; j < NT; ++j) sv[m][j] = acc[m][j];
        if (!DEFER || !more) {
            if (pending) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) store_q(q);
            }
            pending = false;
        }
        if (more) {
            __syncthreads();  // every wave is done with this tile's halo rows
            if constexpr (STREAM) {
                Next::store(halo, 0, 0, nh, nho);
            } else if (down) {
                if constexpr (WSLAB) {
                    if constexpr (ENDR > 0) EndRows::store(halo, y0 + TH, R - 1 + PROG, ev, eo);
                } else {
                    if constexpr (!PREFETCH) Next::load(a, b, y0 + TH, x0, R - 1, nh, nho);
                    Next::store(halo, y0 + TH, R - 1, nh, nho);
                }
            } else {  // a new strip: the whole halo
                int b1, y1, x1;
                tile_origin(t + 1, b1, y1, x1);
                u32x4 v[Full::ITERS];
                uint32_t vo;
                Full::load(a, b1, y1, x1, 0, v, vo);
                Full::store(halo, y1, 0, v, vo);
            }
            __syncthreads();
        }
    }
}

// FP32 implicit GEMM on the vector ALUs (the comparison path).  A workgroup
// computes 64 consecutive output pixels of one output row x 64 output
// channels; thread (tm, tn) holds a 4 x 4 register tile (pixels 4*tm ..,
// channels 4*tn ..).  The reduction runs over steps (r, s, 16-channel chunk):
// a step's A (16 channels x 64 pixels, from NHWC input) and B (16 channels x
// 64 output channels, from KRSC weights) are staged in LDS channel-major and
// double-buffered, the next step's loads in flight while the current step
// computes.  Per channel a thread reads 4 pixels and 4 weights (two 16-byte
// LDS reads, the same addresses across its 16-lane groups) for 16 FMAs
// v_fmac acc, v_a, v_b.  Each output is one FP32 FMA chain in (r, s, c)
// order.
constexpr int kF32M = 64, kF32N = 64, kF32K = 16, kF32Pitch = 68;  // LDS row: 64 values + 4 (bank spread)

template <int C>
__global__ __launch_bounds__(256) void igemm_f32_tiled_kernel(IgemmArgs a, int R, int S) {
    __shared__ __align__(16) float As[2][kF32K][kF32Pitch];
    __shared__ __align__(16) float Bs[2][kF32K][kF32Pitch];
    const int t = threadIdx.x;
    const int tm = t & 15, tn = t >> 4;
    const int tiles_x = (a.out_w + kF32M - 1) / kF32M;
    const int row = blockIdx.x / tiles_x;  // b * out_h + y
    const int x0 = (blockIdx.x - row * tiles_x) * kF32M;
    const int b = row / a.out_h, y = row - b * a.out_h;
    const int n0 = blockIdx.y * kF32N;
    const float *in = static_cast<const float *>(a.in);
    const float *wt = static_cast<const float *>(a.w);
    // staging: thread t loads 4 channels (quad sq) of pixel / output channel sp
    const int sp = t >> 2, sq = t & 3;
    constexpr int CHUNKS = C / kF32K;
    const int steps = R * S * CHUNKS;
    // inputs outside the image load a valid address and are zeroed when
    // stored (zeroing at the load would make the thread wait for it)
    auto load = [&](int step, float4 &va, float4 &vb, bool &ok) {
        const int rs = step / CHUNKS, ch = step - rs * CHUNKS;
        const int r = rs / S, s = rs - r * S;
        const int c = ch * kF32K + sq * 4;
        const int yy = y + r - a.ph, xx = x0 + sp + s - a.pw;
        ok = yy >= 0 && yy < a.h && xx >= 0 && xx < a.wd;
        va = *reinterpret_cast<const float4 *>(in + (ok ? (((size_t)b * a.h + yy) * a.wd + xx) * C + c : 0));
        vb = *reinterpret_cast<const float4 *>(wt + (((size_t)(n0 + sp) * R + r) * S + s) * C + c);
    };
    auto store = [&](int buf, const float4 &va, const float4 &vb, bool ok) {
        const float4 z = ok ? va : make_float4(0.f, 0.f, 0.f, 0.f);
        As[buf][sq * 4 + 0][sp] = z.x;
        As[buf][sq * 4 + 1][sp] = z.y;
        As[buf][sq * 4 + 2][sp] = z.z;
        As[buf][sq * 4 + 3][sp] = z.w;
        Bs[buf][sq * 4 + 0][sp] = vb.x;
        Bs[buf][sq * 4 + 1][sp] = vb.y;
        Bs[buf][sq * 4 + 2][sp] = vb.z;
        Bs[buf][sq * 4 + 3][sp] = vb.w;
    };
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    float4 va, vb;
    bool ok;
    load(0, va, vb, ok);
    store(0, va, vb, ok);
    __syncthreads();
    for (int step = 0; step < steps; ++step) {
        const int cur = step & 1;
        const bool more = step + 1 < steps;
        if (more) load(step + 1, va, vb, ok);
#pragma unroll
        for (int k = 0; k < kF32K; ++k) {
            const float4 av = *reinterpret_cast<const float4 *>(&As[cur][k][tm * 4]);
            const float4 bv = *reinterpret_cast<const float4 *>(&Bs[cur][k][tn * 4]);
            const float ai[4] = {av.x, av.y, av.z, av.w}, bj[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fmaf(ai[i], bj[j], acc[i][j]);
        }
        // the other buffer was last read in the previous step, before its barrier
        if (more) store(cur ^ 1, va, vb, ok);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int x = x0 + 4 * tm + i;
        if (x < a.out_w)
            *reinterpret_cast<float4 *>(a.out + ((size_t)row * a.out_w + x) * a.c_out + n0 + 4 * tn) =
                make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
    }
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

// The batched global-load kernel for (filter, c_in, c_out): unrolled for
// filter sizes 1, 3, 5, 7, the runtime-size walk otherwise.
#define GT_BM(RS)                                                                           \
    {RS, 64, 4, (const void *)&igemm_bf16_mfma_batched_kernel<RS, 64, 4>},                 \
        {RS, 64, 2, (const void *)&igemm_bf16_mfma_batched_kernel<RS, 64, 2>},             \
        {RS, 32, 4, (const void *)&igemm_bf16_mfma_batched_kernel<RS, 32, 4>},             \
        {RS, 32, 2, (const void *)&igemm_bf16_mfma_batched_kernel<RS, 32, 2>}
struct BatchedMfmaEntry {
    int rs, c, nt;
    const void *fn;
};
const BatchedMfmaEntry kBatchedMfma[] = {GT_BM(0), GT_BM(1), GT_BM(3), GT_BM(5), GT_BM(7)};
#undef GT_BM
constexpr size_t kBatchedMfmaSize = sizeof(kBatchedMfma) / sizeof(kBatchedMfma[0]);
std::atomic<int> g_batched_mfma_occupancy[kBatchedMfmaSize];

const BatchedMfmaEntry *batched_mfma_for(int f, int c, int c_out) {
    const int nt = (c_out % 64 == 0) ? 4 : 2;
    const int rs = (f == 1 || f == 3 || f == 5 || f == 7) ? f : 0;
    for (const BatchedMfmaEntry &e : kBatchedMfma)
        if (e.rs == rs && e.c == c && e.nt == nt) return &e;
    return nullptr;
}

const void *valu_kernel_for(int c) {
    if (c == 64) return (const void *)&igemm_f32_tiled_kernel<64>;
    if (c == 32) return (const void *)&igemm_f32_tiled_kernel<32>;
    return nullptr;
}

struct LdsEntry {
    int c, nt, f;  // nt: 16-channel N-tiles per workgroup
    const void *fn;
    int lds, th, threads;
    int g;  // channel groups per workgroup
};
#define GT_L(C, NT, F)                                                                                     \
    {C, NT, F, (const void *)&igemm_bf16_lds_kernel<C, NT, F, F, LdsPlan<C, NT, F>::TH, LdsPlan<C, NT, F>::WM>, \
     LdsPlan<C, NT, F>::bytes, LdsPlan<C, NT, F>::TH, LdsPlan<C, NT, F>::threads, 1}
// two channel groups of NT N-tiles, all weights in LDS, the halo a ring of TH+F-1 rows
#define GT_LG(C, NT, F, TH)                                                                                  \
    {C, 2 * NT, F, (const void *)&igemm_bf16_lds_kernel<C, NT, F, F, TH, kWeightsLds, 2>,                     \
     LdsPlan<C, 2 * NT, F>::ring(TH) + LdsPlan<C, 2 * NT, F>::wbytes, TH, 2 * TH * 64, 2}
const LdsEntry kLdsTable[] = {
    GT_L(64, 4, 1), GT_L(64, 4, 3), GT_L(64, 4, 5), GT_L(64, 4, 7), GT_L(64, 4, 9),
    GT_L(64, 2, 1), GT_L(64, 2, 3), GT_L(64, 2, 5), GT_L(64, 2, 7), GT_L(64, 2, 9),
    GT_L(32, 4, 1), GT_L(32, 4, 3), GT_L(32, 4, 5), GT_L(32, 4, 7), GT_L(32, 4, 9), GT_L(32, 4, 17),
    GT_L(32, 2, 1), GT_L(32, 2, 3), GT_L(32, 2, 5), GT_L(32, 2, 7), GT_L(32, 2, 9), GT_L(32, 2, 17),
    GT_LG(64, 2, 3, 4), GT_LG(32, 2, 3, 4),
};
#undef GT_L
#undef GT_LG
constexpr size_t kLdsTableSize = sizeof(kLdsTable) / sizeof(kLdsTable[0]);
std::atomic<int> g_lds_occupancy[kLdsTableSize];  // resident workgroups per CU, 0 = not yet queried

const LdsEntry *lds_entry(int f, int c, int nt, int g = 1) {
    for (const LdsEntry &e : kLdsTable)
        if (e.g == g && e.c == c && e.nt == nt && e.f == f && e.lds <= state().dev.lds_per_block) return &e;
    return nullptr;
}

// The LDS-staged kernel for (c_in, c_out, f) when instantiated and its LDS
// fits the device; null otherwise.  With c_out a multiple of 64: the
// two-group kernel where there is one (3x3: four-row tiles of 64 channels,
// two waves per SIMD, four tiles per workgroup at N=16, 128x128 instead of
// two, so loads and stores overlap more of the compute; 0-10 % faster
// across hosts), else workgroups of 64 output channels, unless only
// 32-channel workgroups get eight rows (two waves per SIMD); measured on 5x5,
// C=64: 0.059 -> 0.055 ms.
// rows = 4 or 8 asks for the instance with that many output rows per tile
// where the shape has one (the time-optimal instance is not always the
// energy-optimal one); any other value takes the default order.
const LdsEntry *lds_kernel_for(int f, int c, int c_out, int rows = 0) {
    const LdsEntry *cand[3] = {nullptr, nullptr, nullptr};
    if (c_out % 64 != 0) {
        cand[0] = lds_entry(f, c, 2);
    } else {
        const LdsEntry *e4 = lds_entry(f, c, 4), *e2 = lds_entry(f, c, 2);
        const bool two_first = e4 && e4->th < 8 && e2 && e2->th == 8;
        cand[0] = lds_entry(f, c, 4, 2);
        cand[1] = two_first ? e2 : e4;
        cand[2] = two_first ? e4 : e2;
    }
    if (rows == 4 || rows == 8)
        for (const LdsEntry *e : cand)
            if (e && e->th == rows) return e;
    for (const LdsEntry *e : cand)
        if (e) return e;
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
        if (!valu_kernel_for(p.c_in))
            return set_error(GT_E_UNSUPPORTED, "igemm f32: c_in %d not instantiated (32 or 64)", p.c_in);
    }
    return GT_OK;
}

int launch_igemm(const gt_problem &p, const gt_conv_config &c, const void *in, const void *w, void *out,
                 hipStream_t s, int part, int n_parts) {
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
    if (p.kind == GT_IGEMM_BF16_MFMA && p.filt_h == p.filt_w && ((uintptr_t)out & 15) == 0) {
        if (const LdsEntry *e = lds_kernel_for(p.filt_h, p.c_in, p.c_out, c.tile_size_y)) {
            const int64_t all_tiles = (int64_t)p.n * ((p.out_h + e->th - 1) / e->th) * ((p.out_w + kLdsTW - 1) / kLdsTW);
            if (all_tiles >= ((int64_t)1 << 31)) return set_error(GT_E_INVAL, "igemm: too many tiles");
            // part k of n: tiles [all * k / n, all * (k + 1) / n)
            const int64_t tile_lo = all_tiles * part / n_parts, tile_hi = all_tiles * (part + 1) / n_parts;
            const int64_t tiles = tile_hi - tile_lo;
            if (tiles == 0) return GT_OK;  // more parts than tiles: this one is empty
            const int gy = p.c_out / (16 * e->nt);
            const size_t idx = (size_t)(e - kLdsTable);
            int occ = g_lds_occupancy[idx].load(std::memory_order_relaxed);
            if (occ == 0) {
                if (e->lds > 65536)
                    GT_HIP_CHECK(hipFuncSetAttribute(e->fn, hipFuncAttributeMaxDynamicSharedMemorySize, e->lds));
                GT_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, e->fn, e->threads, (size_t)e->lds));
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
            int tiles_per_wg = (int)per, lo = (int)tile_lo, hi = (int)tile_hi;
            void *largs[] = {&a, &tiles_per_wg, &lo, &hi};
            dim3 grid((unsigned)gx, (unsigned)gy);
            GT_HIP_CHECK(hipLaunchKernel(e->fn, grid, dim3(e->threads), largs, (size_t)e->lds, s));
            return GT_OK;
        }
    }
    if (n_parts != 1)
        return set_error(GT_E_UNSUPPORTED, "igemm: a run in parts needs the LDS-staged BF16 kernel (square "
                         "filter, instantiated filter size and channels, 16-byte aligned output)");
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
        if ((uintptr_t)out & 15) return set_error(GT_E_INVAL, "igemm f32: output must be 16-byte aligned");
        const int64_t tiles = (int64_t)p.n * p.out_h * ((p.out_w + kF32M - 1) / kF32M);
        if (tiles >= ((int64_t)1 << 31)) return set_error(GT_E_INVAL, "igemm f32: too many tiles");
        int R = p.filt_h, S = p.filt_w;
        void *fargs[] = {&a, &R, &S};
        dim3 grid((unsigned)tiles, (unsigned)(p.c_out / kF32N));
        GT_HIP_CHECK(hipLaunchKernel(valu_kernel_for(p.c_in), grid, dim3(256), fargs, 0, s));
    }
    return GT_OK;
}


// Shape checks shared by the batched pack and launch: BF16 MFMA, square
// filter, channels instantiated.
static int validate_igemm_batch_shape(const gt_problem &p) {
    if (p.kind != GT_IGEMM_BF16_MFMA) return set_error(GT_E_UNSUPPORTED, "igemm batch: BF16 MFMA problems only");
    if (p.filt_h < 1 || p.filt_h != p.filt_w) return set_error(GT_E_UNSUPPORTED, "igemm batch: square filters only");
    if (p.pad_h < 0 || p.pad_w < 0) return set_error(GT_E_INVAL, "igemm batch: negative padding");
    if (p.c_out < 32 || p.c_out % 32 != 0)
        return set_error(GT_E_UNSUPPORTED, "igemm batch: c_out must be a multiple of 32");
    if (!batched_mfma_for(p.filt_h, p.c_in, p.c_out))
        return set_error(GT_E_UNSUPPORTED, "igemm batch: c_in %d not instantiated (32 or 64)", p.c_in);
    return GT_OK;
}

}  // namespace gt

using namespace gt;

extern "C" int gt_igemm_batch_pack(const gt_problem *shape, const gt_batch_item *items, int32_t n_items,
                                   void *host_blob, size_t capacity, size_t *blob_bytes, int64_t *total_blocks) {
    clear_error();
    if (!shape || !items || n_items < 1 || !blob_bytes || !total_blocks || (capacity && !host_blob))
        return set_error(GT_E_INVAL, "gt_igemm_batch_pack: bad argument");
    int rc = validate_igemm_batch_shape(*shape);
    if (rc) return rc;
    const int f = shape->filt_h;
    const size_t need = sizeof(IgemmBatchDesc) * (size_t)n_items;
    *blob_bytes = need;
    std::vector<IgemmBatchDesc> d((size_t)n_items);
    const int64_t per_block = (int64_t)kMfmaWaves * kMT * 16;
    int64_t blocks = 0;
    for (int32_t k = 0; k < n_items; ++k) {
        const gt_batch_item &it = items[k];
        if (!it.d_in || !it.d_filt || !it.d_out || it.out_h < 1 || it.out_w < 1)
            return set_error(GT_E_INVAL, "gt_igemm_batch_pack: item %d is not valid", k);
        if (it.filt_h != f || it.filt_w != f)
            return set_error(GT_E_INVAL, "gt_igemm_batch_pack: item %d: filter %dx%d, the batch's is %d", k,
                             it.filt_h, it.filt_w, f);
        if ((((uintptr_t)it.d_in) | ((uintptr_t)it.d_filt)) & 15)
            return set_error(GT_E_INVAL, "gt_igemm_batch_pack: item %d: input and weights must be 16-byte aligned", k);
        const int64_t h = (int64_t)it.out_h + f - 1 - 2 * shape->pad_h, w = (int64_t)it.out_w + f - 1 - 2 * shape->pad_w;
        if (h < 1 || w < 1) return set_error(GT_E_INVAL, "gt_igemm_batch_pack: item %d: padding too large", k);
        const int64_t m = (int64_t)it.out_h * it.out_w;
        if (m >= ((int64_t)1 << 31) - per_block || h * w * shape->c_in >= ((int64_t)1 << 31))
            return set_error(GT_E_INVAL, "gt_igemm_batch_pack: item %d too large", k);
        IgemmBatchDesc &x = d[(size_t)k];
        x.in = it.d_in;
        x.w = it.d_filt;
        x.out = static_cast<float *>(it.d_out);
        x.h = (int32_t)h;
        x.wd = (int32_t)w;
        x.out_h = it.out_h;
        x.out_w = it.out_w;
        x.ph = shape->pad_h;
        x.pw = shape->pad_w;
        x.m_total = (int32_t)m;
        x.n = 1;
        x.block_begin = blocks;
        blocks += (m + per_block - 1) / per_block;
    }
    *total_blocks = blocks;
    if (capacity < need) return set_error(GT_E_CAPACITY, "gt_igemm_batch_pack: %zu bytes needed", need);
    memcpy(host_blob, d.data(), need);
    return GT_OK;
}

extern "C" int conv2d_run_igemm_batched(const gt_problem *shape, const void *d_blob, int32_t n_items,
                                        int64_t total_blocks, int32_t grid_blocks, void *hip_stream) {
    clear_error();
    if (!shape || !d_blob || n_items < 1 || total_blocks < 1)
        return set_error(GT_E_INVAL, "conv2d_run_igemm_batched: bad argument");
    if (!state().inited || (state().flags & GT_INIT_HOST_ONLY))
        return set_error(GT_E_STATE, "conv2d_run_igemm_batched: needs gt_init on a device");
    if ((uintptr_t)d_blob & 7)
        return set_error(GT_E_INVAL, "conv2d_run_igemm_batched: descriptor blob must be 8-byte aligned");
    int rc = validate_igemm_batch_shape(*shape);
    if (rc) return rc;
    const BatchedMfmaEntry *e = batched_mfma_for(shape->filt_h, shape->c_in, shape->c_out);
    const int gy = shape->c_out / (16 * e->nt);
    int64_t grid;
    if (grid_blocks <= 0) {
        // about the resident capacity (surplus blocks are strided over)
        const size_t idx = (size_t)(e - kBatchedMfma);
        int occ = g_batched_mfma_occupancy[idx].load(std::memory_order_relaxed);
        if (occ == 0) {
            GT_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, e->fn, 256, 0));
            occ = std::max(1, occ);
            g_batched_mfma_occupancy[idx].store(occ, std::memory_order_relaxed);
        }
        const int64_t resident = std::max<int64_t>(1, (int64_t)std::max(1, state().dev.cu_count) * occ / gy);
        grid = std::min(total_blocks, resident);
    } else {
        grid = std::min<int64_t>(grid_blocks, total_blocks);
    }
    const IgemmBatchDesc *desc = static_cast<const IgemmBatchDesc *>(d_blob);
    int n = n_items, c_out = shape->c_out, rs = shape->filt_h;
    int64_t tb = total_blocks;
    void *args[] = {&desc, &n, &tb, &c_out, &rs};
    GT_HIP_CHECK(hipLaunchKernel(e->fn, dim3((unsigned)grid, (unsigned)gy), dim3(256), args, 0, (hipStream_t)hip_stream));
    return GT_OK;
}
