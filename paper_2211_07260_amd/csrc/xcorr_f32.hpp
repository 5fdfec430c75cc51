// Tunable single-channel FP32 2-D cross-correlation for gfx950.
//
//   out[y][x] = sum_{i < fh} sum_{j < FW} in[y+i][x+j] * w[i][j]     (valid, no flip)
//
// Tunables (the section IV style: thread-block dimensions, work per thread,
// shared-memory use, read path):
//   blockDim.x/y       workgroup shape (runtime)
//   TX, TY             outputs per thread along x / y (template)
//   read path RP       0: the workgroup stages its input halo in LDS;
//                      1: each thread reads global memory (L1/L2) directly
//   LDS padding        runtime row pitch = ceil4(bx*TX + FW - 1) + 4*pad floats
//
// Every thread owns a TY x TX register tile of contiguous outputs.  For each
// filter row i and each of its TY output rows it loads one input row segment
// of TX + FW - 1 floats into registers and issues TX * FW FMAs against the
// filter row, which is wave-uniform and therefore sits in SGPRs (scalar
// loads), so each FMA is v_fmac_f32 acc, s_w, v_in.  Each output's sum is
// accumulated in one FP32 chain in (i, j) order, so every configuration
// produces bit-identical results.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

// Largest vector width (1, 2 or 4 floats) usable for LDS row reads that start
// at a multiple of TX floats inside a 16-byte aligned row.
template <int TX>
struct RowVec {
    static constexpr int value = (TX % 4 == 0) ? 4 : ((TX % 2 == 0) ? 2 : 1);
};

template <int V> struct VecT;
template <> struct VecT<1> { typedef float type; };
template <> struct VecT<2> { typedef float2 type; };
template <> struct VecT<4> { typedef float4 type; };

template <int N, int V>
__device__ __forceinline__ void load_row_lds(float (&row)[N], const float *src) {
    typedef typename VecT<V>::type vt;
    constexpr int NV = N / V;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        vt v = reinterpret_cast<const vt *>(src)[k];
        const float *pv = reinterpret_cast<const float *>(&v);
#pragma unroll
        for (int e = 0; e < V; ++e) row[k * V + e] = pv[e];
    }
#pragma unroll
    for (int k = NV * V; k < N; ++k) row[k] = src[k];
}

// Global rows start at arbitrary float offsets; gfx950 global loads accept
// dword alignment, so use 16-byte loads through memcpy (align 4).
template <int N>
__device__ __forceinline__ void load_row_global(float (&row)[N], const float *src) {
    constexpr int NV = N / 4;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        float4 v;
        __builtin_memcpy(&v, src + 4 * k, sizeof(float4));
        row[4 * k + 0] = v.x;
        row[4 * k + 1] = v.y;
        row[4 * k + 2] = v.z;
        row[4 * k + 3] = v.w;
    }
#pragma unroll
    for (int k = NV * 4; k < N; ++k) row[k] = src[k];
}

template <int TX, int TY, int FW>
__device__ __forceinline__ void fma_row(float (&acc)[TY][TX], int r, const float (&row)[TX + FW - 1],
                                        const float (&wr)[FW]) {
#pragma unroll
    for (int j = 0; j < FW; ++j)
#pragma unroll
        for (int c = 0; c < TX; ++c) acc[r][c] = __builtin_fmaf(row[c + j], wr[j], acc[r][c]);
}

// Store a thread's TY x TX tile at (y, x).  Full tiles of aligned rows use
// 16-byte stores; otherwise each element is bounds-checked.
typedef float f4nt __attribute__((ext_vector_type(4)));
template <int TX, int TY>
__device__ __forceinline__ void store_tile(const float (&acc)[TY][TX], float *out, int out_h, int out_w,
                                           int y, int x, bool full) {
    if constexpr (TX % 4 == 0) {
        if (full) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                float4 *dst = reinterpret_cast<float4 *>(out + (size_t)(y + r) * out_w + x);
#pragma unroll
                for (int k = 0; k < TX / 4; ++k)
                    __builtin_nontemporal_store(f4nt{acc[r][4 * k], acc[r][4 * k + 1], acc[r][4 * k + 2], acc[r][4 * k + 3]}, (f4nt *)&dst[k]);
            }
            return;
        }
    }
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        if (y + r < out_h) {
            float *dst = out + (size_t)(y + r) * out_w;
#pragma unroll
            for (int c = 0; c < TX; ++c)
                if (x + c < out_w) dst[x + c] = acc[r][c];
        }
    }
}

struct XcorrArgs {
    const float *in;
    const float *w;
    float *out;
    int32_t out_h, out_w, in_h, in_w, fh;
    int32_t lds_pitch;  // floats (read path 0)
    int32_t vec_ok;     // input base pointer is 16-byte aligned
    int32_t out_vec_ok; // output base pointer 16-byte aligned and out_w % 4 == 0
};

// One workgroup tile whose top-left output is (x0, y0), LDS read path.  Used
// by the one-launch-per-convolution kernel and by the persistent batched
// kernel, so both produce bit-identical outputs.
template <int TX, int TY, int FW, bool UNROLL_OK = true>
__device__ __forceinline__ void xcorr_tile_lds(const XcorrArgs &a, int x0, int y0, float *lds) {
    constexpr int RW = TX + FW - 1;  // input row segment per thread
    const int bx = blockDim.x, by = blockDim.y;
    const int lx = threadIdx.x * TX, ly = threadIdx.y * TY;
    const int fh = a.fh;
    // The filter is read through the constant address space: its wave-uniform
    // loads become scalar loads into SGPRs regardless of other memory traffic.
    const __attribute__((address_space(4))) float *w = (const __attribute__((address_space(4))) float *)a.w;

    float acc[TY][TX];
#pragma unroll
    for (int r = 0; r < TY; ++r)
#pragma unroll
        for (int c = 0; c < TX; ++c) acc[r][c] = 0.0f;
    const int pitch = a.lds_pitch;
    const int tile_w = bx * TX + FW - 1;
    const int tile_h = by * TY + fh - 1;
    const float *__restrict__ in = a.in;
    // Stage the halo as 16-byte chunks.  Interior blocks (the common case)
    // read whole chunks with no clamping, four chunks in flight per
    // thread; blocks at the right or bottom edge clamp every element
    // (values past the input only feed outputs that are never stored).
    const int tid_x = threadIdx.x, tid_y = threadIdx.y;
    const int nthr = bx * by, tid = tid_y * bx + tid_x;
    const int tw4 = (tile_w + 3) >> 2;
    const int nchunks = tile_h * tw4;
    const bool interior = a.vec_ok && ((a.in_w & 3) == 0) && ((x0 & 3) == 0) &&
                          x0 + 4 * tw4 <= a.in_w && y0 + tile_h <= a.in_h;
    if (interior) {
        // Chunk k of the tile is row k / tw4, column k % tw4; a thread
        // walks k = tid, tid + nthr, ... keeping (row, column) updated
        // incrementally.  Loads past the tile re-read chunk 0 (in bounds)
        // so the four loads issue back to back; their stores are skipped.
        const float4 *src4 = reinterpret_cast<const float4 *>(in + (size_t)y0 * a.in_w + x0);
        float4 *lds4 = reinterpret_cast<float4 *>(lds);
        const int in_w4 = a.in_w >> 2, pitch4 = pitch >> 2;
        const int dr = nthr / tw4, dc = nthr - dr * tw4;
        int r = tid / tw4, c = tid - r * tw4;
        // (named registers, not arrays: the scheduling barrier below would
        // otherwise keep four-element arrays in scratch memory)
        auto fetch = [&](int idx, float4 &v, int &off) {
            const bool ok = idx < nchunks;
            v = src4[ok ? r * in_w4 + c : 0];
            off = ok ? r * pitch4 + c : -1;
            c += dc;
            r += dr;
            if (c >= tw4) {
                c -= tw4;
                ++r;
            }
        };
        for (int idx = tid; idx < nchunks; idx += 4 * nthr) {
            float4 v0, v1, v2, v3;
            int o0, o1, o2, o3;
            fetch(idx, v0, o0);
            fetch(idx + nthr, v1, o1);
            fetch(idx + 2 * nthr, v2, o2);
            fetch(idx + 3 * nthr, v3, o3);
            __builtin_amdgcn_sched_barrier(0);  // keep the four loads ahead of the stores
            if (o0 >= 0) lds4[o0] = v0;
            if (o1 >= 0) lds4[o1] = v1;
            if (o2 >= 0) lds4[o2] = v2;
            if (o3 >= 0) lds4[o3] = v3;
        }
    } else {
        for (int r = tid_y; r < tile_h; r += by) {
            const int gy = min(y0 + r, a.in_h - 1);
            const float *src = in + (size_t)gy * a.in_w;
            float *dst = lds + r * pitch;
            for (int c = tid_x; c < tile_w; c += bx) dst[c] = src[min(x0 + c, a.in_w - 1)];
        }
    }
    __syncthreads();

    constexpr int V = RowVec<TX>::value;
    const float *base = lds + ly * pitch + lx;
    auto filter_row = [&](int i) {
        float wr[FW];
#pragma unroll
        for (int j = 0; j < FW; ++j) wr[j] = w[i * FW + j];
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            float row[RW];
            load_row_lds<RW, V>(row, base + (r + i) * pitch);
            fma_row<TX, TY, FW>(acc, r, row, wr);
        }
    };
    // Square filters with a moderate per-thread tile run the filter rows
    // fully unrolled: the row addresses are then fixed offsets from one base,
    // and a row shared by neighbouring output rows is read from LDS once
    // (fh + ty - 1 row reads instead of fh * ty), which saves time and
    // power.  Bounded by code size (tx*ty*fw^2 FMAs) and, under the
    // 1024-thread bound of 128 VGPRs, by the rows a thread keeps live: a row
    // serves ty output rows, so up to ty rows of tx + fw - 1 values (the one
    // tile past that bound, 4 x 8 at 17x17, spills when unrolled).  Not in the
    // batched kernel for tx < 4, where the hoisted row loads spill.  The FMA
    // order is the same either way.
    constexpr int FMAS = TX * TY * FW * FW;
    constexpr bool UNROLL_ROWS = UNROLL_OK && (FMAS <= 2400 || (FMAS <= 10000 && TY * (TX + FW - 1) <= 128));
    if (UNROLL_ROWS && fh == FW) {
#pragma unroll
        for (int i = 0; i < FW; ++i) filter_row(i);
    } else {
        for (int i = 0; i < fh; ++i) filter_row(i);
    }
    store_tile<TX, TY>(acc, a.out, a.out_h, a.out_w, y0 + ly, x0 + lx,
                       a.out_vec_ok && x0 + bx * TX <= a.out_w && y0 + by * TY <= a.out_h);
}

// One workgroup tile, direct read path (no LDS).
template <int TX, int TY, int FW>
__device__ __forceinline__ void xcorr_tile_direct(const XcorrArgs &a, int x0, int y0) {
    constexpr int RW = TX + FW - 1;
    const int lx = threadIdx.x * TX, ly = threadIdx.y * TY;
    const int fh = a.fh;
    const __attribute__((address_space(4))) float *w = (const __attribute__((address_space(4))) float *)a.w;

    float acc[TY][TX];
#pragma unroll
    for (int r = 0; r < TY; ++r)
#pragma unroll
        for (int c = 0; c < TX; ++c) acc[r][c] = 0.0f;
    // Direct read path.  A thread whose tile hangs over the right or
    // bottom edge computes the tile shifted back inside the output (same
    // sums, in-bounds reads) and stores only its own outputs.
    const int xt = x0 + lx, yt = y0 + ly;
    const int xs = min(xt, a.out_w - TX), ys = min(yt, a.out_h - TY);
    const float *base = a.in + (size_t)ys * a.in_w + xs;
    for (int i = 0; i < fh; ++i) {
        float wr[FW];
#pragma unroll
        for (int j = 0; j < FW; ++j) wr[j] = w[i * FW + j];
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            float row[RW];
            load_row_global<RW>(row, base + (size_t)(r + i) * a.in_w);
            fma_row<TX, TY, FW>(acc, r, row, wr);
        }
    }
#pragma unroll
    for (int r = 0; r < TY; ++r) {
        const int y = ys + r;
        if (y >= yt) {
            float *dst = a.out + (size_t)y * a.out_w;
#pragma unroll
            for (int c = 0; c < TX; ++c) {
                const int x = xs + c;
                if (x >= xt) dst[x] = acc[r][c];
            }
        }
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (linear id mod 8),
// each XCD with its own L2.  Remap so that XCD k processes the k-th eighth of
// the tiles in row-major order: horizontally adjacent tiles, which share
// fw-1 halo columns, then run on the same XCD and share its L2.
__device__ __forceinline__ void xcd_tile(int &tx, int &ty) {
    const int gx = gridDim.x, n = gx * gridDim.y;
    const int lin = blockIdx.y * gx + blockIdx.x;
    int t = lin;
    if ((n & 7) == 0) t = (lin & 7) * (n >> 3) + (lin >> 3);
    ty = t / gx;
    tx = t - ty * gx;
}

template <int TX, int TY, int FW, int RP>
__global__ __launch_bounds__(1024) void xcorr_f32_kernel(XcorrArgs a) {
    int tx, ty;
    xcd_tile(tx, ty);
    const int x0 = tx * blockDim.x * TX, y0 = ty * blockDim.y * TY;
    if constexpr (RP == 0) {
        extern __shared__ __align__(16) float lds[];
        xcorr_tile_lds<TX, TY, FW>(a, x0, y0, lds);
    } else {
        xcorr_tile_direct<TX, TY, FW>(a, x0, y0);
    }
}

struct XcorrEntry {
    int32_t tx, ty, fw, rp;
    const void *fn;
};

}  // namespace gt

// One translation unit per TX value instantiates TY 1..8 x FW x read path.
#define GT_XCORR_ENTRIES_FW(TX, TY, FW) \
    {TX, TY, FW, 0, (const void *)&gt::xcorr_f32_kernel<TX, TY, FW, 0>}, \
    {TX, TY, FW, 1, (const void *)&gt::xcorr_f32_kernel<TX, TY, FW, 1>},
#define GT_XCORR_ENTRIES_TY(TX, TY) \
    GT_XCORR_ENTRIES_FW(TX, TY, 3) GT_XCORR_ENTRIES_FW(TX, TY, 5) \
    GT_XCORR_ENTRIES_FW(TX, TY, 9) GT_XCORR_ENTRIES_FW(TX, TY, 17)
#define GT_XCORR_TABLE(TX)                                                                      \
    extern "C++" const gt::XcorrEntry gt_xcorr_table_tx##TX[] = {                               \
        GT_XCORR_ENTRIES_TY(TX, 1) GT_XCORR_ENTRIES_TY(TX, 2) GT_XCORR_ENTRIES_TY(TX, 3)        \
        GT_XCORR_ENTRIES_TY(TX, 4) GT_XCORR_ENTRIES_TY(TX, 5) GT_XCORR_ENTRIES_TY(TX, 6)        \
        GT_XCORR_ENTRIES_TY(TX, 7) GT_XCORR_ENTRIES_TY(TX, 8) {0, 0, 0, 0, nullptr}};
