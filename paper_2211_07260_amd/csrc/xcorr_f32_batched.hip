// Persistent batched FP32 cross-correlation: many convolutions in one launch.
//
// The host packs a descriptor per convolution (pointers, sizes, and the
// index of its first tile in the concatenated tile list).  A grid sized to
// the device's resident capacity walks the tile list with a static stride
// (item = blockIdx.x, blockIdx.x + gridDim.x, ...): no counters, so the
// launch can be captured in a graph and replayed as is.  Each item runs the
// same LDS tile body as the one-launch-per-convolution kernel, so a
// convolution's output is bit-identical whether it runs alone or batched.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "gt_internal.hpp"
#include "xcorr_f32.hpp"

namespace gt {

struct BatchDesc {
    const float *in;
    const float *w;
    float *out;
    int32_t out_h, out_w;
    int32_t tiles_x;
    int32_t flags;       // bit 0: input 16-byte aligned; bit 1: output aligned and out_w % 4 == 0
    int64_t tile_begin;  // first tile of this convolution in the batch
};
static_assert(sizeof(BatchDesc) == 48, "descriptor layout");

template <int TX, int TY, int FW>
__global__ __launch_bounds__(1024) void xcorr_f32_batched_kernel(const BatchDesc *__restrict__ desc, int n_desc,
                                                                 int64_t total_tiles, int lds_pitch) {
    extern __shared__ __align__(16) float lds[];
    typedef const __attribute__((address_space(4))) BatchDesc cdesc;
    cdesc *d = (cdesc *)desc;
    // Workgroups are dispatched round-robin over the 8 XCDs.  When the grid is
    // a multiple of 8, XCD x walks the x-th eighth of the tile list, so
    // neighbouring tiles of one convolution share that XCD's L2.
    int64_t first = blockIdx.x, last = total_tiles, step = gridDim.x;
    if ((gridDim.x & 7) == 0) {
        const int64_t chunk = (total_tiles + 7) / 8;
        const int x = blockIdx.x & 7;
        first = x * chunk + (blockIdx.x >> 3);
        last = min(total_tiles, (int64_t)(x + 1) * chunk);
        step = gridDim.x >> 3;
    }
    for (int64_t item = first; item < last; item += step) {
        // the convolution holding this tile: last descriptor with tile_begin <= item
        int lo = 0, hi = n_desc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].tile_begin <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t local = item - d[lo].tile_begin;
        const int ty = (int)(local / d[lo].tiles_x), tx = (int)(local - (int64_t)ty * d[lo].tiles_x);
        XcorrArgs a;
        a.in = d[lo].in;
        a.w = d[lo].w;
        a.out = d[lo].out;
        a.out_h = d[lo].out_h;
        a.out_w = d[lo].out_w;
        a.in_h = a.out_h + FW - 1;
        a.in_w = a.out_w + FW - 1;
        a.fh = FW;
        a.lds_pitch = lds_pitch;
        a.vec_ok = d[lo].flags & 1;
        a.out_vec_ok = (d[lo].flags >> 1) & 1;
        __syncthreads();  // the previous item's LDS tile is no longer read
        xcorr_tile_lds<TX, TY, FW, TX % 4 == 0>(a, tx * blockDim.x * TX, ty * blockDim.y * TY, lds);
    }
}

namespace {

struct BatchEntry {
    int tx, ty, fw;
    const void *fn;
};

#define GT_B(TX, TY, FW) {TX, TY, FW, (const void *)&xcorr_f32_batched_kernel<TX, TY, FW>}
#define GT_B_FW(TX, TY) GT_B(TX, TY, 3), GT_B(TX, TY, 5), GT_B(TX, TY, 9), GT_B(TX, TY, 17)
#define GT_B_TY(TX) GT_B_FW(TX, 1), GT_B_FW(TX, 2), GT_B_FW(TX, 4), GT_B_FW(TX, 8)
const BatchEntry kBatchTable[] = {GT_B_TY(1), GT_B_TY(2), GT_B_TY(4), GT_B_TY(8)};
#undef GT_B_TY
#undef GT_B_FW
#undef GT_B

const void *batched_fn(int tx, int ty, int fw) {
    for (const BatchEntry &e : kBatchTable)
        if (e.tx == tx && e.ty == ty && e.fw == fw) return e.fn;
    return nullptr;
}

int validate_batch_config(const gt_conv_config &c, int fw) {
    if (c.read_path != 0) return set_error(GT_E_UNSUPPORTED, "batched: LDS read path only");
    if (c.block_size_x < 1 || c.block_size_y < 1) return set_error(GT_E_INVAL, "batched: bad block size");
    if ((int64_t)c.block_size_x * c.block_size_y > state().dev.max_threads)
        return set_error(GT_E_UNSUPPORTED, "batched: too many threads per block");
    if (!batched_fn(c.tile_size_x, c.tile_size_y, fw))
        return set_error(GT_E_UNSUPPORTED, "batched: tile %dx%d / filter %d not instantiated (tiles 1, 2, 4, 8; "
                         "filters 3, 5, 9, 17)", c.tile_size_x, c.tile_size_y, fw);
    return GT_OK;
}

int64_t batch_lds_bytes(const gt_conv_config &c, int fw) {
    gt_problem p{GT_XCORR_F32, 1, 1, 1, 1, 1, fw, fw, 0, 0};
    return xcorr_lds_bytes(p, c);
}

// Descriptor of item k of a batch whose earlier items cover *tiles tiles;
// advances *tiles.  fw: the batch's filter size.
int fill_desc(const gt_batch_item &it, int k, int fw, const gt_conv_config &cfg, int64_t *tiles, BatchDesc *d) {
    if (!it.d_in || !it.d_filt || !it.d_out || it.out_h < 1 || it.out_w < 1)
        return set_error(GT_E_INVAL, "batch: item %d is not valid", k);
    if (it.filt_h != fw || it.filt_w != fw)
        return set_error(GT_E_INVAL, "batch: item %d: all items need the same square filter (%d)", k, fw);
    if ((int64_t)(it.out_h + fw - 1) * (it.out_w + fw - 1) >= (int64_t)1 << 31)
        return set_error(GT_E_INVAL, "batch: item %d too large", k);
    const int64_t ox = (int64_t)cfg.block_size_x * cfg.tile_size_x, oy = (int64_t)cfg.block_size_y * cfg.tile_size_y;
    const int64_t tx = (it.out_w + ox - 1) / ox, ty = (it.out_h + oy - 1) / oy;
    d->in = static_cast<const float *>(it.d_in);
    d->w = static_cast<const float *>(it.d_filt);
    d->out = static_cast<float *>(it.d_out);
    d->out_h = it.out_h;
    d->out_w = it.out_w;
    d->tiles_x = (int32_t)tx;
    d->flags = ((((uintptr_t)it.d_in & 15) == 0) ? 1 : 0) |
               (((((uintptr_t)it.d_out & 15) == 0) && it.out_w % 4 == 0) ? 2 : 0);
    d->tile_begin = *tiles;
    *tiles += tx * ty;
    return GT_OK;
}

// One persistent launch over a descriptor array in device memory (see
// conv2d_run_batched).
int launch_batched(const BatchDesc *desc, int32_t n_items, int64_t total_tiles, int32_t filt,
                   const gt_conv_config &cfg, int32_t grid_blocks, hipStream_t stream) {
    const int64_t lds = batch_lds_bytes(cfg, filt);
    if (lds > state().dev.lds_per_block) return set_error(GT_E_UNSUPPORTED, "batched: LDS tile too large");
    const void *fn = batched_fn(cfg.tile_size_x, cfg.tile_size_y, filt);
    if (lds > 65536) GT_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int threads = cfg.block_size_x * cfg.block_size_y;
    int64_t grid;
    if (grid_blocks <= 0) {
        // The resident capacity; twice that for the VALU-bound filters (9 and
        // up): workgroups beyond the resident ones start as others finish,
        // which evens out the last round (measured +2-6 % for 17x17, while
        // the HBM-bound 3x3 and 5x5 lose 2-3 % the same way, and a grid
        // balanced to equal tiles per workgroup loses 10 % at 17x17).  A
        // multiple of 8 for the per-XCD tile order.
        int per_cu = 0;
        GT_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, (size_t)lds));
        const int64_t resident = (int64_t)std::max(1, per_cu) * std::max(1, state().dev.cu_count);
        grid = std::min<int64_t>(total_tiles, (filt >= 9 ? 2 : 1) * resident);
        if (grid >= 8) grid = grid / 8 * 8;
    } else {
        grid = std::min<int64_t>(grid_blocks, total_tiles);
    }
    const int pitch = (int)((cfg.block_size_x * cfg.tile_size_x + filt - 1 + 3) / 4 * 4 +
                            4 * (cfg.use_lds_padding ? 1 : 0));
    int n = n_items;
    int64_t tt = total_tiles;
    void *args[] = {&desc, &n, &tt, (void *)&pitch};
    GT_HIP_CHECK(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(cfg.block_size_x, cfg.block_size_y), args,
                                 (size_t)lds, stream));
    return GT_OK;
}

}  // namespace

// ---- the allocation-free batched launch ----
//
// Its descriptors live in `scratch`, a file-scope device array (one copy per
// GPU, held until the process ends), instead of a caller-provided device
// blob.  They reach it through kernel arguments: the host packs up to
// kUploadChunk descriptors into an argument block and a one-wave kernel
// stores them, so the call needs neither device allocation nor a host
// staging buffer that must outlive it, and stays asynchronous on the stream.
// In host code `scratch` names a host-side stand-in: kernels get the device
// address hipGetSymbolAddress returns, kept per device.
constexpr int kUploadChunk = 64;
struct DescChunk {
    int32_t first, n;
    int32_t pad[2];
    BatchDesc d[kUploadChunk];
};
static_assert(sizeof(DescChunk) <= 4096 - 64, "kernel-argument block");

static __device__ __align__(256) BatchDesc scratch[GT_BATCH_NOALLOC_MAX_ITEMS];

__global__ __launch_bounds__(64) void batch_desc_upload_kernel(BatchDesc *dst, DescChunk chunk) {
    const int k = threadIdx.x;
    if (k < chunk.n) {
        // 48 bytes: dword reads of the argument block (8-byte aligned), three
        // 16-byte vector stores (the array is 256-byte aligned, a record 48)
        typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
        const unsigned int *src = reinterpret_cast<const unsigned int *>(&chunk.d[k]);
        u32x4v *to = reinterpret_cast<u32x4v *>(dst + chunk.first + k);
#pragma unroll
        for (int q = 0; q < 3; ++q) to[q] = u32x4v{src[4 * q], src[4 * q + 1], src[4 * q + 2], src[4 * q + 3]};
    }
}

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static BatchDesc *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
static int scratch_ptr(BatchDesc **out) {
    int dev = -1;
    GT_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(GT_E_STATE, "batched (no allocation): device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        GT_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(GT_E_HIP, "batched (no allocation): no device address for the descriptor array");
        g_scratch_ptr[dev] = static_cast<BatchDesc *>(p);
    }
    *out = g_scratch_ptr[dev];
    return GT_OK;
}

}  // namespace gt

using namespace gt;

extern "C" {

int gt_batch_pack(const gt_batch_item *items, int32_t n_items, const gt_conv_config *cfg, void *host_blob,
                  size_t capacity, size_t *blob_bytes, int64_t *total_tiles) {
    clear_error();
    if (!items || n_items < 1 || !cfg || !blob_bytes || !total_tiles || (capacity && !host_blob))
        return set_error(GT_E_INVAL, "gt_batch_pack: bad argument");
    const int fw = items[0].filt_w;
    int rc = validate_batch_config(*cfg, fw);
    if (rc) return rc;
    const size_t need = sizeof(BatchDesc) * (size_t)n_items;
    *blob_bytes = need;
    std::vector<BatchDesc> d((size_t)n_items);
    int64_t tiles = 0;
    for (int32_t k = 0; k < n_items; ++k) {
        rc = fill_desc(items[k], k, fw, *cfg, &tiles, &d[k]);
        if (rc) return rc;
    }
    *total_tiles = tiles;
    if (capacity < need) return set_error(GT_E_CAPACITY, "gt_batch_pack: %zu bytes needed", need);
    memcpy(host_blob, d.data(), need);
    return GT_OK;
}

int conv2d_run_batched(const void *d_blob, int32_t n_items, int64_t total_tiles, int32_t filt,
                       const gt_conv_config *cfg, int32_t grid_blocks, void *hip_stream) {
    clear_error();
    if (!d_blob || n_items < 1 || total_tiles < 1 || !cfg)
        return set_error(GT_E_INVAL, "conv2d_run_batched: bad argument");
    if (!state().inited || (state().flags & GT_INIT_HOST_ONLY))
        return set_error(GT_E_STATE, "conv2d_run_batched: needs gt_init on a device");
    if ((uintptr_t)d_blob & 7) return set_error(GT_E_INVAL, "conv2d_run_batched: descriptor blob must be 8-byte aligned");
    int rc = validate_batch_config(*cfg, filt);
    if (rc) return rc;
    return launch_batched(static_cast<const BatchDesc *>(d_blob), n_items, total_tiles, filt, *cfg, grid_blocks,
                          (hipStream_t)hip_stream);
}

int conv2d_run_batched_noalloc(const gt_batch_item *items, int32_t n_items, const gt_conv_config *cfg,
                               int32_t grid_blocks, void *hip_stream) {
    clear_error();
    if (!items || !cfg) return set_error(GT_E_INVAL, "conv2d_run_batched_noalloc: bad argument");
    if (n_items < 1 || n_items > GT_BATCH_NOALLOC_MAX_ITEMS)
        return set_error(GT_E_INVAL, "conv2d_run_batched_noalloc: %d items; 1 to %d fit the device descriptor array",
                         n_items, GT_BATCH_NOALLOC_MAX_ITEMS);
    if (!state().inited || (state().flags & GT_INIT_HOST_ONLY))
        return set_error(GT_E_STATE, "conv2d_run_batched_noalloc: needs gt_init on a device");
    const int fw = items[0].filt_w;
    int rc = validate_batch_config(*cfg, fw);
    if (rc) return rc;
    // every item is checked before anything is issued
    int64_t tiles = 0;
    for (int32_t k = 0; k < n_items; ++k) {
        BatchDesc d;
        rc = fill_desc(items[k], k, fw, *cfg, &tiles, &d);
        if (rc) return rc;
    }
    if (batch_lds_bytes(*cfg, fw) > state().dev.lds_per_block)
        return set_error(GT_E_UNSUPPORTED, "conv2d_run_batched_noalloc: LDS tile too large");
    BatchDesc *dev_desc = nullptr;
    rc = scratch_ptr(&dev_desc);
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)hip_stream;
    tiles = 0;
    for (int32_t k0 = 0; k0 < n_items; k0 += kUploadChunk) {
        DescChunk chunk;
        memset(&chunk, 0, sizeof chunk);
        chunk.first = k0;
        chunk.n = std::min(kUploadChunk, n_items - k0);
        for (int i = 0; i < chunk.n; ++i) fill_desc(items[k0 + i], k0 + i, fw, *cfg, &tiles, &chunk.d[i]);
        hipLaunchKernelGGL(batch_desc_upload_kernel, dim3(1), dim3(64), 0, stream, dev_desc, chunk);
        GT_HIP_CHECK(hipGetLastError());
    }
    return launch_batched(dev_desc, n_items, tiles, fw, *cfg, grid_blocks, stream);
}

int measure_batched_time_energy(const void *d_blob, int32_t n_items, int64_t total_tiles, int32_t filt,
                                const gt_conv_config *cfg, int32_t grid_blocks, double flops_per_launch,
                                gt_clock clock, const gt_measure_opts *opts, void *hip_stream, gt_measurement *rec) {
    clear_error();
    if (!d_blob || n_items < 1 || total_tiles < 1 || !cfg || !rec || !(flops_per_launch > 0))
        return set_error(GT_E_INVAL, "measure_batched_time_energy: bad argument");
    if (!state().inited || (state().flags & GT_INIT_HOST_ONLY))
        return set_error(GT_E_STATE, "measure_batched_time_energy: needs gt_init on a device");
    if ((uintptr_t)d_blob & 7)
        return set_error(GT_E_INVAL, "measure_batched_time_energy: descriptor blob must be 8-byte aligned");
    int rc = validate_batch_config(*cfg, filt);
    if (rc) return rc;
    const gt_measure_opts o = opts ? *opts : gt_measure_opts{0, -1, 0, 0, -1, 0};
    if (o.window_s > 0 && o.discard_s >= o.window_s)
        return set_error(GT_E_INVAL, "measure_batched_time_energy: discard %.3f s >= window %.3f s", o.discard_s,
                         o.window_s);
    rc = dvfs_apply(clock);
    if (rc) return rc;
    const BatchDesc *desc = static_cast<const BatchDesc *>(d_blob);
    const gt_conv_config c = *cfg;
    return measure_window(
        [&](hipStream_t s) { return launch_batched(desc, n_items, total_tiles, filt, c, grid_blocks, s); },
        flops_per_launch, o, (hipStream_t)hip_stream, rec);
}

// ---- graph capture of a launch sequence ----

int gt_graph_begin(void *hip_stream) {
    clear_error();
    if (!hip_stream) return set_error(GT_E_INVAL, "gt_graph_begin: capture needs a non-null stream");
    GT_HIP_CHECK(hipStreamBeginCapture((hipStream_t)hip_stream, hipStreamCaptureModeThreadLocal));
    return GT_OK;
}

int gt_graph_end(void *hip_stream, void **graph_exec) {
    clear_error();
    if (!hip_stream || !graph_exec) return set_error(GT_E_INVAL, "gt_graph_end: bad argument");
    hipGraph_t g = nullptr;
    GT_HIP_CHECK(hipStreamEndCapture((hipStream_t)hip_stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(GT_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    *graph_exec = ex;
    return GT_OK;
}

int gt_graph_launch(void *graph_exec, void *hip_stream) {
    clear_error();
    if (!graph_exec) return set_error(GT_E_INVAL, "gt_graph_launch: null graph");
    GT_HIP_CHECK(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)hip_stream));
    return GT_OK;
}

int gt_graph_destroy(void *graph_exec) {
    clear_error();
    if (graph_exec) GT_HIP_CHECK(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
    return GT_OK;
}

}  // extern "C"
