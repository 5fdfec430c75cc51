// Host side of the FP32 cross-correlation: configuration checks, LDS sizing,
// kernel lookup and launch.
#include <unordered_map>

#include "gt_internal.hpp"
#include "xcorr_f32.hpp"

extern const gt::XcorrEntry gt_xcorr_table_tx1[], gt_xcorr_table_tx2[], gt_xcorr_table_tx3[],
    gt_xcorr_table_tx4[], gt_xcorr_table_tx5[], gt_xcorr_table_tx6[], gt_xcorr_table_tx7[],
    gt_xcorr_table_tx8[];

namespace gt {

namespace {

int key_of(int tx, int ty, int fw, int rp) { return ((tx * 16 + ty) * 64 + fw) * 2 + rp; }

struct Registry {
    std::unordered_map<int, const void *> fn;
    std::unordered_map<const void *, int64_t> lds_attr;  // dynamic-LDS limit already set
    std::mutex mu;
    Registry() {
        const XcorrEntry *tabs[] = {gt_xcorr_table_tx1, gt_xcorr_table_tx2, gt_xcorr_table_tx3,
                                    gt_xcorr_table_tx4, gt_xcorr_table_tx5, gt_xcorr_table_tx6,
                                    gt_xcorr_table_tx7, gt_xcorr_table_tx8};
        for (const XcorrEntry *t : tabs)
            for (; t->fn; ++t) fn[key_of(t->tx, t->ty, t->fw, t->rp)] = t->fn;
    }
};

Registry &registry() {
    static Registry r;
    return r;
}

}  // namespace

int64_t xcorr_lds_bytes(const gt_problem &p, const gt_conv_config &c) {
    if (c.read_path != 0) return 0;
    const int64_t w = (int64_t)c.block_size_x * c.tile_size_x + p.filt_w - 1;
    const int64_t pitch = (w + 3) / 4 * 4 + 4 * (c.use_lds_padding ? 1 : 0);
    return 4 * pitch * ((int64_t)c.block_size_y * c.tile_size_y + p.filt_h - 1);
}

int validate_xcorr(const gt_problem &p, const gt_conv_config &c, int64_t lds_limit, int max_threads) {
    if (p.n != 1 || p.c_in != 1 || p.c_out != 1 || p.pad_h != 0 || p.pad_w != 0)
        return set_error(GT_E_INVAL, "xcorr: n, c_in, c_out must be 1 and padding 0");
    if (p.out_h < 1 || p.out_w < 1 || p.filt_h < 1 || p.filt_w < 1)
        return set_error(GT_E_INVAL, "xcorr: sizes must be positive");
    if ((int64_t)(p.out_h + p.filt_h - 1) * (p.out_w + p.filt_w - 1) >= (int64_t)1 << 31)
        return set_error(GT_E_INVAL, "xcorr: input too large for 32-bit indexing");
    if (c.block_size_x < 1 || c.block_size_y < 1 || c.tile_size_x < 1 || c.tile_size_y < 1)
        return set_error(GT_E_INVAL, "xcorr: config values must be positive");
    if (c.tile_size_x > 8 || c.tile_size_y > 8)
        return set_error(GT_E_UNSUPPORTED, "xcorr: tile sizes above 8 are not instantiated");
    if (p.filt_w != 3 && p.filt_w != 5 && p.filt_w != 9 && p.filt_w != 17)
        return set_error(GT_E_UNSUPPORTED, "xcorr: filter width %d not instantiated (3, 5, 9, 17)",
                         p.filt_w);
    if (c.read_path != 0 && c.read_path != 1)
        return set_error(GT_E_INVAL, "xcorr: read_path must be 0 or 1");
    if (c.use_lds_padding != 0 && c.use_lds_padding != 1)
        return set_error(GT_E_INVAL, "xcorr: use_lds_padding must be 0 or 1");
    if ((int64_t)c.block_size_x * c.block_size_y > max_threads)
        return set_error(GT_E_UNSUPPORTED, "xcorr: %d x %d threads exceed %d", c.block_size_x,
                         c.block_size_y, max_threads);
    if (c.read_path == 0 && xcorr_lds_bytes(p, c) > lds_limit)
        return set_error(GT_E_UNSUPPORTED, "xcorr: LDS tile of %lld bytes exceeds %lld",
                         (long long)xcorr_lds_bytes(p, c), (long long)lds_limit);
    if (c.read_path == 1 && (c.tile_size_x > p.out_w || c.tile_size_y > p.out_h))
        return set_error(GT_E_UNSUPPORTED, "xcorr: direct read path needs tiles within the output");
    return GT_OK;
}

int launch_xcorr_f32(const gt_problem &p, const gt_conv_config &c, const void *in, const void *w,
                     void *out, hipStream_t s) {
    Registry &reg = registry();
    auto it = reg.fn.find(key_of(c.tile_size_x, c.tile_size_y, p.filt_w, c.read_path));
    if (it == reg.fn.end()) return set_error(GT_E_UNSUPPORTED, "xcorr: no kernel instance");
    const void *fn = it->second;
    const int64_t lds = xcorr_lds_bytes(p, c);
    if (lds > 65536) {
        std::lock_guard<std::mutex> lk(reg.mu);
        auto a = reg.lds_attr.find(fn);
        if (a == reg.lds_attr.end() || a->second < lds) {
            GT_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            reg.lds_attr[fn] = lds;
        }
    }
    XcorrArgs a;
    a.in = static_cast<const float *>(in);
    a.w = static_cast<const float *>(w);
    a.out = static_cast<float *>(out);
    a.out_h = p.out_h;
    a.out_w = p.out_w;
    a.in_h = p.out_h + p.filt_h - 1;
    a.in_w = p.out_w + p.filt_w - 1;
    a.fh = p.filt_h;
    const int64_t tw = (int64_t)c.block_size_x * c.tile_size_x + p.filt_w - 1;
    a.lds_pitch = (int32_t)((tw + 3) / 4 * 4 + 4 * (c.use_lds_padding ? 1 : 0));
    a.vec_ok = (((uintptr_t)in & 15) == 0) ? 1 : 0;
    a.out_vec_ok = ((((uintptr_t)out & 15) == 0) && (p.out_w % 4 == 0)) ? 1 : 0;
    const int64_t ox = (int64_t)c.block_size_x * c.tile_size_x;
    const int64_t oy = (int64_t)c.block_size_y * c.tile_size_y;
    dim3 grid((unsigned)((p.out_w + ox - 1) / ox), (unsigned)((p.out_h + oy - 1) / oy));
    dim3 block((unsigned)c.block_size_x, (unsigned)c.block_size_y);
    if (grid.y > 65535) return set_error(GT_E_UNSUPPORTED, "xcorr: grid.y %u too large", grid.y);
    void *args[] = {&a};
    GT_HIP_CHECK(hipLaunchKernel(fn, grid, block, args, (size_t)lds, s));
    return GT_OK;
}

}  // namespace gt
