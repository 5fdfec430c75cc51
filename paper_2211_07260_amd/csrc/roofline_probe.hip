// Roofline probes: the achievable FP32 vector FMA rate (the same
// v_fmac_f32 acc, s_w, v_in form the convolution issues, packed FP32
// disabled), the HBM copy bandwidth, and the BF16 MFMA issue rate with one
// and two waves per SIMD, measured on the device at hand.
#include <hip/hip_runtime.h>

#include "gt_internal.hpp"

namespace gt {

// Uniform value in [0.5, 1) from a 32-bit integer hash (scalar when k is).
__device__ __forceinline__ float hashed_unit(uint32_t k) {
    k ^= k >> 16;
    k *= 0x7FEB352Du;
    k ^= k >> 15;
    k *= 0x846CA68Bu;
    k ^= k >> 16;
    return __uint_as_float(0x3F000000u | (k >> 9));
}

// 32 independent accumulators, 8 input registers, weights from SGPRs:
// 256 FMAs per loop trip per lane.  Operands are hashed per workgroup and
// lane (no memory is read).  kMix: after every trip the inputs take the
// accumulators' mantissa bits (x in [1, 2)), so the operands keep changing
// the way a real kernel's do (the power a calibration load draws depends on
// operand toggling); the probe leaves them fixed to time the bare FMA rate.
template <bool kMix>
__global__ __launch_bounds__(256) void fma_peak_kernel(float *out, int iters) {
    float acc[32], x[8], s[8];
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = 2.0f * hashed_unit(blockIdx.x * 2048u + threadIdx.x * 8u + k);
        s[k] = hashed_unit(0x9E3779B9u ^ (blockIdx.x * 8u + k));
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
#pragma unroll
            for (int k = 0; k < 32; ++k) acc[k] = __builtin_fmaf(x[(k + j) & 7], s[j], acc[k]);
        }
        if (kMix) {
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = __uint_as_float((__float_as_uint(acc[4 * k + (it & 3)]) & 0x007FFFFFu) | 0x3F800000u);
        }
    }
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < 32; ++k) t += acc[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// 16 independent 16x16x32 BF16 MFMA chains per wave (no loads): the matrix
// cores' issue rate for this instruction.
__global__ __launch_bounds__(256) void mfma_peak_kernel(float *out, int iters) {
    typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    f32x4 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 x, y;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = (__bf16)(1e-3f * (float)(threadIdx.x + k));
        y[k] = (__bf16)(1e-3f * (float)k);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[k], 0, 0, 0);
    }
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

typedef float f4v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(const float4 *__restrict__ src0, float4 *__restrict__ dst0,
                                                   size_t n4) {
    const f4v *src = (const f4v *)src0;
    f4v *dst = (f4v *)dst0;
    const size_t per_trip = (size_t)gridDim.x * 512;
    for (size_t base = (size_t)blockIdx.x * 512 + threadIdx.x; base < n4; base += per_trip) {
        f4v v0 = {0.f, 0.f, 0.f, 0.f}, v1 = v0;
        const bool two = base + 256 < n4;
        v0 = __builtin_nontemporal_load(&src[base]);
        if (two) v1 = __builtin_nontemporal_load(&src[base + 256]);
        __builtin_nontemporal_store(v0, &dst[base]);
        if (two) __builtin_nontemporal_store(v1, &dst[base + 256]);
    }
}

// Synthetic full-load kernels for measure_load: work per launch (flops, or
// bytes moved for the copy) and the launch itself.
namespace {
constexpr int kLoadFmaIters = 256, kLoadMfmaIters = 512;
int load_cus() { return state().dev.cu_count > 0 ? state().dev.cu_count : 256; }
}  // namespace

int load_work(int kind, size_t bytes, double *work) {
    const int cus = load_cus();
    switch (kind) {
        case GT_LOAD_FP32_FMA: {
            const int blocks = cus * 8;
            if ((size_t)blocks * 256 * sizeof(float) > bytes)
                return set_error(GT_E_INVAL, "measure_load: buffer too small for the FMA load");
            *work = 2.0 * 256.0 * kLoadFmaIters * (double)blocks * 256;
            return GT_OK;
        }
        case GT_LOAD_BF16_MFMA: {
            const int blocks = cus * 2;
            if ((size_t)blocks * 256 * sizeof(float) > bytes)
                return set_error(GT_E_INVAL, "measure_load: buffer too small for the MFMA load");
            *work = 16384.0 * 16.0 * kLoadMfmaIters * (double)blocks * 4;
            return GT_OK;
        }
        case GT_LOAD_COPY: {
            const size_t half = (bytes / 2) / 16 * 16;
            if (half < (1u << 20)) return set_error(GT_E_INVAL, "measure_load: the copy load needs >= 2 MiB");
            *work = 2.0 * (double)half;
            return GT_OK;
        }
        default:
            return set_error(GT_E_INVAL, "measure_load: unknown load kind %d", kind);
    }
}

int launch_load(int kind, void *buf, size_t bytes, hipStream_t s) {
    const int cus = load_cus();
    float *out = static_cast<float *>(buf);
    if (kind == GT_LOAD_FP32_FMA) {
        const int blocks = cus * 8;
        hipLaunchKernelGGL(fma_peak_kernel<true>, dim3(blocks), dim3(256), 0, s, out, kLoadFmaIters);
    } else if (kind == GT_LOAD_BF16_MFMA) {
        hipLaunchKernelGGL(mfma_peak_kernel, dim3(cus * 2), dim3(256), 0, s, out, kLoadMfmaIters);
    } else {
        const size_t half = (bytes / 2) / 16 * 16;
        const float4 *src = static_cast<const float4 *>(buf);
        float4 *dst = reinterpret_cast<float4 *>(static_cast<char *>(buf) + half);
        hipLaunchKernelGGL(copy_kernel, dim3(cus * 64), dim3(256), 0, s, src, dst, half / 16);
    }
    GT_HIP_CHECK(hipGetLastError());
    return GT_OK;
}

}  // namespace gt

using namespace gt;

extern "C" int gt_roofline_probe(void *d_buf, size_t bytes, void *hip_stream, double *fp32_fma_tflops,
                                 double *copy_gbs) {
    clear_error();
    if (!d_buf || !fp32_fma_tflops || !copy_gbs) return set_error(GT_E_INVAL, "gt_roofline_probe: null argument");
    if (!state().inited || (state().flags & GT_INIT_HOST_ONLY))
        return set_error(GT_E_STATE, "gt_roofline_probe: needs gt_init on a device");
    const size_t half = (bytes / 2) / 16 * 16;
    if (half < (1u << 20)) return set_error(GT_E_INVAL, "gt_roofline_probe: buffer must hold at least 2 MiB");
    hipStream_t s = (hipStream_t)hip_stream;
    const int cus = state().dev.cu_count > 0 ? state().dev.cu_count : 256;
    const int blocks = cus * 8, iters = 2048;
    if ((size_t)blocks * 256 * sizeof(float) > bytes)
        return set_error(GT_E_INVAL, "gt_roofline_probe: buffer too small");
    float *out = static_cast<float *>(d_buf);
    hipEvent_t a, b;
    GT_HIP_CHECK(hipEventCreate(&a));
    GT_HIP_CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(fma_peak_kernel<false>, dim3(blocks), dim3(256), 0, s, out, iters);  // warm
    GT_HIP_CHECK(hipEventRecord(a, s));
    hipLaunchKernelGGL(fma_peak_kernel<false>, dim3(blocks), dim3(256), 0, s, out, iters);
    GT_HIP_CHECK(hipEventRecord(b, s));
    GT_HIP_CHECK(hipEventSynchronize(b));
    float ms = 0;
    GT_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    *fp32_fma_tflops = 2.0 * 256.0 * iters * (double)blocks * 256 / (ms * 1e-3) / 1e12;

    const size_t n4 = half / 16;
    const float4 *src = static_cast<const float4 *>(d_buf);
    float4 *dst = reinterpret_cast<float4 *>(static_cast<char *>(d_buf) + half);
    hipLaunchKernelGGL(copy_kernel, dim3(cus * 64), dim3(256), 0, s, src, dst, n4);
    GT_HIP_CHECK(hipEventRecord(a, s));
    const int reps = 10;
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(copy_kernel, dim3(cus * 64), dim3(256), 0, s, src, dst, n4);
    GT_HIP_CHECK(hipEventRecord(b, s));
    GT_HIP_CHECK(hipEventSynchronize(b));
    GT_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    *copy_gbs = 2.0 * (double)n4 * 16 * reps / (ms * 1e-3) / 1e9;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return GT_OK;
}

extern "C" int gt_mfma_probe(void *d_buf, size_t bytes, void *hip_stream, double *tflops_1wave,
                             double *tflops_2wave) {
    clear_error();
    if (!d_buf || !tflops_1wave || !tflops_2wave) return set_error(GT_E_INVAL, "gt_mfma_probe: null argument");
    if (!state().inited || (state().flags & GT_INIT_HOST_ONLY))
        return set_error(GT_E_STATE, "gt_mfma_probe: needs gt_init on a device");
    hipStream_t s = (hipStream_t)hip_stream;
    const int cus = state().dev.cu_count > 0 ? state().dev.cu_count : 256;
    const int iters = 4000;
    if ((size_t)cus * 2 * 256 * sizeof(float) > bytes) return set_error(GT_E_INVAL, "gt_mfma_probe: buffer too small");
    float *out = static_cast<float *>(d_buf);
    hipEvent_t a, b;
    GT_HIP_CHECK(hipEventCreate(&a));
    GT_HIP_CHECK(hipEventCreate(&b));
    double *res[2] = {tflops_1wave, tflops_2wave};
    for (int w = 1; w <= 2; ++w) {  // w workgroups of 4 waves per CU: w waves per SIMD
        const int blocks = cus * w;
        hipLaunchKernelGGL(mfma_peak_kernel, dim3(blocks), dim3(256), 0, s, out, 16);  // warm
        GT_HIP_CHECK(hipEventRecord(a, s));
        hipLaunchKernelGGL(mfma_peak_kernel, dim3(blocks), dim3(256), 0, s, out, iters);
        GT_HIP_CHECK(hipEventRecord(b, s));
        GT_HIP_CHECK(hipEventSynchronize(b));
        float ms = 0;
        GT_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
        *res[w - 1] = 16384.0 * 16.0 * iters * (double)blocks * 4 / (ms * 1e-3) / 1e12;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return GT_OK;
}
