/*
 * Oracle (test infrastructure only): plain FP64 CPU reference for the
 * convolution workloads the tuner measures.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load this file's library;
 * the product path never does.
 *
 * The paper fixes no convolution kernel; the workload definition it is
 * checked against is the textbook one.  Tunable-kernel style follows the
 * paper's Experimental setup section (GEMM tunables: tile sizes, thread-block
 * dimensions, shared-memory use); the quantity computed here is the plain
 * definition:
 *
 *   single channel (valid region, no flip):
 *     out[y][x] = sum_{i<fh} sum_{j<fw} in[y+i][x+j] * w[i][j]
 *
 *   multi channel, NHWC activations, KRSC weights, stride 1, zero padding:
 *     out[n][h][x][co] = sum_{ci,r,s} in[n][h+r-ph][x+s-pw][ci] * wt[co][r][s][ci]
 *
 * Every FP32 (or BF16-valued FP32) input is widened exactly to FP64 and
 * accumulated in FP64, in the loop order of the definition.  OpenMP over
 * output rows is used only to bound wall time; it does not change any
 * individual sum.
 */
#include <stddef.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* in: in_h x in_w row-major; w: fh x fw row-major;
 * out: (in_h-fh+1) x (in_w-fw+1) row-major FP64.  Returns 0, or -1 on bad sizes. */
int oracle_xcorr2d_f64(const float *in, int64_t in_h, int64_t in_w,
                       const float *w, int64_t fh, int64_t fw,
                       double *out, int nthreads)
{
    if (fh < 1 || fw < 1 || in_h < fh || in_w < fw)
        return -1;
    const int64_t oh = in_h - fh + 1, ow = in_w - fw + 1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t y = 0; y < oh; ++y) {
        for (int64_t x = 0; x < ow; ++x) {
            double s = 0.0;
            for (int64_t i = 0; i < fh; ++i)
                for (int64_t j = 0; j < fw; ++j)
                    s += (double)in[(y + i) * in_w + (x + j)] * (double)w[i * fw + j];
            out[y * ow + x] = s;
        }
    }
    return 0;
}

/* x: [n][h][w][c_in]; wt: [c_out][fh][fw][c_in]; out: [n][oh][ow][c_out]
 * with oh = h + 2*ph - fh + 1, ow = w + 2*pw - fw + 1 (stride 1). */
int oracle_conv_nhwc_f64(const float *x, int64_t n, int64_t h, int64_t w, int64_t c_in,
                         const float *wt, int64_t c_out, int64_t fh, int64_t fw,
                         int64_t ph, int64_t pw, double *out, int nthreads)
{
    if (n < 0 || c_in < 1 || c_out < 1 || fh < 1 || fw < 1 || ph < 0 || pw < 0)
        return -1;
    const int64_t oh = h + 2 * ph - fh + 1, ow = w + 2 * pw - fw + 1;
    if (oh < 1 || ow < 1)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for collapse(2) schedule(static)
#endif
    for (int64_t b = 0; b < n; ++b) {
        for (int64_t y = 0; y < oh; ++y) {
            for (int64_t xo = 0; xo < ow; ++xo) {
                for (int64_t co = 0; co < c_out; ++co) {
                    double s = 0.0;
                    for (int64_t r = 0; r < fh; ++r) {
                        const int64_t yi = y + r - ph;
                        if (yi < 0 || yi >= h)
                            continue;
                        for (int64_t q = 0; q < fw; ++q) {
                            const int64_t xi = xo + q - pw;
                            if (xi < 0 || xi >= w)
                                continue;
                            const float *px = x + ((b * h + yi) * w + xi) * c_in;
                            const float *pk = wt + ((co * fh + r) * fw + q) * c_in;
                            for (int64_t ci = 0; ci < c_in; ++ci)
                                s += (double)px[ci] * (double)pk[ci];
                        }
                    }
                    out[((b * oh + y) * ow + xo) * c_out + co] = s;
                }
            }
        }
    }
    return 0;
}

/* The same definition at selected output pixels only: pts holds n_pts
 * (b, y, x) triples; out receives c_out values per pixel, [n_pts][c_out].
 * For checking outputs too large to compute whole on the CPU. */
int oracle_conv_nhwc_points_f64(const float *x, int64_t n, int64_t h, int64_t w, int64_t c_in,
                                const float *wt, int64_t c_out, int64_t fh, int64_t fw,
                                int64_t ph, int64_t pw, const int64_t *pts, int64_t n_pts,
                                double *out, int nthreads)
{
    if (n < 1 || c_in < 1 || c_out < 1 || fh < 1 || fw < 1 || ph < 0 || pw < 0 || n_pts < 0)
        return -1;
    const int64_t oh = h + 2 * ph - fh + 1, ow = w + 2 * pw - fw + 1;
    for (int64_t k = 0; k < n_pts; ++k)
        if (pts[3 * k] < 0 || pts[3 * k] >= n || pts[3 * k + 1] < 0 || pts[3 * k + 1] >= oh ||
            pts[3 * k + 2] < 0 || pts[3 * k + 2] >= ow)
            return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t k = 0; k < n_pts; ++k) {
        const int64_t b = pts[3 * k], y = pts[3 * k + 1], xo = pts[3 * k + 2];
        for (int64_t co = 0; co < c_out; ++co) {
            double s = 0.0;
            for (int64_t r = 0; r < fh; ++r) {
                const int64_t yi = y + r - ph;
                if (yi < 0 || yi >= h)
                    continue;
                for (int64_t q = 0; q < fw; ++q) {
                    const int64_t xi = xo + q - pw;
                    if (xi < 0 || xi >= w)
                        continue;
                    const float *px = x + ((b * h + yi) * w + xi) * c_in;
                    const float *pk = wt + ((co * fh + r) * fw + q) * c_in;
                    for (int64_t ci = 0; ci < c_in; ++ci)
                        s += (double)px[ci] * (double)pk[ci];
                }
            }
            out[k * c_out + co] = s;
        }
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
