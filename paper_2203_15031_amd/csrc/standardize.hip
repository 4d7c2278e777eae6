// standardize.hip -- centring and scaling of the data matrix.
//
// Section 2.2 of the paper assumes columns centred and scaled so that
// x_k^T x_k = n (s_kk = 1).  These kernels compute the column means and the
// scales c_k = (sum_i (x_ik - mean_k)^2 / n)^{-1/2} (the C of Proposition 1)
// and write the standardised data in the layout the covariance kernel of each
// precision reads.  All are single HBM passes over X.
#include "common.hpp"

namespace spmesl {

// Column sums about a shift (the column's first entry, which keeps the
// one-pass variance accurate): partial[(2r) * p + j] = sum (x - K_j),
// partial[(2r+1) * p + j] = sum (x - K_j)^2 over row chunk r.
__global__ __launch_bounds__(256) void k_colstats_partial(const double *__restrict__ X,
                                                          int64_t n, int64_t p, int64_t ldx,
                                                          int64_t rows_per,
                                                          double *__restrict__ partial)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (j >= p) return;
    double K = X[j];
    int64_t i0 = (int64_t)r * rows_per;
    int64_t i1 = i0 + rows_per < n ? i0 + rows_per : n;
    double s1 = 0.0, s2 = 0.0;
    int64_t i = i0;
    for (; i + 4 <= i1; i += 4) {
        double x0 = X[i * ldx + j], x1 = X[(i + 1) * ldx + j];
        double x2 = X[(i + 2) * ldx + j], x3 = X[(i + 3) * ldx + j];
        double d0 = x0 - K, d1 = x1 - K, d2 = x2 - K, d3 = x3 - K;
        s1 += d0;
        s2 += d0 * d0;
        s1 += d1;
        s2 += d1 * d1;
        s1 += d2;
        s2 += d2 * d2;
        s1 += d3;
        s2 += d3 * d3;
    }
    for (; i < i1; ++i) {
        double d = X[i * ldx + j] - K;
        s1 += d;
        s2 += d * d;
    }
    partial[(2 * (int64_t)r) * p + j] = s1;
    partial[(2 * (int64_t)r + 1) * p + j] = s2;
}

// Combine the chunks in a fixed order; mean_j = K + s1/n,
// var_j = (s2 - s1^2/n)/n, scale_j = var_j^{-1/2}.
__global__ __launch_bounds__(256) void k_colstats_final(const double *__restrict__ X, int64_t n,
                                                        int64_t p, int rchunks,
                                                        const double *__restrict__ partial,
                                                        double *__restrict__ mean,
                                                        double *__restrict__ scale,
                                                        int *__restrict__ flags,
                                                        int *__restrict__ zero_cnt)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p) return;
    if (zero_cnt) zero_cnt[j] = 0;  // a per-column counter the covariance kernel appends to
    double s1 = 0.0, s2 = 0.0;
    // fixed summation order; loads issued eight chunks at a time
    for (int r0 = 0; r0 < rchunks; r0 += 8) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            int r = r0 + u;
            a[u] = r < rchunks ? partial[(2 * (int64_t)r) * p + j] : 0.0;
            b[u] = r < rchunks ? partial[(2 * (int64_t)r + 1) * p + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s1 += a[u];
            s2 += b[u];
        }
    }
    double K = X[j];
    double nn = (double)n;
    if (!isfinite(s1) || !isfinite(s2) || !isfinite(K)) {
        atomicOr(flags, 1);
        mean[j] = 0.0;
        scale[j] = 1.0;
        return;
    }
    double ss = s2 - s1 * s1 / nn;
    if (!(ss > 0.0)) {
        atomicOr(flags, 2);
        mean[j] = K;
        scale[j] = 1.0;
        return;
    }
    mean[j] = K + s1 / nn;
    scale[j] = 1.0 / sqrt(ss / nn);
}

int colstats_rchunks(int64_t n, int64_t p)
{
    // enough blocks to cover the machine, each thread summing >= 8 rows
    int64_t colblocks = (p + 255) / 256;
    int64_t want = (2048 + colblocks - 1) / colblocks;
    int64_t maxr = (n + 7) / 8;
    int64_t r = want < maxr ? want : maxr;
    if (r < 1) r = 1;
    if (r > 256) r = 256;
    return (int)r;
}

void launch_colstats(const double *X, int64_t n, int64_t p, int64_t ldx, double *partial,
                     int rchunks, double *mean, double *scale, int *flags, int *zero_cnt, hipStream_t s)
{
    int64_t rows_per = (n + rchunks - 1) / rchunks;
    dim3 g((unsigned)((p + 255) / 256), (unsigned)rchunks);
    hipLaunchKernelGGL(k_colstats_partial, g, dim3(256), 0, s, X, n, p, ldx, rows_per, partial);
    hipLaunchKernelGGL(k_colstats_final, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, s, X, n,
                       p, rchunks, partial, mean, scale, flags, zero_cnt);
}

template <typename T>
__global__ __launch_bounds__(256) void k_standardize(const double *__restrict__ X, int64_t n,
                                                     int64_t p, int64_t ldx,
                                                     const double *__restrict__ mean,
                                                     const double *__restrict__ scale,
                                                     T *__restrict__ Xs)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t i = blockIdx.y;
    if (j >= p) return;
    for (; i < n; i += gridDim.y) Xs[i * p + j] = (T)((X[i * ldx + j] - mean[j]) * scale[j]);
}

void launch_standardize_f64(const double *X, int64_t n, int64_t p, int64_t ldx,
                            const double *mean, const double *scale, double *Xs, hipStream_t s)
{
    unsigned gy = (unsigned)(n < 1024 ? n : 1024);
    hipLaunchKernelGGL(k_standardize<double>, dim3((unsigned)((p + 255) / 256), gy), dim3(256), 0,
                       s, X, n, p, ldx, mean, scale, Xs);
}

void launch_standardize_f32(const double *X, int64_t n, int64_t p, int64_t ldx,
                            const double *mean, const double *scale, float *Xs, hipStream_t s)
{
    unsigned gy = (unsigned)(n < 1024 ? n : 1024);
    hipLaunchKernelGGL(k_standardize<float>, dim3((unsigned)((p + 255) / 256), gy), dim3(256), 0,
                       s, X, n, p, ldx, mean, scale, Xs);
}

// round-to-nearest-even float -> bfloat16 bits (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Transposing standardisation for the mixed form.  Block: 64 (j) x 4 (i
// lanes); tile 64 samples x 64 variables staged through LDS so that both
// the read of X (rows) and the writes of Xt/hi/lo (variable-major) are
// coalesced.
__global__ __launch_bounds__(256) void k_standardize_split(
    const double *__restrict__ X, int64_t n, int64_t p, int64_t ldx,
    const double *__restrict__ mean, const double *__restrict__ scale, double *__restrict__ Xt,
    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int64_t npad)
{
    __shared__ double tile[64][65];
    int64_t i0 = (int64_t)blockIdx.x * 64;
    int64_t j0 = (int64_t)blockIdx.y * 64;
    int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    int64_t j = j0 + tx;
    double m = j < p ? mean[j] : 0.0, c = j < p ? scale[j] : 0.0;
    for (int r = ty; r < 64; r += 4) {
        int64_t i = i0 + r;
        tile[r][tx] = (i < n && j < p) ? (X[i * ldx + j] - m) * c : 0.0;
    }
    __syncthreads();
    // write: thread tx walks samples, ty walks variables
    for (int v = ty; v < 64; v += 4) {
        int64_t jj = j0 + v;
        int64_t ii = i0 + tx;
        if (jj >= p) continue;
        double x = tile[tx][v];
        if (ii < n) Xt[jj * n + ii] = x;
        if (ii < npad) {
            float f = (float)x;
            uint16_t h = bf16_bits(f);
            uint16_t l = bf16_bits(f - bf16_value(h));
            hi[jj * npad + ii] = ii < n ? h : (uint16_t)0;
            lo[jj * npad + ii] = ii < n ? l : (uint16_t)0;
        }
    }
}

// The mixed form's statistics and split in one pass over X.  A block owns a
// strip of SW variables over all n samples: the strip is read once into LDS
// (coalesced rows of SW doubles), the column means and centred sums of
// squares are taken from LDS in two passes in a fixed order, and the same
// block writes Xt and the bf16 split variable-major.  It also zeroes the
// strip's screen counters (the covariance kernel appends to them).
template <int SW>
__global__ __launch_bounds__(256) void k_stats_split(const double *__restrict__ X, int64_t n, int64_t p,
                                                     int64_t ldx, double *__restrict__ mean,
                                                     double *__restrict__ scale, double *__restrict__ Xt,
                                                     uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                     int64_t npad, int *__restrict__ flags,
                                                     int *__restrict__ zero_cnt)
{
    constexpr int SWP = SW + 1;         // odd row stride: by-variable reads hit distinct banks
    constexpr int G = 256 / SW;         // row groups
    extern __shared__ double strip[];   // n x SWP
    __shared__ double part[G][SW];
    __shared__ double mv[SW], cv[SW];
    const int t = threadIdx.x;
    const int v = t % SW, g = t / SW;
    const int64_t j0 = (int64_t)blockIdx.x * SW;
    const int64_t j = j0 + v;
    for (int64_t i = g; i < n; i += G) strip[i * SWP + v] = j < p ? X[i * ldx + j] : 0.0;
    __syncthreads();
    double s1 = 0.0;
    for (int64_t i = g; i < n; i += G) s1 += strip[i * SWP + v];
    part[g][v] = s1;
    __syncthreads();
    if (t < SW) {
        double a = 0.0;
        for (int q = 0; q < G; ++q) a += part[q][t];
        mv[t] = a / (double)n;
    }
    __syncthreads();
    const double m = mv[v];
    double s2 = 0.0;
    for (int64_t i = g; i < n; i += G) {
        const double d = strip[i * SWP + v] - m;
        s2 += d * d;
    }
    __syncthreads();  // every thread has read mv and part before part is reused
    part[g][v] = s2;
    __syncthreads();
    if (t < SW) {
        double a = 0.0;
        for (int q = 0; q < G; ++q) a += part[q][t];
        const int64_t jj = j0 + t;
        const double mm = mv[t];
        double c;
        if (!isfinite(mm) || !isfinite(a)) {
            if (jj < p) atomicOr(flags, 1);
            mv[t] = 0.0;
            c = 1.0;
        } else if (!(a > 0.0)) {
            if (jj < p) atomicOr(flags, 2);
            c = 1.0;
        } else {
            c = 1.0 / sqrt(a / (double)n);
        }
        cv[t] = c;
        if (jj < p) {
            mean[jj] = mv[t];
            scale[jj] = c;
            if (zero_cnt) zero_cnt[jj] = 0;
        }
    }
    __syncthreads();
    for (int w = 0; w < SW; ++w) {
        const int64_t jj = j0 + w;
        if (jj >= p) break;
        const double mm = mv[w], cc = cv[w];
        for (int64_t i = t; i < npad; i += 256) {
            const double x = i < n ? (strip[i * SWP + w] - mm) * cc : 0.0;
            if (i < n) Xt[jj * n + i] = x;
            const float f = (float)x;
            const uint16_t h = bf16_bits(f);
            hi[jj * npad + i] = h;
            lo[jj * npad + i] = bf16_bits(f - bf16_value(h));
        }
    }
}

// Strip width for the fused kernel: 8 variables (64-byte row segments) when
// the LDS strip fits 64 KB, else 4; 0 when neither does.  At n = 400,
// p = 5000 the 8-wide strips (625 blocks, about five per CU) take 17 us where
// 16-wide ones (313 blocks, two per CU) took 23 us and 4-wide ones 20 us.
static int stats_split_width(int64_t n)
{
    for (int sw = 8; sw >= 4; sw >>= 1)
        if ((size_t)n * (sw + 1) * 8 <= (size_t)64 * 1024) return sw;
    return 0;
}

bool launch_stats_split(const double *X, int64_t n, int64_t p, int64_t ldx, double *mean,
                        double *scale, double *Xt, uint16_t *hi, uint16_t *lo, int64_t npad,
                        int *flags, int *zero_cnt, hipStream_t s)
{
    const int sw = stats_split_width(n);
    if (sw == 0) return false;
    const size_t lds = (size_t)n * (sw + 1) * 8;
    const unsigned blocks = (unsigned)((p + sw - 1) / sw);
    if (sw == 8)
        hipLaunchKernelGGL(k_stats_split<8>, dim3(blocks), dim3(256), lds, s, X, n, p, ldx, mean, scale,
                           Xt, hi, lo, npad, flags, zero_cnt);
    else
        hipLaunchKernelGGL(k_stats_split<4>, dim3(blocks), dim3(256), lds, s, X, n, p, ldx, mean, scale,
                           Xt, hi, lo, npad, flags, zero_cnt);
    return true;
}

void launch_standardize_split(const double *X, int64_t n, int64_t p, int64_t ldx,
                              const double *mean, const double *scale, double *Xt,
                              uint16_t *hi, uint16_t *lo, int64_t npad, hipStream_t s)
{
    dim3 g((unsigned)((npad + 63) / 64), (unsigned)((p + 63) / 64));
    hipLaunchKernelGGL(k_standardize_split, g, dim3(256), 0, s, X, n, p, ldx, mean, scale, Xt,
                       hi, lo, npad);
}

__global__ __launch_bounds__(256) void k_pack_columns(const double *__restrict__ X, int64_t n, int64_t p,
                                                      int64_t ldx, const double *__restrict__ Y, int64_t m,
                                                      int64_t ldy, double *__restrict__ Xa)
{
    const int64_t pa = p + m;
    const int64_t total = n * pa;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t i = e / pa, j = e - i * pa;
        Xa[e] = j < p ? X[i * ldx + j] : Y[i * ldy + (j - p)];
    }
}

void launch_pack_columns(const double *X, int64_t n, int64_t p, int64_t ldx, const double *Y, int64_t m,
                         int64_t ldy, double *Xa, hipStream_t s)
{
    int64_t blocks = (n * (p + m) + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pack_columns, dim3((unsigned)blocks), dim3(256), 0, s, X, n, p, ldx, Y, m, ldy, Xa);
}

} // namespace spmesl
