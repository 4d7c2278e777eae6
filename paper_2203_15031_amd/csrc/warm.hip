// warm.hip -- the stored column state of a warm start.
//
// Algorithm 1 starts each regression from beta = 0, sigma = 1; a caller may
// instead start it from earlier coefficients and noise levels (a previous
// solve at another penalty, or one stopped by an iteration cap).  The
// minimiser of Eq. (eq:spmesl) is unique, so the start changes the work,
// not the result.  This kernel turns a dense B0 (p x p, row-major, column k
// the coefficients of response k) into the per-column working sets the
// column solves resume from.
//
// A block owns 64 consecutive columns (one lane each) and splits the rows
// of B0 over its 16 waves in contiguous ranges, so every load is a coalesced
// row segment.  Two passes over the block's column strip: the first counts
// each wave's nonzeros per column, the second writes them at the offsets of
// an exclusive scan over the waves, so each column's list is in ascending
// row order (the order the solver keeps its working sets in).
#include "common.hpp"

namespace spmesl {

constexpr int kWarmWaves = 16;

template <typename T>
__global__ __launch_bounds__(kWave *kWarmWaves) void k_warm_start(
    const double *__restrict__ B0, const double *__restrict__ sigma0, int64_t p,
    const double *__restrict__ scale, int original, double lambda0, int *__restrict__ w_cnt,
    int *__restrict__ w_idx, T *__restrict__ w_beta, double *__restrict__ sigma,
    double *__restrict__ lam_used, int *__restrict__ col_status)
{
    __shared__ int cnt[kWarmWaves][kWave];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t k = (int64_t)blockIdx.x * kWave + lane;
    const bool col = k < p;
    const int64_t rows = (p + kWarmWaves - 1) / kWarmWaves;
    const int64_t j0 = (int64_t)wv * rows;
    const int64_t j1 = j0 + rows < p ? j0 + rows : p;
    const double ck = col ? scale[k] : 1.0;
    // the value stored for (j, k), or 0 when (j, k) is not kept
    auto value = [&](int64_t j, double b) -> T {
        if (j == k || b == 0.0) return T(0);
        const double v = original ? b * ck / scale[j] : b;
        return (T)v;
    };
    int c = 0;
    if (B0 && col)
        for (int64_t j = j0; j < j1; ++j) c += value(j, B0[j * p + k]) != T(0);
    cnt[wv][lane] = c;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kWarmWaves; ++w) {
        off += w < wv ? cnt[w][lane] : 0;
        tot += cnt[w][lane];
    }
    if (B0 && col && off < kWMax)
        for (int64_t j = j0; j < j1 && off < kWMax; ++j) {
            const T v = value(j, B0[j * p + k]);
            if (v != T(0)) {
                w_idx[k * kWMax + off] = (int)j;
                w_beta[k * kWMax + off] = v;
                ++off;
            }
        }
    if (wv == 0 && col) {
        double sg = 1.0;
        if (sigma0) {
            const double v = original ? sigma0[k] * ck : sigma0[k];
            if (v > 0.0 && v < 1e300) sg = v;
        }
        w_cnt[k] = tot < kWMax ? tot : kWMax;
        sigma[k] = sg;
        lam_used[k] = sg * lambda0;
        col_status[k] = kColWarm;
    }
}

template <typename T>
void launch_warm_start(const double *B0, const double *sigma0, int64_t p, const double *scale, int original,
                       double lambda0, int *w_cnt, int *w_idx, T *w_beta, double *sigma, double *lam_used,
                       int *col_status, hipStream_t s)
{
    const unsigned blocks = (unsigned)((p + kWave - 1) / kWave);
    hipLaunchKernelGGL(k_warm_start<T>, dim3(blocks), dim3(kWave * kWarmWaves), 0, s, B0, sigma0, p, scale,
                       original, lambda0, w_cnt, w_idx, w_beta, sigma, lam_used, col_status);
}

template void launch_warm_start<double>(const double *, const double *, int64_t, const double *, int, double,
                                        int *, int *, double *, double *, double *, int *, hipStream_t);
template void launch_warm_start<float>(const double *, const double *, int64_t, const double *, int, double,
                                       int *, int *, float *, double *, double *, int *, hipStream_t);

} // namespace spmesl
