// colsolve.hip -- the p scaled-lasso regressions of SPMESL, one wavefront
// per response column k.
//
// What is computed (Eq. (eq:spmesl) with beta_kk = 0): Algorithm 1 of the
// paper on response x_k, in covariance form.  With standardised data the
// gradient of the lasso step is g_j = x_j^T (x_k - X beta)/n = s_jk -
// sum_l S_jl beta_l, the coordinate update of Section 3.1 is
//     a_j = g_j + beta_j,  beta_j <- Soft_lambda(a_j),  g <- g - S_{:,j} delta_j
// (S_jj = 1), and the noise update of Eq. (eq:sigma) is
//     sigma^2 = ||x_k - X beta||^2 / n = 1 - beta^T (s_k + g).
//
// How (design for gfx950, not the paper's GPU design):
//   * Working set.  Coordinates outside a working set W stay at zero; a
//     KKT pass over all p coordinates finds every j outside W with
//     |g_j| > lambda + tol and adds it; the column is done when a pass finds
//     none.  Coordinates outside W would not move in a cyclic sweep anyway,
//     so the fixed point is Algorithm 1's.
//   * Inside W the cyclic sweep keeps the paper's ascending order, but the
//     wave evaluates every remaining coordinate of the sweep at once and
//     jumps to the first one whose soft-threshold changes it; coordinates it
//     skips have delta = 0 under the current gradient, which only changes at
//     a nonzero delta.  A sweep costs (nonzero updates + 1) wave steps.
//   * S restricted to W lives in LDS; one lane owns one coordinate of W.
//   * The outer loop is Algorithm 1's: lambda = sigma lambda0, sweeps until
//     the largest change is < tol, then sigma; stop when |d sigma| < tol.
//
// Phases of one solve:
//   fresh  : screen (the KKT pass at beta = 0 reads row k of S only), first
//            working-set solve; with defer_kkt the column stops there and the
//            row-tiled pass of kkt.hip checks every column reading S once;
//   resume : columns that pass flagged (or that outgrew 32 coordinates) take
//            their violators from the pending list, re-solve, and finish with
//            in-wave KKT passes (rows of S streamed per column).
// Two tiers: 32-coordinate working sets (four columns per workgroup) and
// 128-coordinate ones (one per workgroup).  Beyond 128 the column goes to
// the dense tier (dense.hip), which has no bound on the working set.
#include "colsolve_column.hpp"

namespace spmesl {


// KCH, KU: groups per lane in flight and support rows per step in the
// in-wave KKT passes.  NW > 1 (the re-solves of flagged columns): when the
// flagged columns fit one per block, the block's waves work on one column
// together.  Each wave runs the column's solve itself (same inputs, same
// instructions, so the same path and values in every wave), the KKT passes
// are split over the waves by ranges of j, and only the first wave writes
// the column's results.  FIRST: the first solves when the row-tiled KKT pass
// follows (each column is left deferred after one working-set solve), with
// none of the other paths compiled in; the rare column with more candidates
// than its list holds is handed to the wide kernel, which screens in the wave.
// The closed-form step of slow inner loops (direct_fixed_point) is compiled
// into the first solves and the re-solves, not into the first solves with
// in-wave KKT passes (large p), where its registers would halve the waves per
// SIMD.
template <typename T, int LW, int NW, int KCH, int KU, int MINW = 1, bool FIRST = false>
__global__ __launch_bounds__(kWave *NW) __attribute__((amdgpu_waves_per_eu(MINW))) void k_colsolve(ColArgs<T> A, int tier)
{
    static_assert(NW <= kCoopMax, "waves sharing a KKT pass");
    __shared__ WaveSm<T, LW> smem[NW];
    const int wv = threadIdx.x / kWave;
    WaveSm<T, LW> &sm = smem[wv];
    const int64_t nwork = A.mode ? (int64_t)*A.work_cnt : A.p - A.k0;
    constexpr bool DIRECT = FIRST || NW > 1;
    if constexpr (NW > 1) {
        if (A.mode && nwork <= (int64_t)gridDim.x) {
            __shared__ KktCoop coop;
            for (int64_t gw = blockIdx.x; gw < nwork; gw += gridDim.x)
                solve_column<T, LW, KCH, KU, false, DIRECT>(A, sm, (int64_t)A.work_list[gw], tier, wv, NW, &coop);
            return;
        }
    }
    const int64_t gw0 = (int64_t)blockIdx.x * NW + wv;
    for (int64_t gw = gw0; gw < nwork; gw += (int64_t)gridDim.x * NW) {
        const int64_t k = A.mode ? (int64_t)A.work_list[gw] : A.k0 + gw;
        solve_column<T, LW, KCH, KU, FIRST, DIRECT>(A, sm, k, tier);
    }
}

template <typename T>
void launch_colsolve(const ColArgs<T> &a, int tier, hipStream_t s)
{
    if (tier == 0 && a.mode) {
        // re-solves of flagged columns: 512 blocks of four waves.  Up to 512
        // columns (the usual case) get a block each and share its waves in
        // their KKT passes, which stream rows of S and are bound by the bytes
        // one wave can hold in flight; more columns take one wave each.
        hipLaunchKernelGGL((k_colsolve<T, 32, 4, 4, 4>), dim3(512), dim3(kWave * 4), 0, s, a, 0);
    } else if (tier == 0 && a.defer_kkt && a.screened) {
        // first solves: one column per workgroup, so a column's slot frees as
        // soon as it is done
        hipLaunchKernelGGL((k_colsolve<T, 32, 1, 4, 2, 1, true>), dim3((unsigned)(a.p - a.k0)), dim3(kWave), 0,
                           s, a, 0);
    } else if (tier == 0) {
        // first solves with in-wave KKT passes; float: three waves per SIMD
        // to hide the load latency
        hipLaunchKernelGGL((k_colsolve<T, 32, 1, 4, 2, sizeof(T) == 4 ? 3 : 1>), dim3((unsigned)(a.p - a.k0)),
                           dim3(kWave), 0, s, a, 0);
    } else {
        // the (short) escalation queue, one column per block.  Float: two
        // waves per block share each column's in-wave KKT passes, which
        // stream (|supp| + 1) rows of S and dominate these columns at large
        // p (two 128-coordinate working sets fit the LDS of a block; double
        // ones do not)
        unsigned blocks = (unsigned)(a.p < 256 ? a.p : 256);
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((k_colsolve<T, kWMax, 2, 4, 2>), dim3(blocks), dim3(kWave * 2), 0, s, a, 1);
        else
            hipLaunchKernelGGL((k_colsolve<T, kWMax, 1, 4, 2>), dim3(blocks), dim3(kWave), 0, s, a, 1);
    }
}

// The first solves of many problems in one launch: block b solves column
// k0 + b - off[d] of problem d (the row-tiled pass follows, as in the
// single-problem first solves).
template <typename T>
__global__ __launch_bounds__(kWave) void k_colsolve_first_grouped(const ColArgs<T> *__restrict__ tab,
                                                                  const int64_t *__restrict__ off, int nd)
{
    __shared__ WaveSm<T, 32> sm;
    const int64_t g = blockIdx.x;
    const int d = group_of(off, nd, g);
    const ColArgs<T> &A = tab[d];
    solve_column<T, 32, 4, 2, true, true>(A, sm, A.k0 + (g - off[d]), 0);
}

// The list-driven solves of many problems: item g is entry g - off[d] of
// problem d's work list; one wave per column (no shared KKT passes).
template <typename T, int LW, int NW, int KCH, int KU>
__global__ __launch_bounds__(kWave *NW) void k_colsolve_list_grouped(const ColArgs<T> *__restrict__ tab,
                                                                     const int64_t *__restrict__ off, int nd,
                                                                     int tier)
{
    __shared__ WaveSm<T, LW> smem[NW];
    const int wv = threadIdx.x / kWave;
    const int64_t total = off[nd];
    for (int64_t g = (int64_t)blockIdx.x * NW + wv; g < total; g += (int64_t)gridDim.x * NW) {
        const int d = group_of(off, nd, g);
        const ColArgs<T> &A = tab[d];
        solve_column<T, LW, KCH, KU, false, (NW > 1)>(A, smem[wv], (int64_t)A.work_list[g - off[d]], tier);
    }
}

template <typename T>
void launch_colsolve_first_grouped(const ColArgs<T> *tab, const int64_t *off, int nd, int64_t total,
                                   hipStream_t s)
{
    if (total <= 0) return;
    hipLaunchKernelGGL((k_colsolve_first_grouped<T>), dim3((unsigned)total), dim3(kWave), 0, s, tab, off, nd);
}

template <typename T>
void launch_colsolve_list_grouped(const ColArgs<T> *tab, const int64_t *off, int nd, int tier, hipStream_t s)
{
    if (tier == 0) {
        hipLaunchKernelGGL((k_colsolve_list_grouped<T, 32, 4, 4, 4>), dim3(512), dim3(kWave * 4), 0, s, tab, off,
                           nd, 0);
    } else if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((k_colsolve_list_grouped<T, kWMax, 2, 4, 2>), dim3(256), dim3(kWave * 2), 0, s, tab,
                           off, nd, 1);
    } else {
        hipLaunchKernelGGL((k_colsolve_list_grouped<T, kWMax, 1, 4, 2>), dim3(256), dim3(kWave), 0, s, tab, off,
                           nd, 1);
    }
}

template void launch_colsolve_first_grouped<double>(const ColArgs<double> *, const int64_t *, int, int64_t,
                                                    hipStream_t);
template void launch_colsolve_first_grouped<float>(const ColArgs<float> *, const int64_t *, int, int64_t,
                                                   hipStream_t);
template void launch_colsolve_list_grouped<double>(const ColArgs<double> *, const int64_t *, int, int, hipStream_t);
template void launch_colsolve_list_grouped<float>(const ColArgs<float> *, const int64_t *, int, int, hipStream_t);

template void launch_colsolve<double>(const ColArgs<double> &, int, hipStream_t);
template void launch_colsolve<float>(const ColArgs<float> &, int, hipStream_t);

} // namespace spmesl
