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
//     KKT pass over all p coordinates (a streamed read of row k of S and of
//     the rows of the current support) finds every j outside W with
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
// Two tiers: a 32-coordinate working set with four columns per workgroup,
// and a 128-coordinate one (one column per workgroup) that resumes columns
// the first tier hands over.  Beyond 128 the column reports SPMESL_EWORKSET.
#include "colsolve_dev.hpp"

namespace spmesl {

template <typename T, int LW>
__device__ void solve_column(const ColArgs<T> &A, WaveSm<T, LW> &sm, int64_t k);

template <typename T, int LW, int NW>
__global__ __launch_bounds__(kWave *NW) void k_colsolve(ColArgs<T> A)
{
    __shared__ WaveSm<T, LW> smem[NW];
    const int wv = threadIdx.x / kWave;
    WaveSm<T, LW> &sm = smem[wv];
    const int64_t gw0 = (int64_t)blockIdx.x * NW + wv;
    // tier 2 walks the escalation queue with a small grid
    const int64_t nwork = A.resume ? (int64_t)*A.esc_cnt : A.p;
    for (int64_t gw = gw0; gw < nwork; gw += (int64_t)gridDim.x * NW) {
        const int64_t k = A.resume ? (int64_t)A.esc_list[gw] : gw;
        solve_column<T, LW>(A, sm, k);
    }
}

template <typename T, int LW>
__device__ void solve_column(const ColArgs<T> &A, WaveSm<T, LW> &sm, int64_t k)
{
    const int lane = lane_id();
    if (*A.flags) {
        // bad input: leave an empty, well-formed list for every consumer
        if (lane == 0) {
            A.w_cnt[k] = 0;
            A.sigma[k] = 1.0;
            A.lam_used[k] = (double)A.lambda0;
            A.col_status[k] = kColOk;
            if (A.band_cnt) A.band_cnt[k] = 0;
        }
        return;
    }
    const int64_t p = A.p;
    ColState<T, LW> st;
    SolveCounts cnt = {0, 0, 0};
    int rounds = 0, status = kColOk, maxw = 0;
    if (A.resume) {
        st.w = A.w_cnt[k];
        for (int q = lane; q < st.w; q += kWave) {
            sm.widx[q] = A.w_idx[k * kWMax + q];
            sm.wbeta[q] = A.w_beta[k * kWMax + q];
        }
        st.sigma = (T)A.sigma[k];
        st.lam_used = (T)A.lam_used[k];
        wave_sync();
        load_working_set(A.S, p, k, sm, st);
    } else {
        st.w = 0;
        st.sigma = T(1);
        st.lam_used = A.lambda0;
#pragma unroll
        for (int s = 0; s < ColState<T, LW>::NS; ++s) st.g[s] = st.b[s] = st.sv[s] = T(0);
    }
    const bool band = A.band > T(0);
    for (;;) {
        int ns = build_support(sm, st);
        int npend = kkt_pass(A.S, p, k, sm, st.w, ns, st.lam_used + A.kkt_tol, band,
                             st.lam_used - A.band, A.band_cnt, A.band_idx);
        if (npend == 0) break;
        if (rounds >= A.max_rounds) {
            status = kColNoconv;
            break;
        }
        ++rounds;
        int np = npend < kPendMax ? npend : kPendMax;
        if (st.w + np > LW) {
            if (LW < kWMax && !A.resume) {
                // hand the column to the wider tier from its current state
                store_column(A, k, sm, st, kColOk);
                if (lane == 0) {
                    int pos = atomicAdd(A.esc_cnt, 1);
                    A.esc_list[pos] = (int)k;
                    atomicAdd(&A.counters[kCntEscalated], 1ull);
                }
                return;
            }
            np = LW - st.w;
            if (np <= 0) {
                status = kColWorkset;
                break;
            }
        }
        merge_pending(sm, st, np);
        maxw = st.w > maxw ? st.w : maxw;
        load_working_set(A.S, p, k, sm, st);
        status = scaled_lasso_W(sm, st, A.lambda0, A.tol, A.max_outer, A.max_sweeps, cnt);
        if (status != kColOk) break;
    }
    store_column(A, k, sm, st, status);
    if (lane == 0) {
        atomicAdd(&A.counters[kCntOuter], (unsigned long long)cnt.outer);
        atomicAdd(&A.counters[kCntSweeps], (unsigned long long)cnt.sweeps);
        atomicAdd(&A.counters[kCntUpdates], (unsigned long long)cnt.updates);
        atomicAdd(&A.counters[kCntRounds], (unsigned long long)rounds);
        atomicMax(&A.counters[kCntMaxW], (unsigned long long)maxw);
        atomicMax(&A.counters[kCntMaxOuter], (unsigned long long)cnt.outer);
        if (status != kColOk) {
            atomicAdd(&A.counters[kCntNoconv], 1ull);
            atomicOr(A.status_bits, status == kColWorkset ? 4 : (status == kColDegenerate ? 2 : 1));
        }
    }
}

template <typename T>
void launch_colsolve(const ColArgs<T> &a, hipStream_t s)
{
    if (!a.resume) {
        constexpr int NW = 4;
        unsigned blocks = (unsigned)((a.p + NW - 1) / NW);
        hipLaunchKernelGGL((k_colsolve<T, 32, NW>), dim3(blocks), dim3(kWave * NW), 0, s, a);
    } else {
        // one wave per block walking the (short) escalation queue
        unsigned blocks = (unsigned)(a.p < 256 ? a.p : 256);
        hipLaunchKernelGGL((k_colsolve<T, kWMax, 1>), dim3(blocks), dim3(kWave), 0, s, a);
    }
}

template void launch_colsolve<double>(const ColArgs<double> &, hipStream_t);
template void launch_colsolve<float>(const ColArgs<float> &, hipStream_t);

} // namespace spmesl
