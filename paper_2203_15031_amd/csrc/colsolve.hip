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
#include "colsolve_dev.hpp"

namespace spmesl {

template <typename T, int LW, int KCH, int KU, bool FIRST = false, bool DIRECT = true>
__device__ void solve_column(const ColArgs<T> &A, WaveSm<T, LW> &sm, int64_t k, int tier, int part = 0,
                             int nparts = 1, KktCoop *cp = nullptr);

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

// per-column counters: set by the first solve, accumulated by later phases
template <typename T>
__device__ void record_info(const ColArgs<T> &A, int64_t k, const SolveCounts &cnt, int rounds)
{
    int *ci = A.colinfo + k * 4;
    if (A.mode == 0) {
        ci[0] = cnt.outer;
        ci[1] = cnt.sweeps;
        ci[2] = cnt.updates;
        ci[3] = rounds;
    } else {
        ci[0] += cnt.outer;
        ci[1] += cnt.sweeps;
        ci[2] += cnt.updates;
        ci[3] += rounds;
    }
}

// Hand column k to the next tier: its state (W, beta, sigma) and its np
// pending candidates are stored, and k joins the 128-coordinate tier's queue
// (from the 32-coordinate tier) or the dense tier's (from the 128 one, with
// the status kColDenseQ; in the mixed form the double polish hands such a
// column to the dense tier in double, so the float stage has no dense tier).
// `unsolved`: the stored state is a warm start no solve has run on yet (the
// wide kernel then solves it even with no pending candidates)
template <typename T, int LW>
__device__ __forceinline__ void escalate(const ColArgs<T> &A, int64_t k, const WaveSm<T, LW> &sm,
                         const ColState<T, LW> &st, int np, const SolveCounts &cnt, int rounds,
                         bool unsolved = false)
{
    const int lane = lane_id();
    const bool dense = LW >= kWMax;
    store_column(A, k, sm, st, dense ? (int)kColDenseQ : (unsolved ? (int)kColWarm : (int)kColOk), false);
    if (lane == 0) record_info(A, k, cnt, rounds);
    for (int i = lane; i < np; i += kWave) A.pend_idx[k * kPendMax + i] = sm.pend[i];
    if (lane == 0) {
        A.pend_cnt[k] = np;
        int pos = atomicAdd(dense ? A.dense_cnt : A.esc_cnt, 1);
        (dense ? A.dense_list : A.esc_list)[pos] = (int)k;
        atomicAdd(&A.counters[kCntEscalated], 1ull);
    }
}

template <typename T, int LW, int KCH, int KU, bool FIRST, bool DIRECT>
__device__ __forceinline__ void solve_column(const ColArgs<T> &A, WaveSm<T, LW> &sm, int64_t k, int tier,
                                             int part, int nparts, KktCoop *cp)
{
    const int lane = lane_id();
    const bool writer = part == 0;  // the wave that writes the column's results
    if (*A.flags) {
        // bad input: leave an empty, well-formed column for every consumer
        if (writer && lane == 0) {
            A.w_cnt[k] = 0;
            A.supp_cnt[k] = 0;
            A.pend_cnt[k] = 0;
            A.colinfo[k * 4 + 0] = A.colinfo[k * 4 + 1] = 0;
            A.colinfo[k * 4 + 2] = A.colinfo[k * 4 + 3] = 0;
            A.sigma[k] = 1.0;
            A.lam_used[k] = (double)A.lambda0;
            A.col_status[k] = kColOk;
            if (A.band_cnt) A.band_cnt[k] = 0;
        }
        return;
    }
    const int64_t p = A.p;
    const bool band = A.band > T(0);
    ColState<T, LW> st;
    unsigned rlo[ColState<T, LW>::kRows], rhi[ColState<T, LW>::kRowsHi];
    SolveCounts cnt = {0, 0, 0};
    int rounds = 0, status = kColOk;
    bool deferred = false;

    if (FIRST || A.mode == 0) {
        st.w = 0;
        st.sigma = T(1);
        st.lam_used = A.lambda0;
#pragma unroll
        for (int s = 0; s < ColState<T, LW>::NS; ++s) st.g[s] = st.b[s] = st.sv[s] = T(0);
        // the count and (speculatively: the list holds kPendMax = 64 slots
        // per column) the candidates, in one round of loads
        int nc = A.screened ? A.pend_cnt[k] : -1;
        const int cfirst = A.screened ? A.pend_idx[k * kPendMax + lane] : 0;
        if (A.warm) {
            // a warm start: W, beta and sigma from the stored state (the
            // screen's candidates are merged into W below)
            const int wc = A.w_cnt[k];
            if (wc > LW) {
                // more than this tier holds: the wide kernel resumes the
                // stored state, with the screen (when its list holds it) as
                // the pending candidates; its in-wave KKT passes find the rest
                if (writer && lane == 0) {
                    if (!(nc >= 0 && nc <= kPendMax)) A.pend_cnt[k] = 0;
                    A.colinfo[k * 4 + 0] = A.colinfo[k * 4 + 1] = 0;
                    A.colinfo[k * 4 + 2] = A.colinfo[k * 4 + 3] = 0;
                    int pos = atomicAdd(A.esc_cnt, 1);
                    A.esc_list[pos] = (int)k;
                    atomicAdd(&A.counters[kCntEscalated], 1ull);
                }
                return;
            }
            for (int q = lane; q < wc; q += kWave) {
                sm.widx[q] = A.w_idx[k * kWMax + q];
                sm.wbeta[q] = A.w_beta[k * kWMax + q];
            }
            st.w = wc;
#pragma unroll
            for (int s = 0; s < ColState<T, LW>::NS; ++s) {
                int q = s * kWave + lane;
                st.b[s] = q < wc ? A.w_beta[k * kWMax + q] : T(0);
            }
            st.sigma = (T)A.sigma[k];
            st.lam_used = (T)A.lam_used[k];
            wave_sync();
        }
        if (FIRST && !(nc >= 0 && nc <= kPendMax)) {
            // too many candidates for the list: the wide kernel screens in
            // the wave (resumed from W = {}, or the warm start, with no
            // pending candidates)
            if (writer) escalate(A, k, sm, st, 0, cnt, rounds, A.warm != 0);
            return;
        } else if (nc > kPendMax) {
            // too many candidates for the list: screen in the wave below
            wave_sync();
            if (writer && lane == 0) A.pend_cnt[k] = 0;
        } else if (nc >= 0) {
            // the screen taken with S: W = its candidates (those that are
            // predictors: j < pv)
            const bool keep = lane < nc && cfirst < A.pv;
            const unsigned long long km = __ballot(keep);
            if (keep) sm.pend[lanes_below(km)] = cfirst;
            nc = (int)__popcll(km);
            wave_sync();
            if (writer && lane == 0) A.pend_cnt[k] = 0;
            int np = nc > 0 ? sort_unique_small(sm.pend, nc) : 0;
            if (st.w + np > LW) {
                if (writer) escalate(A, k, sm, st, np, cnt, rounds, A.warm != 0);
                return;
            }
            if (np > 0 || st.w > 0) {
                ++rounds;
                if (np > 0) merge_pending(sm, st, np);
                load_working_set(A.S, p, k, sm, st, rlo, rhi);
                status = scaled_lasso_W<T, LW, DIRECT>(sm, st, rlo, rhi, A.lambda0, A.tol, A.max_outer, A.max_sweeps, cnt);
                if (A.defer_kkt && status == kColOk) deferred = true;
            } else if (A.defer_kkt) {
                // beta = 0 passes the screen; the row-tiled pass still
                // records the column's near-threshold band (mixed form)
                deferred = true;
            }
        }
    } else if constexpr (!FIRST) {
        st.w = A.w_cnt[k];
        st.w = st.w < 0 ? 0 : (st.w > LW ? LW : st.w);
        for (int q = lane; q < st.w; q += kWave) {
            sm.widx[q] = A.w_idx[k * kWMax + q];
            sm.wbeta[q] = A.w_beta[k * kWMax + q];
        }
#pragma unroll
        for (int s = 0; s < ColState<T, LW>::NS; ++s) {
            int q = s * kWave + lane;
            st.b[s] = q < st.w ? A.w_beta[k * kWMax + q] : T(0);
            st.g[s] = st.sv[s] = T(0);
        }
        st.sigma = (T)A.sigma[k];
        st.lam_used = (T)A.lam_used[k];
        // a warm start handed over unsolved (read with the rest of the state)
        const bool unsolved = A.warm && A.col_status[k] == kColWarm;
        int np = A.pend_cnt[k];
        np = np < 0 ? 0 : (np > kPendMax ? kPendMax : np);
        for (int i = lane; i < np; i += kWave) sm.pend[i] = A.pend_idx[k * kPendMax + i];
        wave_sync();
        // every wave of a shared column has read its state before the
        // first write to it (the barrier also completes those loads)
        if (cp) __syncthreads();
        if (writer && lane == 0) A.pend_cnt[k] = 0;
        if (np > 0) {
            np = sort_unique_small(sm.pend, np);
            if (st.w + np > LW) {
                if (writer) escalate(A, k, sm, st, np, cnt, rounds, unsolved);
                return;
            }
            ++rounds;
            merge_pending(sm, st, np);
            load_working_set(A.S, p, k, sm, st, rlo, rhi);
            status = scaled_lasso_W<T, LW, DIRECT>(sm, st, rlo, rhi, A.lambda0, A.tol, A.max_outer, A.max_sweeps, cnt);
        } else {
            load_working_set(A.S, p, k, sm, st, rlo, rhi);
            // a warm start handed over unsolved: solve it before the KKT passes
            if (unsolved)
                status = scaled_lasso_W<T, LW, DIRECT>(sm, st, rlo, rhi, A.lambda0, A.tol, A.max_outer, A.max_sweeps, cnt);
        }
    }

    while (!FIRST && status == kColOk && !deferred) {
        int ns = build_support(sm, st);
        int npend = kkt_pass<T, T, LW, KCH, KU>(A.S, p, A.pv, k, sm, st.w, ns, st.lam_used + A.kkt_tol, band,
                                                st.lam_used - A.band, A.band_cnt, A.band_idx, part,
                                                nparts, cp);
        if (npend == 0) break;
        if (rounds >= A.max_rounds) {
            status = kColNoconv;
            break;
        }
        int np = npend < kPendMax ? npend : kPendMax;
        if (st.w + np > LW) {
            if (writer) escalate(A, k, sm, st, np, cnt, rounds);
            return;
        }
        ++rounds;
        merge_pending(sm, st, np);
        load_working_set(A.S, p, k, sm, st, rlo, rhi);
        status = scaled_lasso_W<T, LW, DIRECT>(sm, st, rlo, rhi, A.lambda0, A.tol, A.max_outer, A.max_sweeps, cnt);
        if (A.mode == 0 && A.defer_kkt && status == kColOk) {
            deferred = true;
            break;
        }
    }
    if (!writer) return;
    store_column(A, k, sm, st, deferred ? (int)kColDeferred : status, true);
    if (lane == 0) {
        // deferred: the row-tiled pass appends to these lists; error: the
        // band list may predate the final support, so drop it
        if (deferred || status != kColOk) {
            A.pend_cnt[k] = 0;
            if (A.band_cnt) A.band_cnt[k] = 0;
        }
        record_info(A, k, cnt, rounds);
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
