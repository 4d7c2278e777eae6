// colsolve_column.hpp -- the solve of one response column by one wavefront
// (Algorithm 1 in covariance form with a working set; see colsolve.hip for
// the design): the first solve, the resume of a column the KKT pass
// flagged, and the hand-over of a column that outgrows its tier.  Shared by
// the column-solve kernels and the kernel that re-solves and polishes the
// flagged columns of the mixed form in one launch.
#pragma once
#include "colsolve_dev.hpp"

namespace spmesl {

// Returns true when the column's state was stored as final for this tier
// (false: handed to the next tier, or a wave that does not write).
template <typename T, int LW, int KCH, int KU, bool FIRST = false, bool DIRECT = true>
__device__ bool solve_column(const ColArgs<T> &A, WaveSm<T, LW> &sm, int64_t k, int tier, int part = 0,
                             int nparts = 1, KktCoop *cp = nullptr);

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
__device__ __forceinline__ bool solve_column(const ColArgs<T> &A, WaveSm<T, LW> &sm, int64_t k, int tier,
                                             int part, int nparts, KktCoop *cp)
{
    const int lane = lane_id();
    const bool writer = part == 0;  // the wave that writes the column's results
    // a first solve marks its column handed over (2) until it stores it final
    // (0); the row-tiled KKT pass marks the columns it flags (1)
    if (A.mark && A.mode == 0 && writer && lane == 0) A.mark[k] = *A.flags ? 0 : 2;
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
        return writer;
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
                return false;
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
            return false;
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
                return false;
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
                return false;
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
            return false;
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
    if (!writer) return false;
    store_column(A, k, sm, st, deferred ? (int)kColDeferred : status, true);
    if (lane == 0) {
        // deferred: the row-tiled pass appends to these lists; error: the
        // band list may predate the final support, so drop it
        if (deferred || status != kColOk) {
            A.pend_cnt[k] = 0;
            if (A.band_cnt) A.band_cnt[k] = 0;
        }
        record_info(A, k, cnt, rounds);
        if (A.mark && A.mode == 0) A.mark[k] = 0;
    }
    return true;
}

} // namespace spmesl
