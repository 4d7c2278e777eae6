// kkt.hip -- one KKT pass over every column, reading S once.
//
// After each column's first working-set solve, the lasso optimality
// conditions of Eq. (eqn:lasso) must be checked for every coordinate j
// outside the working set: |g_jk| <= lambda_k (+ tol) with
//     g_jk = s_jk - sum_{l in supp(beta_k)} S_jl beta_lk.
// A wave per column would stream the rows of S of its support from HBM, so S
// is re-read once per support entry of every column.  Here a workgroup
// stages RJ rows of S in LDS instead (one HBM read of S in total), and each
// thread walks the columns: the supports are read slot-major (coalesced
// across threads) and the gathers S_jl hit LDS.  Violators go to the
// column's pending list and the column to the dirty list; in the mixed form
// the near-threshold band (j off the support with |g_jk| > lambda_k - band)
// is recorded for the double polish.  Only columns left deferred by their
// first solve are examined.
#include "common.hpp"

namespace spmesl {

int kkt_rows_per_block(int64_t p, size_t elem, size_t lds_budget)
{
    for (int rj = 8; rj >= 1; rj >>= 1)
        if ((size_t)rj * (size_t)p * elem <= lds_budget) return rj;
    return 0;
}

constexpr int kKktThreads = 512;
constexpr int kKktQ = kSuppPad;  // support entries preloaded per column

// Rare path for one flagged pair (j, k): recompute g_jk from the staged row
// and the column's support, then record a violation / band entry.
template <typename T>
__device__ __forceinline__ void kkt_flagged(const KktArgs<T> &A, int64_t k, int64_t j,
                                         const T *__restrict__ row)
{
    const int64_t p = A.p;
    int cnt = A.supp_cnt[k];
    cnt = cnt < 0 ? 0 : (cnt > kWMax ? kWMax : cnt);
    const T lam = (T)A.lam_used[k];
    T g = row[k];
    for (int q = 0; q < cnt; ++q) {
        int64_t l = A.supp_idx[(int64_t)q * p + k];
        l = l < 0 ? 0 : (l >= p ? p - 1 : l);
        g -= A.supp_val[(int64_t)q * p + k] * row[l];
    }
    const T a = g < T(0) ? -g : g;
    const bool over = a > lam + A.kkt_tol;
    const bool near = A.band > T(0) && a > lam - A.band;
    if (!over && !near) return;
    // membership of j in the working set (a short ascending list)
    const int *wl = A.w_idx + k * kWMax;
    int lo = 0, hi = A.w_cnt[k];
    hi = hi < 0 ? 0 : (hi > kWMax ? kWMax : hi);
    const int wn = hi;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (wl[mid] < (int)j) lo = mid + 1;
        else hi = mid;
    }
    const bool inW = lo < wn && wl[lo] == (int)j;
    if (over && !inW) {
        int slot = atomicAdd(&A.pend_cnt[k], 1);
        if (slot < kPendMax) A.pend_idx[k * kPendMax + slot] = (int)j;
        if (slot == 0) {
            int d = atomicAdd(A.dirty_cnt, 1);
            A.dirty_list[d] = (int)k;
        }
    }
    if (near) {
        bool inS = false;
        for (int q = 0; q < cnt; ++q) inS |= A.supp_idx[(int64_t)q * p + k] == (int)j;
        if (!inS) {
            int slot = atomicAdd(&A.band_cnt[k], 1);
            if (slot < kBandMax) A.band_idx[k * kBandMax + slot] = (int)j;
        }
    }
}

// Persistent blocks: block b owns rows [b * rpb, (b + 1) * rpb) of S.  For
// each chunk of kKktThreads * CPT columns the block loads every thread's
// CPT columns (support, lambda) into registers once, then streams its row
// tiles of RJ rows through LDS, so S is read once per column chunk (once when
// p <= kKktThreads * CPT) and the support lists once per block and chunk.
template <typename T, int RJ, int CPT>
__global__ __launch_bounds__(kKktThreads) void k_kkt_rows(KktArgs<T> A, int64_t rpb)
{
    extern __shared__ __align__(16) unsigned char kkt_lds[];
    T *rows = reinterpret_cast<T *>(kkt_lds);
    if (*A.flags) return;
    const int64_t p = A.p;
    const int64_t rb = (int64_t)blockIdx.x * rpb;
    const int64_t re = rb + rpb < p ? rb + rpb : p;
    if (rb >= p) return;
    const int tid = threadIdx.x;
    for (int64_t cbase = 0; cbase < p; cbase += (int64_t)CPT * kKktThreads) {
        int64_t kk[CPT];
        int cnt[CPT];
        T lam[CPT];
        bool act[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            kk[u] = cbase + (int64_t)u * kKktThreads + tid;
            act[u] = kk[u] < p && A.col_status[kk[u]] == kColDeferred;
            cnt[u] = act[u] ? A.supp_cnt[kk[u]] : 0;
            cnt[u] = cnt[u] < 0 ? 0 : (cnt[u] > kWMax ? kWMax : cnt[u]);
            lam[u] = act[u] ? (T)A.lam_used[kk[u]] : T(0);
        }
        // the first kKktQ slots are always written (padding (k, 0) past the
        // support), so these loads do not wait for the counts
        int li[CPT][kKktQ];
        T lv[CPT][kKktQ];
#pragma unroll
        for (int u = 0; u < CPT; ++u)
#pragma unroll
            for (int q = 0; q < kKktQ; ++q) {
                const int64_t kq = kk[u] < p ? kk[u] : 0;
                int v = A.supp_idx[(int64_t)q * p + kq];
                li[u][q] = v < 0 ? 0 : (v >= p ? (int)(p - 1) : v);
                lv[u][q] = A.supp_val[(int64_t)q * p + kq];
            }
        for (int64_t j0 = rb; j0 < re; j0 += RJ) {
            const int64_t nr = (re - j0) < RJ ? (re - j0) : RJ;
            __syncthreads();  // previous tile consumed
            {
                // rows j0 .. j0+nr-1 of S are contiguous: 16-byte loads, four in
                // flight per thread before any is stored
                const T *src = A.S + j0 * p;
                const int64_t tot = nr * p;
                constexpr int V = 16 / sizeof(T);
                const bool aligned = ((uintptr_t)src & 15u) == 0;
                const int64_t nvec = aligned ? tot / V : 0;
                typedef __attribute__((ext_vector_type(4))) unsigned int u4;
                const u4 *s4 = reinterpret_cast<const u4 *>(src);
                u4 *d4 = reinterpret_cast<u4 *>(rows);
                for (int64_t e0 = tid; e0 < nvec; e0 += 4 * (int64_t)kKktThreads) {
                    u4 t[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        int64_t e = e0 + (int64_t)u * kKktThreads;
                        if (e < nvec) t[u] = s4[e];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        int64_t e = e0 + (int64_t)u * kKktThreads;
                        if (e < nvec) d4[e] = t[u];
                    }
                }
                for (int64_t e = nvec * V + tid; e < tot; e += kKktThreads) rows[e] = src[e];
            }
            __syncthreads();
            // gradients of every (row, column) pair; only a flag leaves the
            // unrolled body
            unsigned long long flagged = 0ull;
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                if (!act[u]) continue;
                const int64_t k = kk[u];
                T acc[RJ];
#pragma unroll
                for (int r = 0; r < RJ; ++r) acc[r] = r < nr ? rows[r * p + k] : T(0);
#pragma unroll
                for (int q = 0; q < kKktQ; ++q)
#pragma unroll
                    for (int r = 0; r < RJ; ++r)
                        if (r < nr) acc[r] -= lv[u][q] * rows[r * p + li[u][q]];
                for (int q = kKktQ; q < cnt[u]; ++q) {
                    int64_t l = A.supp_idx[(int64_t)q * p + k];
                    l = l < 0 ? 0 : (l >= p ? p - 1 : l);
                    const T v = A.supp_val[(int64_t)q * p + k];
#pragma unroll
                    for (int r = 0; r < RJ; ++r)
                        if (r < nr) acc[r] -= v * rows[r * p + l];
                }
                const T lo_thr = A.band > T(0) ? lam[u] - A.band : lam[u] + A.kkt_tol;
#pragma unroll
                for (int r = 0; r < RJ; ++r) {
                    const T a = acc[r] < T(0) ? -acc[r] : acc[r];
                    if (r < nr && j0 + r != k && a > lo_thr) flagged |= 1ull << (u * RJ + r);
                }
            }
            while (flagged) {
                const int bit = __builtin_ctzll(flagged);
                flagged &= flagged - 1;
                const int u = bit / RJ, r = bit % RJ;
                const int64_t k = cbase + (int64_t)u * kKktThreads + tid;
                kkt_flagged<T>(A, k, j0 + r, rows + (int64_t)r * p);
            }
        }
    }
}

template <typename T, int RJ, int CPT>
static void launch_kkt_rows_c(const KktArgs<T> &a, hipStream_t s)
{
    // one block per CU, each owning a contiguous range of rows
    int64_t nblk = 256;
    int64_t rpb = (a.p + nblk - 1) / nblk;
    rpb = (rpb + RJ - 1) / RJ * RJ;
    nblk = (a.p + rpb - 1) / rpb;
    const size_t lds = (size_t)RJ * (size_t)a.p * sizeof(T);
    hipLaunchKernelGGL((k_kkt_rows<T, RJ, CPT>), dim3((unsigned)nblk), dim3(kKktThreads), lds, s, a,
                       rpb);
}

// rj: rows that fit in LDS.  Columns per thread: enough to cover p in one
// chunk (S read once) within the register budget; rows per tile are then
// capped so the unrolled gathers stay in registers.
template <typename T>
void launch_kkt_rows(const KktArgs<T> &a, int rj, hipStream_t s)
{
    const int64_t need = (a.p + kKktThreads - 1) / kKktThreads;
    if constexpr (sizeof(T) == 4) {
        if (need <= 4) {
            if (rj >= 4) launch_kkt_rows_c<T, 4, 4>(a, s);
            else if (rj == 2) launch_kkt_rows_c<T, 2, 4>(a, s);
            else launch_kkt_rows_c<T, 1, 4>(a, s);
        } else if (need <= 6) {
            if (rj >= 4) launch_kkt_rows_c<T, 4, 6>(a, s);
            else if (rj == 2) launch_kkt_rows_c<T, 2, 6>(a, s);
            else launch_kkt_rows_c<T, 1, 6>(a, s);
        } else {
            if (rj >= 2) launch_kkt_rows_c<T, 2, 10>(a, s);
            else launch_kkt_rows_c<T, 1, 10>(a, s);
        }
    } else {
        if (need <= 2) {
            if (rj >= 8) launch_kkt_rows_c<T, 8, 2>(a, s);
            else if (rj == 4) launch_kkt_rows_c<T, 4, 2>(a, s);
            else if (rj == 2) launch_kkt_rows_c<T, 2, 2>(a, s);
            else launch_kkt_rows_c<T, 1, 2>(a, s);
        } else if (need <= 4) {
            if (rj >= 4) launch_kkt_rows_c<T, 4, 4>(a, s);
            else if (rj == 2) launch_kkt_rows_c<T, 2, 4>(a, s);
            else launch_kkt_rows_c<T, 1, 4>(a, s);
        } else if (need <= 6) {
            if (rj >= 2) launch_kkt_rows_c<T, 2, 6>(a, s);
            else launch_kkt_rows_c<T, 1, 6>(a, s);
        } else {
            launch_kkt_rows_c<T, 1, 8>(a, s);
        }
    }
}

template void launch_kkt_rows<double>(const KktArgs<double> &, int, hipStream_t);
template void launch_kkt_rows<float>(const KktArgs<float> &, int, hipStream_t);

} // namespace spmesl
