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

constexpr int kKktThreads = 1024;
constexpr int kKktQ = 4;      // support entries preloaded per column

template <typename T, int RJ>
__device__ void kkt_check(const KktArgs<T> &A, int64_t k, int64_t j, T g, T lam, int cnt)
{
    const int64_t p = A.p;
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

template <typename T, int RJ>
__global__ __launch_bounds__(kKktThreads) void k_kkt_rows(KktArgs<T> A)
{
    extern __shared__ __align__(16) unsigned char kkt_lds[];
    T *rows = reinterpret_cast<T *>(kkt_lds);
    constexpr int kKktCols = sizeof(T) == 8 ? 2 : 4;  // columns a thread handles at once
    if (*A.flags) return;
    const int64_t p = A.p;
    const int64_t j0 = (int64_t)blockIdx.x * RJ;
    const int64_t nr = (p - j0) < RJ ? (p - j0) : RJ;
    // rows j0 .. j0+nr-1 of S are contiguous
    const T *src = A.S + j0 * p;
    const int64_t tot = nr * p;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) rows[e] = src[e];
    __syncthreads();
    for (int64_t kb = threadIdx.x; kb < p; kb += (int64_t)kKktCols * blockDim.x) {
        int64_t kk[kKktCols];
        int cnt[kKktCols];
        T lam[kKktCols];
        bool act[kKktCols];
        // all metadata loads of the group first, then all support loads
#pragma unroll
        for (int u = 0; u < kKktCols; ++u) {
            kk[u] = kb + (int64_t)u * blockDim.x;
            act[u] = kk[u] < p && A.col_status[kk[u]] == kColDeferred;
            cnt[u] = act[u] ? A.supp_cnt[kk[u]] : 0;
            cnt[u] = cnt[u] < 0 ? 0 : (cnt[u] > kWMax ? kWMax : cnt[u]);
            lam[u] = act[u] ? (T)A.lam_used[kk[u]] : T(0);
        }
        int li[kKktCols][kKktQ];
        T lv[kKktCols][kKktQ];
#pragma unroll
        for (int u = 0; u < kKktCols; ++u)
#pragma unroll
            for (int q = 0; q < kKktQ; ++q) {
                bool ok = q < cnt[u];
                li[u][q] = ok ? A.supp_idx[(int64_t)q * p + kk[u]] : 0;
                lv[u][q] = ok ? A.supp_val[(int64_t)q * p + kk[u]] : T(0);
            }
#pragma unroll
        for (int u = 0; u < kKktCols; ++u) {
            if (!act[u]) continue;
            const int64_t k = kk[u];
            T acc[RJ];
#pragma unroll
            for (int r = 0; r < RJ; ++r) acc[r] = r < nr ? rows[r * p + k] : T(0);
#pragma unroll
            for (int q = 0; q < kKktQ; ++q) {
                const int64_t l = li[u][q] < 0 ? 0 : (li[u][q] >= p ? p - 1 : li[u][q]);
#pragma unroll
                for (int r = 0; r < RJ; ++r)
                    if (r < nr) acc[r] -= lv[u][q] * rows[r * p + l];
            }
            for (int q = kKktQ; q < cnt[u]; ++q) {
                int64_t l = A.supp_idx[(int64_t)q * p + k];
                l = l < 0 ? 0 : (l >= p ? p - 1 : l);
                const T v = A.supp_val[(int64_t)q * p + k];
#pragma unroll
                for (int r = 0; r < RJ; ++r)
                    if (r < nr) acc[r] -= v * rows[r * p + l];
            }
#pragma unroll
            for (int r = 0; r < RJ; ++r) {
                const int64_t j = j0 + r;
                if (r < nr && j != k) kkt_check<T, RJ>(A, k, j, acc[r], lam[u], cnt[u]);
            }
        }
    }
}

template <typename T>
void launch_kkt_rows(const KktArgs<T> &a, int rj, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.p + rj - 1) / rj);
    const size_t lds = (size_t)rj * (size_t)a.p * sizeof(T);
    const dim3 b(kKktThreads);
    switch (rj) {
    case 8: hipLaunchKernelGGL((k_kkt_rows<T, 8>), dim3(blocks), b, lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_kkt_rows<T, 4>), dim3(blocks), b, lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_kkt_rows<T, 2>), dim3(blocks), b, lds, s, a); break;
    default: hipLaunchKernelGGL((k_kkt_rows<T, 1>), dim3(blocks), b, lds, s, a); break;
    }
}

template void launch_kkt_rows<double>(const KktArgs<double> &, int, hipStream_t);
template void launch_kkt_rows<float>(const KktArgs<float> &, int, hipStream_t);

} // namespace spmesl
