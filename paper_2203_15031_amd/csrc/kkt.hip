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
#include <type_traits>

#include "common.hpp"

namespace spmesl {

// Two tile buffers of rj rows each (plus a 16-byte group of slack at either
// end) must fit the LDS budget.
static int64_t kkt_buffer_elems(int64_t p, int rj, size_t elem)
{
    const int64_t v = (int64_t)(16 / elem);
    return ((int64_t)rj * p + 2 * v + v - 1) / v * v;
}

// Flagged pairs of a block, examined after its row tiles (so that the few
// long chains of global loads they take hold no barrier of the tile loop).
constexpr int kKktFlagCap = 384;
struct KktFlagList {
    int n;
    int jk[2 * kKktFlagCap];
};

int kkt_rows_per_block(int64_t p, size_t elem, size_t lds_budget)
{
    lds_budget -= sizeof(KktFlagList);
    for (int rj = 4; rj >= 1; rj >>= 1)
        if (2 * (size_t)kkt_buffer_elems(p, rj, elem) * elem <= lds_budget) return rj;
    return 0;
}

constexpr int kKktThreads = 1024;
constexpr int kKktQ = 8;  // support entries held in registers per column

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

// Start the copy of elements [src, src + tot) of S into LDS with the direct
// global-to-LDS path (16 bytes per lane; a wave fills 1 KB of consecutive
// LDS).  Whole 16-byte groups are moved, so the tile starts at
// buf + (src's element offset within its group); the partial groups at
// either end bring a few neighbouring elements of S, all inside S's
// 256-byte-aligned workspace region.  Completion is awaited by the caller
// (vmcnt, then a barrier).
template <typename T>
__device__ __forceinline__ const T *kkt_issue_tile(const T *src, int64_t tot, T *buf)
{
    constexpr int V = 16 / sizeof(T);
    constexpr int NWV = kKktThreads / kWave;
    const uintptr_t a = (uintptr_t)src;
    const int lofs = (int)((a & 15u) / sizeof(T));
    const char *g0 = reinterpret_cast<const char *>(a & ~(uintptr_t)15u);
    const int64_t ng = (lofs + tot + V - 1) / V;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (int64_t e0 = (int64_t)wv * kWave; e0 < ng; e0 += (int64_t)NWV * kWave) {
        const int64_t e = e0 + lane;
        if (e < ng)
            __builtin_amdgcn_global_load_lds(
                g0 + e * 16, (__attribute__((address_space(3))) void *)(buf + e0 * V), 16, 0, 0);
    }
    return buf + lofs;
}

// Persistent blocks: block b owns rows [b * rpb, (b + 1) * rpb) of S.  For
// each chunk of kKktThreads * CPT columns every thread loads its CPT
// columns' first kKktQ support entries and thresholds into registers once;
// the block's row tiles of RJ rows then stream through two LDS buffers, the
// copy of tile t + 1 in flight while tile t is examined.  S is read once per
// column chunk (once when p <= kKktThreads * CPT).
//
// The register copy of a support holds its indices as 16-bit halves when
// PK (p <= 65535) and its coefficients as floats.  For double S that makes
// the examination a filter: the float coefficients move each gradient by at
// most 2^-24 ||beta||_1 (|S_jl| <= 1), so pairs are flagged against the
// threshold lowered by twice that, and every flagged pair is recomputed
// exactly from the double coefficients before anything is recorded.
template <typename T, int RJ, int CPT, bool PK>
__device__ __forceinline__ void kkt_rows_body(const KktArgs<T> &A, int64_t rpb, int64_t bstride, int64_t bid,
                                              unsigned char *kkt_lds, KktFlagList &fl)
{
    T *const buf0 = reinterpret_cast<T *>(kkt_lds);
    if (*A.flags) return;
    if (threadIdx.x == 0) fl.n = 0;  // visible after the chunk loop's first barrier
    const int64_t p = A.p;
    const int64_t rb = bid * rpb;
    const int64_t re = rb + rpb < p ? rb + rpb : p;
    if (rb >= p) return;
    const int tid = threadIdx.x;
    const int ntile = (int)((re - rb + RJ - 1) / RJ);
    constexpr int NI = PK ? kKktQ / 2 : kKktQ;
    for (int64_t cbase = 0; cbase < p; cbase += (int64_t)CPT * kKktThreads) {
        __syncthreads();  // the previous chunk's last tile has been read
        const T *tile = kkt_issue_tile<T>(A.S + rb * p, (re - rb < RJ ? re - rb : RJ) * p, buf0);
        int cnt[CPT];  // support size; -1 for a column not examined
        T thr[CPT];
        unsigned li[CPT][NI];
        float lv[CPT][kKktQ];
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int64_t k = cbase + (int64_t)u * kKktThreads + tid;
            const int64_t kq = k < p ? k : 0;
            // with PK every offset fits 32 bits: one offset register per
            // column against a scalar base per slot
            const unsigned ko = (unsigned)kq;
            auto at = [&](const auto *base, int64_t q) {
                typedef typename std::remove_const<typename std::remove_pointer<decltype(base)>::type>::type E;
                if constexpr (PK)
                    return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(base + q * p) +
                                                        ko * (unsigned)sizeof(E));
                else
                    return base[q * p + kq];
            };
            const bool act = k < p && at(A.col_status, 0) == kColDeferred;
            int c = act ? at(A.supp_cnt, 0) : -1;
            cnt[u] = c < -1 ? 0 : (c > kWMax ? kWMax : c);
            T l1 = T(0);
#pragma unroll
            for (int q = 0; q < kKktQ; ++q) {
                // slots past the count hold stale values: replaced by (0, 0),
                // which adds nothing
                int v = at(A.supp_idx, q);
                v = v < 0 ? 0 : (v >= (int)p - 1 ? (int)p - 1 : v);
                const T b = at(A.supp_val, q);
                const bool in = q < cnt[u];
                v = in ? v : 0;
                lv[u][q] = in ? (float)b : 0.0f;
                if (in) l1 += b < T(0) ? -b : b;
                if (PK) {
                    if (q & 1) li[u][q / 2] |= (unsigned)v << 16;
                    else li[u][q / 2] = (unsigned)v;
                } else {
                    li[u][q] = (unsigned)v;
                }
            }
            const T lam = act ? (T)at(A.lam_used, 0) : T(0);
            T t = A.band > T(0) ? lam - A.band : lam + A.kkt_tol;
            if (sizeof(T) == 8) t -= l1 * (T)(1.0 / 8388608.0);
            thr[u] = t;
        }
        for (int t = 0; t < ntile; ++t) {
            const int64_t j0 = rb + (int64_t)t * RJ;
            const int64_t nr = (re - j0) < RJ ? (re - j0) : RJ;
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of tile t have landed
            __syncthreads();                // ... and every wave's; tile t - 1 is no longer read
            const T *cur = tile;
            if (t + 1 < ntile) {
                const int64_t j1 = j0 + RJ;
                const int64_t n1 = (re - j1) < RJ ? (re - j1) : RJ;
                tile = kkt_issue_tile<T>(A.S + j1 * p, n1 * p, buf0 + ((t + 1) & 1) * bstride);
            }
            // gradients of every (row, column) pair; only a flag leaves the
            // unrolled body
            unsigned long long flagged = 0ull;
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                // opaque per tile: the slot masks and row offsets derived
                // from these are recomputed rather than held across tiles
                int cu = cnt[u];
                int kl = (int)(cbase + (int64_t)u * kKktThreads) + tid;
                asm volatile("" : "+v"(cu), "+v"(kl));
                if (cu < 0) continue;
                const int64_t k = kl;
                // rows past the tile's end (last tile of a range) read stale
                // LDS; their results are discarded by the flag test
                T acc[RJ];
#pragma unroll
                for (int r = 0; r < RJ; ++r) acc[r] = cur[r * p + k];
                // rows of this tile that are in the column's support: they sit
                // at |g| = lambda and are neither violators nor band entries,
                // so they must not take the rare path below
                unsigned supm = 0u;
                // slots in two groups of four, each without per-slot
                // branches (padding adds zero), so their gathers issue
                // together
#pragma unroll
                for (int g = 0; g < kKktQ; g += 4) {
                    if (g > 0 && cu <= g) break;
#pragma unroll
                    for (int q = g; q < g + 4; ++q) {
                        // the empty asm keeps the packed forms live across
                        // tiles instead of every unpacked index, row offset
                        // and converted coefficient
                        unsigned w = PK ? li[u][q / 2] : li[u][q];
                        float v32 = lv[u][q];
                        asm volatile("" : "+v"(w), "+v"(v32));
                        const int l = PK ? (int)((w >> ((q & 1) * 16)) & 0xffffu) : (int)w;
                        const T v = (T)v32;
#pragma unroll
                        for (int r = 0; r < RJ; ++r) acc[r] -= v * cur[r * p + l];
                        const unsigned d = (unsigned)(l - (int)j0);
                        if (q < cu && d < (unsigned)RJ) supm |= 1u << d;
                    }
                }
                for (int q = kKktQ; q < cu; ++q) {
                    int64_t l = A.supp_idx[(int64_t)q * p + k];
                    l = l < 0 ? 0 : (l >= p ? p - 1 : l);
                    const T v = A.supp_val[(int64_t)q * p + k];
#pragma unroll
                    for (int r = 0; r < RJ; ++r) acc[r] -= v * cur[r * p + l];
                    const unsigned d = (unsigned)(l - j0);
                    if (d < (unsigned)RJ) supm |= 1u << d;
                }
#pragma unroll
                for (int r = 0; r < RJ; ++r) {
                    const T a = acc[r] < T(0) ? -acc[r] : acc[r];
                    if (r < nr && j0 + r != k && a > thr[u] && !((supm >> r) & 1u))
                        flagged |= 1ull << (u * RJ + r);
                }
            }
            while (flagged) {
                const int bit = __builtin_ctzll(flagged);
                flagged &= flagged - 1;
                const int u = bit / RJ, r = bit % RJ;
                const int64_t k = cbase + (int64_t)u * kKktThreads + tid;
                const int pos = atomicAdd(&fl.n, 1);
                if (pos < kKktFlagCap) {
                    fl.jk[2 * pos] = (int)(j0 + r);
                    fl.jk[2 * pos + 1] = (int)k;
                } else {
                    kkt_flagged<T>(A, k, j0 + r, cur + (int64_t)r * p);  // list full
                }
            }
        }
        // the chunk's flagged pairs, re-read from S in global memory
        __syncthreads();
        const int nf = fl.n < kKktFlagCap ? fl.n : kKktFlagCap;
        for (int i = tid; i < nf; i += kKktThreads) {
            const int64_t j = fl.jk[2 * i], k = fl.jk[2 * i + 1];
            kkt_flagged<T>(A, k, j, A.S + j * p);
        }
        __syncthreads();
        if (tid == 0) fl.n = 0;
    }
}

template <typename T, int RJ, int CPT, bool PK>
__global__ __launch_bounds__(kKktThreads) void k_kkt_rows(KktArgs<T> A, int64_t rpb, int64_t bstride)
{
    extern __shared__ __align__(16) unsigned char kkt_lds[];
    __shared__ KktFlagList fl;
    kkt_rows_body<T, RJ, CPT, PK>(A, rpb, bstride, blockIdx.x, kkt_lds, fl);
}

// The same pass over many problems in one launch: block b is block
// b - off[d] of problem d.
template <typename T, int RJ, int CPT, bool PK>
__global__ __launch_bounds__(kKktThreads) void k_kkt_rows_grouped(const KktJob<T> *__restrict__ tab,
                                                                  const int64_t *__restrict__ off, int nd)
{
    extern __shared__ __align__(16) unsigned char kkt_lds[];
    __shared__ KktFlagList fl;
    const int64_t b = blockIdx.x;
    const int d = group_of(off, nd, b);
    const KktJob<T> &J = tab[d];
    kkt_rows_body<T, RJ, CPT, PK>(J.a, J.rpb, J.bstride, b - off[d], kkt_lds, fl);
}

template <typename T, int RJ, int CPT>
static void launch_kkt_rows_c(const KktArgs<T> &a, hipStream_t s)
{
    // one block per CU, each owning a contiguous range of rows
    int64_t nblk = 256;
    int64_t rpb = (a.p + nblk - 1) / nblk;
    rpb = (rpb + RJ - 1) / RJ * RJ;
    nblk = (a.p + rpb - 1) / rpb;
    const int64_t bstride = kkt_buffer_elems(a.p, RJ, sizeof(T));
    const size_t lds = 2 * (size_t)bstride * sizeof(T);
    if (a.p <= 65535)
        hipLaunchKernelGGL((k_kkt_rows<T, RJ, CPT, true>), dim3((unsigned)nblk), dim3(kKktThreads), lds,
                           s, a, rpb, bstride);
    else
        hipLaunchKernelGGL((k_kkt_rows<T, RJ, CPT, false>), dim3((unsigned)nblk), dim3(kKktThreads), lds,
                           s, a, rpb, bstride);
}

// rj: rows per tile that fit LDS twice.  Columns per thread: enough to cover
// p in one chunk (S read once), up to five for float and three for double
// (the register budget of 16 waves per CU); larger p takes several chunks.
template <typename T, int RJ>
static void launch_kkt_rows_r(const KktArgs<T> &a, hipStream_t s)
{
    const int64_t need = (a.p + kKktThreads - 1) / kKktThreads;
    if (need <= 1) launch_kkt_rows_c<T, RJ, 1>(a, s);
    else if (need <= 2) launch_kkt_rows_c<T, RJ, 2>(a, s);
    else if constexpr (sizeof(T) == 8) launch_kkt_rows_c<T, RJ, 3>(a, s);  // 5 would spill
    else if (need <= 3) launch_kkt_rows_c<T, RJ, 3>(a, s);
    else launch_kkt_rows_c<T, RJ, 5>(a, s);
}

template <typename T>
void launch_kkt_rows(const KktArgs<T> &a, int rj, hipStream_t s)
{
    if (rj >= 4) launch_kkt_rows_r<T, 4>(a, s);
    else if (rj == 2) launch_kkt_rows_r<T, 2>(a, s);
    else launch_kkt_rows_r<T, 1>(a, s);
}

template void launch_kkt_rows<double>(const KktArgs<double> &, int, hipStream_t);
template void launch_kkt_rows<float>(const KktArgs<float> &, int, hipStream_t);

template <typename T>
KktJob<T> kkt_job(const KktArgs<T> &a, int rj, int64_t *blocks)
{
    int64_t nblk = 256;
    int64_t rpb = (a.p + nblk - 1) / nblk;
    rpb = (rpb + rj - 1) / rj * rj;
    nblk = (a.p + rpb - 1) / rpb;
    KktJob<T> j{};
    j.a = a;
    j.rpb = rpb;
    j.bstride = kkt_buffer_elems(a.p, rj, sizeof(T));
    *blocks = nblk;
    return j;
}

template <typename T, int RJ, int CPT>
static void launch_kkt_grouped_c(const KktJob<T> *tab, const int64_t *off, int nd, int64_t blocks, int64_t pmax,
                                 hipStream_t s)
{
    const size_t lds = 2 * (size_t)kkt_buffer_elems(pmax, RJ, sizeof(T)) * sizeof(T);
    if (pmax <= 65535)
        hipLaunchKernelGGL((k_kkt_rows_grouped<T, RJ, CPT, true>), dim3((unsigned)blocks), dim3(kKktThreads), lds,
                           s, tab, off, nd);
    else
        hipLaunchKernelGGL((k_kkt_rows_grouped<T, RJ, CPT, false>), dim3((unsigned)blocks), dim3(kKktThreads), lds,
                           s, tab, off, nd);
}

template <typename T, int RJ>
static void launch_kkt_grouped_r(const KktJob<T> *tab, const int64_t *off, int nd, int64_t blocks, int64_t pmax,
                                 hipStream_t s)
{
    const int64_t need = (pmax + kKktThreads - 1) / kKktThreads;
    if (need <= 1) launch_kkt_grouped_c<T, RJ, 1>(tab, off, nd, blocks, pmax, s);
    else if (need <= 2) launch_kkt_grouped_c<T, RJ, 2>(tab, off, nd, blocks, pmax, s);
    else if constexpr (sizeof(T) == 8) launch_kkt_grouped_c<T, RJ, 3>(tab, off, nd, blocks, pmax, s);
    else if (need <= 3) launch_kkt_grouped_c<T, RJ, 3>(tab, off, nd, blocks, pmax, s);
    else launch_kkt_grouped_c<T, RJ, 5>(tab, off, nd, blocks, pmax, s);
}

template <typename T>
void launch_kkt_rows_grouped(const KktJob<T> *tab, const int64_t *off, int nd, int64_t blocks, int rj,
                             int64_t pmax, hipStream_t s)
{
    if (blocks <= 0) return;
    if (rj >= 4) launch_kkt_grouped_r<T, 4>(tab, off, nd, blocks, pmax, s);
    else if (rj == 2) launch_kkt_grouped_r<T, 2>(tab, off, nd, blocks, pmax, s);
    else launch_kkt_grouped_r<T, 1>(tab, off, nd, blocks, pmax, s);
}

template KktJob<double> kkt_job<double>(const KktArgs<double> &, int, int64_t *);
template KktJob<float> kkt_job<float>(const KktArgs<float> &, int, int64_t *);
template void launch_kkt_rows_grouped<double>(const KktJob<double> *, const int64_t *, int, int64_t, int, int64_t,
                                              hipStream_t);
template void launch_kkt_rows_grouped<float>(const KktJob<float> *, const int64_t *, int, int64_t, int, int64_t,
                                             hipStream_t);

} // namespace spmesl
