// syrk.hip -- the sample covariance S = Xs^T Xs / n on the matrix cores.
//
// S is the only dense contraction of the method (n p^2 multiply-adds).  Only
// the upper triangle of 64x64 (or 128x128) tiles is computed; each tile is
// written twice, once as is and once transposed, so S is stored full and
// every row of S is a contiguous read for the solver.  The diagonal is set
// to exactly 1 (s_jj = 1 for standardised columns, Section 2.2), which the
// coordinate update relies on.
//
// Three forms:
//   * double: v_mfma_f64_16x16x4f64, Xs row-major n x p;
//   * float : v_mfma_f32_16x16x4f32, same layout;
//   * mixed : two-term bfloat16 split x = hi + lo of float(x), products
//             hi*hi + hi*lo + lo*hi accumulated in float by
//             v_mfma_f32_16x16x32_bf16 from variable-major hi/lo panels.
//
// Operand layout of the 16x16xK MFMAs used here (wave64): lane l supplies
// row l%16 of A and column l%16 of B, at k-block l/16.  Accumulator element r
// of lane l is D[4*(l/16) + r][l%16] for the float-output MFMAs and
// D[4*r + l/16][l%16] for the double one (checked on the device).
#include "common.hpp"

namespace spmesl {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 type; };
template <> struct Acc<float> { typedef f4 type; };

// row of accumulator element r of `lane` within a 16x16 block
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return 4 * r + (lane >> 4); }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

// The screen (see Screen): entry s_jk = v makes j a candidate of column k.
// Candidates of a tile are collected in LDS (a short list; an LDS atomic
// returns quickly) and flushed with one round of global atomics per tile, so
// no wave waits on a global atomic inside the store loops.
constexpr int kScreenTile = 512;  // candidates a tile collects before storing directly

struct ScreenLds {
    int n;
    int jk[2 * kScreenTile];
};

template <typename T>
__device__ __forceinline__ void screen_entry(ScreenLds &L, int *cnt, int *idx, T thr, int64_t j,
                                             int64_t k, T v)
{
    const bool hit = cnt && j != k && (v < T(0) ? -v : v) > thr;
    if (!__ballot(hit)) return;  // the common case: one wave-uniform branch
    if (hit) {
        const int q = atomicAdd(&L.n, 1);
        if (q < kScreenTile) {
            L.jk[2 * q] = (int)j;
            L.jk[2 * q + 1] = (int)k;
        } else {
            const int pos = atomicAdd(&cnt[k], 1);
            if (pos < kPendMax) idx[k * kPendMax + pos] = (int)j;
        }
    }
}

// After the tile's entries are collected (and a barrier): store them.  The
// persistent kernel calls this for a tile while the next tile's first stage
// is being copied, so the atomics' round trip overlaps the copy.
__device__ __forceinline__ void screen_flush(ScreenLds &L, int *cnt, int *idx)
{
    if (!cnt) return;
    const int m = L.n < kScreenTile ? L.n : kScreenTile;
    for (int q = threadIdx.x; q < m; q += blockDim.x) {
        const int j = L.jk[2 * q], k = L.jk[2 * q + 1];
        const int pos = atomicAdd(&cnt[k], 1);
        if (pos < kPendMax) idx[(int64_t)k * kPendMax + pos] = j;
    }
}

// Map a linear block id to an upper-triangle tile (bj <= bk), with blocks
// that share a row panel kept on the same XCD (blocks are dispatched to
// the 8 XCDs round-robin).
__device__ __forceinline__ void tile_of_block(int T, int *bj, int *bk)
{
    int nb = gridDim.x, bid = blockIdx.x;
    int x = bid & 7, q = nb >> 3, r = nb & 7;
    int t = x * q + (x < r ? x : r) + (bid >> 3);
    int row = 0;
    while (t >= T - row) {
        t -= T - row;
        ++row;
    }
    *bj = row;
    *bk = row + t;
}

constexpr int kSyrkKC = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_syrk_mfma(const T *__restrict__ Xs, int64_t n, int64_t p,
                                                   T *__restrict__ S, int Tt, T invn, T thr,
                                                   int *__restrict__ scnt, int *__restrict__ sidx)
{
    typedef typename Acc<T>::type AccT;
    __shared__ union {
        struct {
            T a[kSyrkKC][64];
            T b[kSyrkKC][64];
        } in;
        T out[64][65];
    } sm;
    __shared__ ScreenLds scr;
    int bj, bk;
    tile_of_block(Tt, &bj, &bk);
    const int64_t j0 = (int64_t)bj * 64, k0 = (int64_t)bk * 64;
    if (threadIdx.x == 0) scr.n = 0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    AccT acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = AccT{0, 0, 0, 0};

    // loader mapping: rows lr and lr + 16 of the chunk, 4 consecutive columns
    const int lr = tid >> 4, lc = (tid & 15) * 4;
    constexpr int NL = kSyrkKC / 16;
    T ra[NL][4], rb[NL][4];
    auto fetch = [&](int64_t i0) {
#pragma unroll
        for (int h = 0; h < NL; ++h) {
            int64_t i = i0 + lr + 16 * h;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int64_t ja = j0 + lc + e, kb = k0 + lc + e;
                ra[h][e] = (i < n && ja < p) ? Xs[i * p + ja] : T(0);
                rb[h][e] = (i < n && kb < p) ? Xs[i * p + kb] : T(0);
            }
        }
    };
    fetch(0);
    for (int64_t i0 = 0; i0 < n; i0 += kSyrkKC) {
#pragma unroll
        for (int h = 0; h < NL; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sm.in.a[lr + 16 * h][lc + e] = ra[h][e];
                sm.in.b[lr + 16 * h][lc + e] = rb[h][e];
            }
        __syncthreads();
        if (i0 + kSyrkKC < n) fetch(i0 + kSyrkKC);  // in flight during the MFMAs below
#pragma unroll
        for (int kk = 0; kk < kSyrkKC; kk += 4) {
            T av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = sm.in.a[kk + (lane >> 4)][32 * wm + 16 * a + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = sm.in.b[kk + (lane >> 4)][32 * wn + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
    // stage the tile (scaled by 1/n) for coalesced direct and mirrored writes
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sm.out[32 * wm + 16 * a + acc_row<T>(lane, r)][32 * wn + 16 * b + (lane & 15)] =
                    acc[a][b][r] * invn;
    __syncthreads();
    // a diagonal tile takes its upper triangle for both halves, so S is
    // symmetric bit for bit whatever the accumulation order
    const bool diag = bj == bk;
    for (int e = tid; e < 64 * 64; e += 256) {
        int rr = e >> 6, cc = e & 63;
        int64_t j = j0 + rr, k = k0 + cc;
        if (j < p && k < p) {
            const T v = (j == k) ? T(1) : ((diag && rr > cc) ? sm.out[cc][rr] : sm.out[rr][cc]);
            S[j * p + k] = v;
            screen_entry(scr, scnt, sidx, thr, j, k, v);
        }
    }
    if (bj != bk) {
        for (int e = tid; e < 64 * 64; e += 256) {
            int rr = e >> 6, cc = e & 63;  // row of the mirrored tile = k index
            int64_t k = k0 + rr, j = j0 + cc;
            if (j < p && k < p) {
                const T v = sm.out[cc][rr];
                S[k * p + j] = v;
                screen_entry(scr, scnt, sidx, thr, k, j, v);
            }
        }
    }
    __syncthreads();
    screen_flush(scr, scnt, sidx);
}

template <typename T>
static void launch_syrk_t(const T *Xs, int64_t n, int64_t p, T *S, T thr, const Screen &sc, hipStream_t s)
{
    int Tt = (int)((p + 63) / 64);
    int64_t ntiles = (int64_t)Tt * (Tt + 1) / 2;
    hipLaunchKernelGGL(k_syrk_mfma<T>, dim3((unsigned)ntiles), dim3(256), 0, s, Xs, n, p, S, Tt,
                       (T)(1.0 / (double)n), thr, sc.cnt, sc.idx);
}

void launch_syrk_f64(const double *Xs, int64_t n, int64_t p, double *S, const Screen &sc, hipStream_t s)
{
    launch_syrk_t<double>(Xs, n, p, S, sc.thr64, sc, s);
}
void launch_syrk_f32(const float *Xs, int64_t n, int64_t p, float *S, const Screen &sc, hipStream_t s)
{
    launch_syrk_t<float>(Xs, n, p, S, sc.thr32, sc, s);
}

// ---------------------------------------------------------------------------
// mixed form: bf16 split, 128 x 128 tiles, 64 samples per stage
//
// Persistent blocks walk the upper-triangle tile list (tiles of one row
// panel kept on one XCD).  A stage (the hi and lo panels of the tile's row
// and column blocks, 128 variables x 64 samples each, 64 KB) is copied to LDS
// by the direct global-to-LDS path; the output tile of the epilogue reuses
// the same LDS.  At 66 KB of LDS two blocks share a CU, so one block's copy
// overlaps the other's matrix-core work (measured faster than one block per
// CU with two stage buffers).
//
// LDS layout of a panel: row m (a variable) holds its 64 samples as eight
// 16-byte chunks, chunk c stored in slot c ^ f(m), f(m) = (m & 7) ^ ((m >> 3)
// & 1).  The operand reads (16 lanes on 16 consecutive rows, one chunk each)
// then touch distinct banks with either 32 or 64 LDS banks.
// ---------------------------------------------------------------------------
constexpr int kBfKC = 64;                   // samples per stage
constexpr int kBfPanel = 128 * kBfKC * 2;   // bytes of one panel (16 KB)
constexpr int kBfStage = 4 * kBfPanel;      // hi_J, lo_J, hi_K, lo_K
constexpr int kBfOutLd = 129;               // padded row of the staged output tile
constexpr int kBfOut = 128 * kBfOutLd * 4;  // output tile; the stage fits inside
static_assert(kBfOut >= kBfStage, "stage and output tile share the LDS");
constexpr int kBfLds = kBfOut + (int)sizeof(ScreenLds);  // + the tile's screen candidates

__device__ __forceinline__ int bf_swz(int m) { return (m & 7) ^ ((m >> 3) & 1); }

// Upper-triangle tile number -> (row block, column block), row-major order.
__device__ __forceinline__ void bf_tile(int t, int T, int *bj, int *bk)
{
    int row = 0;
    while (t >= T - row) {
        t -= T - row;
        ++row;
    }
    *bj = row;
    *bk = row + t;
}

// Issue the copies of one stage: samples [i0, i0 + 64) of variables j0.. and
// k0.. (hi and lo).  A diagonal tile copies its one panel pair only.  Rows
// past p load row p - 1 (valid memory; those results are never stored).
__device__ __forceinline__ void bf_issue(const uint16_t *__restrict__ hi, const uint16_t *__restrict__ lo,
                                         int64_t npad, int64_t p, int64_t j0, int64_t k0, int64_t i0,
                                         bool diag, unsigned char *stage)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int npan = diag ? 2 : 4;
    // 16 groups of 8 rows per panel; one 1 KB wave instruction per group
    for (int blk = wv; blk < npan * 16; blk += 4) {
        const int pnl = blk >> 4, grp = blk & 15;
        const int m = grp * 8 + (lane >> 3);
        const int c = (lane & 7) ^ bf_swz(m);
        int64_t v = ((pnl < 2) ? j0 : k0) + m;
        v = v < p ? v : p - 1;
        const uint16_t *src = ((pnl & 1) ? lo : hi) + v * npad + i0 + c * 8;
        __builtin_amdgcn_global_load_lds(
            src, (__attribute__((address_space(3))) void *)(stage + pnl * kBfPanel + grp * 1024), 16, 0, 0);
    }
}

__global__ __launch_bounds__(256) void k_syrk_bf16x3(const uint16_t *__restrict__ hi,
                                                     const uint16_t *__restrict__ lo,
                                                     int64_t npad, int64_t p,
                                                     float *__restrict__ S, int Tt, float invn,
                                                     float thr, int *__restrict__ scnt,
                                                     int *__restrict__ sidx)
{
    extern __shared__ __align__(16) unsigned char bf_lds[];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int ntiles = Tt * (Tt + 1) / 2;
    // tiles of XCD x = blockIdx % 8 form one contiguous range of the list
    const int nb = gridDim.x, x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int nbx = (nb >> 3) + ((nb & 7) > x ? 1 : 0);
    const int q = ntiles >> 3, r = ntiles & 7;
    const int tbeg = x * q + (x < r ? x : r), tend = tbeg + q + (x < r ? 1 : 0);
    const int nst = (int)(npad / kBfKC);

    ScreenLds &scr = *reinterpret_cast<ScreenLds *>(bf_lds + kBfOut);
    bool pending = false;  // the previous tile's screen candidates await their flush
    int t = tbeg + slot;
    for (; t < tend; t += nbx) {
        int bj, bk;
        bf_tile(t, Tt, &bj, &bk);
        const int64_t j0 = (int64_t)bj * 128, k0 = (int64_t)bk * 128;
        const bool diag = bj == bk;
        const int pk = diag ? 0 : 2;
        f4 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
        for (int st = 0; st < nst; ++st) {
            __syncthreads();
            bf_issue(hi, lo, npad, p, j0, k0, (int64_t)st * kBfKC, diag, bf_lds);
            if (st == 0 && pending) screen_flush(scr, scnt, sidx);  // the previous tile's
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const unsigned char *sb = bf_lds;
#pragma unroll
            for (int kk = 0; kk < kBfKC; kk += 32) {
                const int c = kk / 8 + (lane >> 4);
                bf8 ha[4], la[4], hb[4], lb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int m = 64 * wm + 16 * a + (lane & 15);
                    const int off = m * 128 + ((c ^ bf_swz(m)) << 4);
                    ha[a] = *reinterpret_cast<const bf8 *>(sb + off);
                    la[a] = *reinterpret_cast<const bf8 *>(sb + kBfPanel + off);
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int m = 64 * wn + 16 * b + (lane & 15);
                    const int off = m * 128 + ((c ^ bf_swz(m)) << 4);
                    hb[b] = *reinterpret_cast<const bf8 *>(sb + pk * kBfPanel + off);
                    lb[b] = *reinterpret_cast<const bf8 *>(sb + (pk + 1) * kBfPanel + off);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(la[a], hb[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[a], lb[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[a], hb[b], acc[a][b], 0, 0, 0);
                    }
            }
        }
        __syncthreads();
        // every thread is past the previous tile's flush (stage barriers)
        if (tid == 0) scr.n = 0;
        float *outc = reinterpret_cast<float *>(bf_lds);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    outc[(64 * wm + 16 * a + 4 * (lane >> 4) + rr) * kBfOutLd + 64 * wn + 16 * b + (lane & 15)] =
                        acc[a][b][rr] * invn;
        __syncthreads();
        for (int e = tid; e < 128 * 128; e += 256) {
            const int rr = e >> 7, cc = e & 127;
            const int64_t j = j0 + rr, k = k0 + cc;
            if (j < p && k < p) {
                const float v = (j == k) ? 1.0f
                                         : ((diag && rr > cc) ? outc[cc * kBfOutLd + rr] : outc[rr * kBfOutLd + cc]);
                S[j * p + k] = v;
                screen_entry(scr, scnt, sidx, thr, j, k, v);
            }
        }
        if (!diag) {
            for (int e = tid; e < 128 * 128; e += 256) {
                const int rr = e >> 7, cc = e & 127;
                const int64_t k = k0 + rr, j = j0 + cc;
                if (j < p && k < p) {
                    const float v = outc[cc * kBfOutLd + rr];
                    S[k * p + j] = v;
                    screen_entry(scr, scnt, sidx, thr, k, j, v);
                }
            }
        }
        pending = true;
    }
    if (pending) {
        __syncthreads();
        screen_flush(scr, scnt, sidx);
    }
}

void launch_syrk_bf16x3(const uint16_t *hi, const uint16_t *lo, int64_t n, int64_t npad,
                        int64_t p, float *S, const Screen &sc, hipStream_t s)
{
    (void)n;
    int Tt = (int)((p + 127) / 128);
    int64_t ntiles = (int64_t)Tt * (Tt + 1) / 2;
    // two blocks per CU (the LDS of a block), at most one per tile
    int64_t grid = ntiles < 512 ? ntiles : 512;
    hipLaunchKernelGGL(k_syrk_bf16x3, dim3((unsigned)grid), dim3(256), kBfLds, s, hi, lo, npad, p, S,
                       Tt, (float)(1.0 / (double)n), sc.thr32, sc.cnt, sc.idx);
}

} // namespace spmesl
