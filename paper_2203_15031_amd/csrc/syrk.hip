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
template <int N>
struct ScreenLds {
    static constexpr int kCap = N;  // candidates a tile collects before storing directly
    int n;
    int jk[2 * N];
};

// Entry s_jk = v makes j a candidate of column k when |v| > thr and j < pv
// (pv: the candidate variables; p for SPMESL).
template <typename L, typename T>
__device__ __forceinline__ void screen_entry(L &lst, int *cnt, int *idx, T thr, int64_t pv, int64_t j, int64_t k,
                                             T v)
{
    const bool hit = cnt && j != k && j < pv && (v < T(0) ? -v : v) > thr;
    if (!__ballot(hit)) return;  // the common case: one wave-uniform branch
    if (hit) {
        const int q = atomicAdd(&lst.n, 1);
        if (q < L::kCap) {
            lst.jk[2 * q] = (int)j;
            lst.jk[2 * q + 1] = (int)k;
        } else {
            const int pos = atomicAdd(&cnt[k], 1);
            if (pos < kPendMax) idx[k * kPendMax + pos] = (int)j;
        }
    }
}

// Entry s_jk = s_kj = v of a symmetric pair (j != k) makes j a candidate of
// column k and k one of column j; v = 0 records nothing.  The wave's hits
// take their list slots with one LDS atomic.
template <typename L, typename T>
__device__ __forceinline__ void screen_pair(L &lst, int *cnt, int *idx, T thr, int64_t j, int64_t k, T v)
{
    const bool hit = cnt && j != k && (v < T(0) ? -v : v) > thr;
    const unsigned long long mask = __ballot(hit);
    if (!mask) return;  // the common case: one wave-uniform branch
    const int lead = __builtin_ffsll((long long)mask) - 1;
    int base = 0;
    if (lane_id() == lead) base = atomicAdd(&lst.n, 2 * __popcll(mask));
    base = __shfl(base, lead);
    if (!hit) return;
    const int q = base + 2 * lanes_below(mask);
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int a = (int)(d ? k : j), b = (int)(d ? j : k);  // a joins column b
        if (q + d < L::kCap) {
            lst.jk[2 * (q + d)] = a;
            lst.jk[2 * (q + d) + 1] = b;
        } else {
            const int pos = atomicAdd(&cnt[b], 1);
            if (pos < kPendMax) idx[(int64_t)b * kPendMax + pos] = a;
        }
    }
}

// Per-wave candidate lists (no atomics): wave w appends to its own segment
// and keeps the count in a wave-uniform register.
template <int NW, int N>
struct ScreenWaves {
    static constexpr int kCap = N;  // entries per wave
    int n[NW];
    int jk[NW][2 * N];
};

template <typename L, typename T>
__device__ __forceinline__ void screen_pair_wave(L &lst, int wv, int &count, int *cnt, int *idx, T thr,
                                                 int64_t j, int64_t k, T v)
{
    const bool hit = cnt && j != k && (v < T(0) ? -v : v) > thr;
    const unsigned long long mask = __ballot(hit);
    if (!mask) return;
    const int q = count + 2 * lanes_below(mask);
    count += 2 * __popcll(mask);
    if (!hit) return;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int a = (int)(d ? k : j), b = (int)(d ? j : k);  // a joins column b
        if (q + d < L::kCap) {
            lst.jk[wv][2 * (q + d)] = a;
            lst.jk[wv][2 * (q + d) + 1] = b;
        } else {
            const int pos = atomicAdd(&cnt[b], 1);
            if (pos < kPendMax) idx[(int64_t)b * kPendMax + pos] = a;
        }
    }
}

template <int NW, int N>
__device__ __forceinline__ void screen_flush_waves(ScreenWaves<NW, N> &lst, int *cnt, int *idx)
{
    if (!cnt) return;
    for (int w = 0; w < NW; ++w) {
        const int m = lst.n[w] < N ? lst.n[w] : N;
        for (int q0 = threadIdx.x; q0 < m; q0 += 8 * (int)blockDim.x) {
            int jj[8], pos[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + u * (int)blockDim.x;
                pos[u] = kPendMax;
                jj[u] = 0;
                if (q < m) {
                    jj[u] = lst.jk[w][2 * q];
                    pos[u] = atomicAdd(&cnt[lst.jk[w][2 * q + 1]], 1);
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + u * (int)blockDim.x;
                if (q < m && pos[u] < kPendMax) idx[(int64_t)lst.jk[w][2 * q + 1] * kPendMax + pos[u]] = jj[u];
            }
        }
    }
}

// After the tile's entries are collected (and a barrier): store them.  The
// persistent kernel calls this for a tile while the next tile's first stage
// is being copied, so the atomics' round trip overlaps the copy.
template <typename L>
__device__ __forceinline__ void screen_flush(L &lst, int *cnt, int *idx)
{
    if (!cnt) return;
    const int m = lst.n < L::kCap ? lst.n : L::kCap;
    // up to eight independent atomics per thread in flight, then the stores
    for (int q0 = threadIdx.x; q0 < m; q0 += 8 * (int)blockDim.x) {
        int jj[8], pos[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * (int)blockDim.x;
            pos[u] = kPendMax;
            jj[u] = 0;
            if (q < m) {
                jj[u] = lst.jk[2 * q];
                pos[u] = atomicAdd(&cnt[lst.jk[2 * q + 1]], 1);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * (int)blockDim.x;
            if (q < m && pos[u] < kPendMax) idx[(int64_t)lst.jk[2 * q + 1] * kPendMax + pos[u]] = jj[u];
        }
    }
}

// Blocks that share a row panel are kept on the same XCD (blocks are
// dispatched to the 8 XCDs round-robin): the position of block bid of nb in
// an order that gives each XCD a contiguous run.
__device__ __forceinline__ int64_t xcd_order(int64_t nb, int64_t bid)
{
    const int64_t x = bid & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (bid >> 3);
}

// Upper-triangle tile t (bj <= bk, row by row) of a T x T tiling.
__device__ __forceinline__ void tri_tile(int T, int64_t t, int *bj, int *bk)
{
    int row = 0;
    while (t >= T - row) {
        t -= T - row;
        ++row;
    }
    *bj = row;
    *bk = row + (int)t;
}

// Map a linear block id to an upper-triangle tile, XCD-aware.
__device__ __forceinline__ void tile_of_block(int T, int *bj, int *bk)
{
    tri_tile(T, xcd_order(gridDim.x, blockIdx.x), bj, bk);
}

constexpr int kSyrkKC = 32;

template <typename T>
struct SyrkMfmaSm {
    union {
        struct {
            T a[kSyrkKC][64];
            T b[kSyrkKC][64];
        } in;
        T out[64][65];
    };
};

// One 64 x 64 tile (bj, bk) of S by the block; scr: the screen's list (a
// 64 x 64 tile: about 6 per row at the workloads here).
template <typename T>
__device__ __forceinline__ void syrk_mfma_tile(const T *__restrict__ Xs, int64_t n, int64_t p, T *__restrict__ S,
                                               int bj, int bk, T invn, T thr, int64_t pv, int *__restrict__ scnt,
                                               int *__restrict__ sidx, SyrkMfmaSm<T> &sm, ScreenLds<512> &scr)
{
    typedef typename Acc<T>::type AccT;
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
            screen_entry(scr, scnt, sidx, thr, pv, j, k, v);
        }
    }
    if (bj != bk) {
        for (int e = tid; e < 64 * 64; e += 256) {
            int rr = e >> 6, cc = e & 63;  // row of the mirrored tile = k index
            int64_t k = k0 + rr, j = j0 + cc;
            if (j < p && k < p) {
                const T v = sm.out[cc][rr];
                S[k * p + j] = v;
                screen_entry(scr, scnt, sidx, thr, pv, k, j, v);
            }
        }
    }
    __syncthreads();
    screen_flush(scr, scnt, sidx);
}

template <typename T>
__global__ __launch_bounds__(256) void k_syrk_mfma(const T *__restrict__ Xs, int64_t n, int64_t p,
                                                   T *__restrict__ S, int Tt, T invn, T thr, int64_t pv,
                                                   int *__restrict__ scnt, int *__restrict__ sidx)
{
    __shared__ SyrkMfmaSm<T> sm;
    __shared__ ScreenLds<512> scr;
    int bj, bk;
    tile_of_block(Tt, &bj, &bk);
    syrk_mfma_tile<T>(Xs, n, p, S, bj, bk, invn, thr, pv, scnt, sidx, sm, scr);
}

// ---------------------------------------------------------------------------
// double form: 128 x 128 tiles.  Four waves of 64 x 64 (sixteen 16 x 16
// accumulator blocks each): per 4-sample step a wave reads 8 operands from
// LDS for 16 matrix-core operations, twice the 64 x 64 tile's ratio, and the
// panels of a stage (16 samples) give 16 flops per byte read from L2.  Each
// entry takes its products in the same sample order as the 64 x 64 kernel,
// so S is the same to the bit.  The epilogue stages the tile through LDS in
// two halves of 64 rows (two blocks per CU fit), each written directly and
// transposed; a diagonal tile writes its lower-left block as the mirror of
// its upper-right one in the first half and takes its upper triangle for
// both halves of each diagonal block, so S is symmetric bit for bit.
// ---------------------------------------------------------------------------
constexpr int kD = 128;   // tile edge
constexpr int kDKC = 16;  // samples per stage
constexpr int kDPad = 16; // LDS row padding of the stage panels (doubles)

struct SyrkD128Sm {
    union {
        struct {
            double a[kDKC][kD + kDPad];
            double b[kDKC][kD + kDPad];
        } in;
        double out[64][kD + 1];  // one half of the tile
    };
};

__device__ __forceinline__ void syrk_d128_tile(const double *__restrict__ Xs, int64_t n, int64_t p,
                                               double *__restrict__ S, int bj, int bk, double invn, double thr,
                                               int64_t pv, int *__restrict__ scnt, int *__restrict__ sidx,
                                               SyrkD128Sm &sm, ScreenLds<1024> &scr)
{
    const int64_t j0 = (int64_t)bj * kD, k0 = (int64_t)bk * kD;
    if (threadIdx.x == 0) scr.n = 0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};

    // loader: 32 threads per sample row, 4 consecutive variables each; rows
    // lr and lr + 8 of the stage
    const int lr = tid >> 5, lc = (tid & 31) * 4;
    constexpr int NL = kDKC / 8;
    const bool even = (p & 1) == 0;  // 16-byte aligned pairs (j0, lc even)
    double ra[NL][4], rb[NL][4];
    auto fetch1 = [&](int64_t i, int64_t c0, double *r) {
        if (i < n && c0 + 3 < p && even) {
            const double2 x0 = *reinterpret_cast<const double2 *>(Xs + i * p + c0);
            const double2 x1 = *reinterpret_cast<const double2 *>(Xs + i * p + c0 + 2);
            r[0] = x0.x;
            r[1] = x0.y;
            r[2] = x1.x;
            r[3] = x1.y;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) r[e] = (i < n && c0 + e < p) ? Xs[i * p + c0 + e] : 0.0;
        }
    };
    auto fetch = [&](int64_t i0) {
#pragma unroll
        for (int h = 0; h < NL; ++h) {
            const int64_t i = i0 + lr + 8 * h;
            fetch1(i, j0 + lc, ra[h]);
            fetch1(i, k0 + lc, rb[h]);
        }
    };
    fetch(0);
    for (int64_t i0 = 0; i0 < n; i0 += kDKC) {
#pragma unroll
        for (int h = 0; h < NL; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sm.in.a[lr + 8 * h][lc + e] = ra[h][e];
                sm.in.b[lr + 8 * h][lc + e] = rb[h][e];
            }
        __syncthreads();
        if (i0 + kDKC < n) fetch(i0 + kDKC);  // in flight during the MFMAs below
#pragma unroll
        for (int kk = 0; kk < kDKC; kk += 4) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = sm.in.a[kk + (lane >> 4)][64 * wm + 16 * a + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = sm.in.b[kk + (lane >> 4)][64 * wn + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }

    const bool diag = bj == bk;
    for (int h = 0; h < 2; ++h) {
        // rows 64h .. 64h + 63 of the tile (scaled by 1/n), from the waves
        // that hold them
        if (wm == h) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        sm.out[16 * a + acc_row<double>(lane, r)][64 * wn + 16 * b + (lane & 15)] =
                            acc[a][b][r] * invn;
        }
        __syncthreads();
        // direct rows j = j0 + 64h + rr; a diagonal tile's second half leaves
        // columns 0..63 to the first half's mirror
        const int c0 = (diag && h == 1) ? 64 : 0;
        for (int e = tid; e < 64 * kD; e += 256) {
            const int rr = e >> 7, cc = e & (kD - 1);
            const int R = 64 * h + rr;
            const int64_t j = j0 + R, k = k0 + cc;
            if (cc >= c0 && j < p && k < p) {
                double v;
                if (j == k)
                    v = 1.0;
                else if (diag && R > cc)
                    v = sm.out[cc - 64 * h][R];  // the upper-triangle value
                else
                    v = sm.out[rr][cc];
                S[j * p + k] = v;
                screen_entry(scr, scnt, sidx, thr, pv, j, k, v);
            }
        }
        // mirrored: S[k][j] for the half's 64 columns j; a diagonal tile
        // mirrors only its upper-right block (first half)
        if (!diag || h == 0) {
            const int kc0 = diag ? 64 : 0;
            for (int e = tid; e < kD * 64; e += 256) {
                const int kc = e >> 6, jc = e & 63;
                const int64_t k = k0 + kc, j = j0 + 64 * h + jc;
                if (kc >= kc0 && j < p && k < p) {
                    const double v = sm.out[jc][kc];
                    S[k * p + j] = v;
                    screen_entry(scr, scnt, sidx, thr, pv, k, j, v);
                }
            }
        }
        __syncthreads();  // the half is read before the next one is staged
    }
    screen_flush(scr, scnt, sidx);
}

__global__ __launch_bounds__(256, 2) void k_syrk_d128(const double *__restrict__ Xs, int64_t n, int64_t p,
                                                      double *__restrict__ S, int Tt, double invn, double thr,
                                                      int64_t pv, int *__restrict__ scnt, int *__restrict__ sidx)
{
    __shared__ SyrkD128Sm sm;
    __shared__ ScreenLds<1024> scr;
    int bj, bk;
    tile_of_block(Tt, &bj, &bk);
    syrk_d128_tile(Xs, n, p, S, bj, bk, invn, thr, pv, scnt, sidx, sm, scr);
}

__global__ __launch_bounds__(256, 2) void k_syrk_d128_grouped(const SyrkJobT<double> *__restrict__ tab,
                                                              const int64_t *__restrict__ off, int nd)
{
    __shared__ SyrkD128Sm sm;
    __shared__ ScreenLds<1024> scr;
    const int64_t t = xcd_order(gridDim.x, blockIdx.x);
    const int d = group_of(off, nd, t);
    const SyrkJobT<double> &J = tab[d];
    int bj, bk;
    tri_tile(J.Tt, t - off[d], &bj, &bk);
    syrk_d128_tile(J.Xs, J.n, J.p, J.S, bj, bk, J.invn, J.thr, J.pv, J.scnt, J.sidx, sm, scr);
}

// Tile edge of the double form: 128 when its upper-triangle tiles fill the
// chip (at least 256), else 64 (small p: the 64 x 64 kernel keeps more CUs
// busy).  Both kernels give each entry its products in the same sample order,
// so S is the same to the bit either way.
int syrk_f64_edge(int64_t p)
{
    const int64_t t = (p + kD - 1) / kD;
    return t * (t + 1) / 2 >= 256 ? kD : 64;
}

// The tiles of many problems in one launch, one tile per block: block b
// (in the XCD-aware order) is tile b - off[d] of problem d.
template <typename T>
__global__ __launch_bounds__(256) void k_syrk_mfma_grouped(const SyrkJobT<T> *__restrict__ tab,
                                                           const int64_t *__restrict__ off, int nd)
{
    __shared__ SyrkMfmaSm<T> sm;
    __shared__ ScreenLds<512> scr;
    const int64_t t = xcd_order(gridDim.x, blockIdx.x);
    const int d = group_of(off, nd, t);
    const SyrkJobT<T> &J = tab[d];
    int bj, bk;
    tri_tile(J.Tt, t - off[d], &bj, &bk);
    syrk_mfma_tile<T>(J.Xs, J.n, J.p, J.S, bj, bk, J.invn, J.thr, J.pv, J.scnt, J.sidx, sm, scr);
}

template <typename T>
SyrkJobT<T> syrk_job_mfma(const T *Xs, int64_t n, int64_t p, T *S, const Screen &sc, int edge, int64_t *tiles)
{
    SyrkJobT<T> j{};
    j.Xs = Xs;
    j.n = n;
    j.p = p;
    j.S = S;
    j.Tt = (int)((p + edge - 1) / edge);
    j.invn = (T)(1.0 / (double)n);
    if constexpr (sizeof(T) == 8)
        j.thr = (T)sc.thr64;
    else
        j.thr = (T)sc.thr32;
    j.pv = sc.pv > 0 ? sc.pv : p;
    j.scnt = sc.cnt;
    j.sidx = sc.idx;
    *tiles = (int64_t)j.Tt * (j.Tt + 1) / 2;
    return j;
}

template <typename T>
void launch_syrk_mfma_grouped(const SyrkJobT<T> *tab, const int64_t *tile_off, int nd, int64_t tiles, int edge,
                              hipStream_t s)
{
    if (tiles <= 0) return;
    if (sizeof(T) == 8 && edge == kD)
        hipLaunchKernelGGL(k_syrk_d128_grouped, dim3((unsigned)tiles), dim3(256), 0, s,
                           (const SyrkJobT<double> *)tab, tile_off, nd);
    else
        hipLaunchKernelGGL(k_syrk_mfma_grouped<T>, dim3((unsigned)tiles), dim3(256), 0, s, tab, tile_off, nd);
}

template SyrkJobT<double> syrk_job_mfma<double>(const double *, int64_t, int64_t, double *, const Screen &, int,
                                                int64_t *);
template SyrkJobT<float> syrk_job_mfma<float>(const float *, int64_t, int64_t, float *, const Screen &, int,
                                              int64_t *);
template void launch_syrk_mfma_grouped<double>(const SyrkJobT<double> *, const int64_t *, int, int64_t, int,
                                               hipStream_t);
template void launch_syrk_mfma_grouped<float>(const SyrkJobT<float> *, const int64_t *, int, int64_t, int,
                                              hipStream_t);

template <typename T>
static void launch_syrk_t(const T *Xs, int64_t n, int64_t p, T *S, T thr, const Screen &sc, hipStream_t s)
{
    const int edge = sizeof(T) == 8 ? syrk_f64_edge(p) : 64;
    const int Tt = (int)((p + edge - 1) / edge);
    const int64_t ntiles = (int64_t)Tt * (Tt + 1) / 2;
    if (sizeof(T) == 8 && edge == kD)
        hipLaunchKernelGGL(k_syrk_d128, dim3((unsigned)ntiles), dim3(256), 0, s, (const double *)Xs, n, p,
                           (double *)S, Tt, 1.0 / (double)n, (double)thr, sc.pv > 0 ? sc.pv : p, sc.cnt, sc.idx);
    else
        hipLaunchKernelGGL(k_syrk_mfma<T>, dim3((unsigned)ntiles), dim3(256), 0, s, Xs, n, p, S, Tt,
                           (T)(1.0 / (double)n), thr, sc.pv > 0 ? sc.pv : p, sc.cnt, sc.idx);
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
// mixed form: bf16 split, 256 x 256 tiles, 32 samples per stage
//
// A block of 8 waves (64 x 128 each) computes one 256 x 256 tile; blocks
// loop over the upper-triangle tile list when it is longer than the grid.
// A stage (hi and lo of the tile's 256 row and 256 column variables over 32
// samples, 64 KB) is copied to LDS by the direct global-to-LDS path into two
// alternating buffers, so the copy of stage s + 1 is in flight while stage s
// feeds the matrix cores.  Against 128 x 128 tiles this halves the panel
// traffic per flop; measured at p = 5000 it takes 64 us where the 128 x 128
// form at two blocks per CU took 85 us and the register-staged form 103 us.
//
// LDS layout of a panel: row m (a variable) holds its 32 samples as four
// 16-byte chunks, chunk c in slot c ^ f(m), f(m) = ((m >> 1) ^ (m >> 2)) & 3.
// The operand reads (16 lanes on 16 consecutive rows, one chunk each) then
// touch distinct banks with either 32 or 64 LDS banks.
//
// The epilogue writes S from the accumulators, directly (64-byte row
// segments) and transposed (16-byte stores of four consecutive columns),
// with no LDS staging; the screen of the first solves is taken on the same
// values (each pair for both columns).
// ---------------------------------------------------------------------------
constexpr int kBfTile = 256;
constexpr int kBfKC = 32;                     // samples per stage (one MFMA k-step)
constexpr int kBfPanel = kBfTile * kBfKC * 2; // 16 KB: 256 rows x 64 B
constexpr int kBfStage = 4 * kBfPanel;        // hi_J, lo_J, hi_K, lo_K
typedef ScreenWaves<8, 448> BfScreen;        // fills the LDS left by the two stages
constexpr int kBfLds = 2 * kBfStage + (int)sizeof(BfScreen);
static_assert(kBfLds <= 160 * 1024, "LDS of one block");

__device__ __forceinline__ int bf_swz(int m) { return ((m >> 1) ^ (m >> 2)) & 3; }

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

// Issue the copies of one stage: samples [i0, i0 + 32) of variables j0.. and
// k0.. (hi and lo).  A diagonal tile copies its one panel pair only.  Rows
// past p load row p - 1 (valid memory; those results are never stored).
__device__ __forceinline__ void bf_issue(const uint16_t *__restrict__ hi, const uint16_t *__restrict__ lo,
                                         int64_t npad, int64_t p, int64_t j0, int64_t k0, int64_t i0,
                                         bool diag, unsigned char *stage)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int npan = diag ? 2 : 4;
    // 16 groups of 16 rows per panel; one 1 KB wave instruction per group
    for (int blk = wv; blk < npan * 16; blk += 8) {
        const int pnl = blk >> 4, grp = blk & 15;
        const int m = grp * 16 + (lane >> 2);
        const int c = (lane & 3) ^ bf_swz(m);
        int64_t v = ((pnl < 2) ? j0 : k0) + m;
        v = v < p ? v : p - 1;
        const uint16_t *src = ((pnl & 1) ? lo : hi) + v * npad + i0 + c * 8;
        __builtin_amdgcn_global_load_lds(
            src, (__attribute__((address_space(3))) void *)(stage + pnl * kBfPanel + grp * 1024), 16, 0, 0);
    }
}

// One 256 x 256 tile (bj, bk) of one problem's S, by the whole block.
__device__ __forceinline__ void bf_tile_run(const uint16_t *__restrict__ hi, const uint16_t *__restrict__ lo,
                                            int64_t npad, int64_t p, float *__restrict__ S, float invn, float thr,
                                            int *__restrict__ scnt, int *__restrict__ sidx, int bj, int bk,
                                            unsigned char *bf_lds)
{
    BfScreen &scr = *reinterpret_cast<BfScreen *>(bf_lds + 2 * kBfStage);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w & 3, wn = w >> 2;
    const int nst = (int)(npad / kBfKC);
    const bool vec_ok = (p & 3) == 0;  // rows of S 16-byte aligned
    {
        const int64_t j0 = (int64_t)bj * kBfTile, k0 = (int64_t)bk * kBfTile;
        const bool diag = bj == bk;
        const int pk = diag ? 0 : 2;  // panels the column block reads
        f4 acc[4][8];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = f4{0, 0, 0, 0};
        __syncthreads();  // the previous tile's epilogue and flush are done with the LDS
        int nscr = 0;     // this wave's screen entries (wave-uniform)
        bf_issue(hi, lo, npad, p, j0, k0, 0, diag, bf_lds);
        for (int st = 0; st < nst; ++st) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of stage st have landed
            __syncthreads();                // ... every wave's; stage st - 1 is consumed
            if (st + 1 < nst)
                bf_issue(hi, lo, npad, p, j0, k0, (int64_t)(st + 1) * kBfKC, diag,
                         bf_lds + ((st + 1) & 1) * kBfStage);
            const unsigned char *sb = bf_lds + (st & 1) * kBfStage;
            const int c = lane >> 4;
            bf8 ha[4], la[4], hb[8], lb[8];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int m = 64 * wm + 16 * a + (lane & 15);
                const int off = m * 64 + ((c ^ bf_swz(m)) << 4);
                ha[a] = *reinterpret_cast<const bf8 *>(sb + off);
                la[a] = *reinterpret_cast<const bf8 *>(sb + kBfPanel + off);
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int m = 128 * wn + 16 * b + (lane & 15);
                const int off = m * 64 + ((c ^ bf_swz(m)) << 4);
                hb[b] = *reinterpret_cast<const bf8 *>(sb + pk * kBfPanel + off);
                lb[b] = *reinterpret_cast<const bf8 *>(sb + (pk + 1) * kBfPanel + off);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(la[a], hb[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[a], lb[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha[a], hb[b], acc[a][b], 0, 0, 0);
                }
        }
        // epilogue, straight from the accumulators: lane l holds rows
        // jb .. jb + 3 (jb = 4 (l / 16) within the 16 x 16 block) of column
        // kk = l % 16.  Direct: 16 lanes store 64 consecutive bytes of a row
        // of S; mirrored: the lane's four rows are four consecutive columns
        // of row kk, one 16-byte store.  A diagonal tile stores its upper
        // triangle both ways, so S is symmetric bit for bit.
        const int g4 = 4 * (lane >> 4), c16 = lane & 15;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int64_t kk = k0 + 128 * wn + 16 * b + c16;
                const int64_t jb = j0 + 64 * wm + 16 * a + g4;
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = jb + r == kk ? 1.0f : acc[a][b][r] * invn;
                // screen: a pair above the threshold is a candidate of both
                // columns (every lane takes part in the ballots)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool mine = jb + r < p && kk < p && (!diag || jb + r < kk);
                    screen_pair_wave(scr, w, nscr, scnt, sidx, thr, jb + r, kk, mine ? v[r] : 0.0f);
                }
                if (kk >= p) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (jb + r < p && (!diag || jb + r <= kk)) S[(jb + r) * p + kk] = v[r];
                if (vec_ok && jb + 3 < p && (!diag || kk > jb + 3)) {
                    *reinterpret_cast<f4 *>(&S[kk * p + jb]) = f4{v[0], v[1], v[2], v[3]};
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (jb + r < p && (!diag || kk > jb + r)) S[kk * p + jb + r] = v[r];
                }
            }
        if (lane == 0) scr.n[w] = nscr;
        __syncthreads();
        screen_flush_waves(scr, scnt, sidx);
    }
}

__global__ __launch_bounds__(512) void k_syrk_bf16x3(const uint16_t *__restrict__ hi,
                                                     const uint16_t *__restrict__ lo,
                                                     int64_t npad, int64_t p,
                                                     float *__restrict__ S, int Tt, float invn,
                                                     float thr, int *__restrict__ scnt,
                                                     int *__restrict__ sidx)
{
    extern __shared__ __align__(16) unsigned char bf_lds[];
    const int ntiles = Tt * (Tt + 1) / 2;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int bj, bk;
        bf_tile(t, Tt, &bj, &bk);
        bf_tile_run(hi, lo, npad, p, S, invn, thr, scnt, sidx, bj, bk, bf_lds);
    }
}

// The tiles of many problems in one launch: tile g is tile g - off[d] of
// problem d (its own upper-triangle order).
__global__ __launch_bounds__(512) void k_syrk_bf16x3_grouped(const SyrkJob *__restrict__ tab,
                                                             const int64_t *__restrict__ off, int nd)
{
    extern __shared__ __align__(16) unsigned char bf_lds[];
    const int64_t total = off[nd];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int d = group_of(off, nd, g);
        const SyrkJob &J = tab[d];
        int bj, bk;
        bf_tile((int)(g - off[d]), J.Tt, &bj, &bk);
        bf_tile_run(J.hi, J.lo, J.npad, J.p, J.S, J.invn, J.thr, J.scnt, J.sidx, bj, bk, bf_lds);
    }
}

SyrkJob syrk_job_bf16x3(const uint16_t *hi, const uint16_t *lo, int64_t n, int64_t npad, int64_t p, float *S,
                        const Screen &sc, int64_t *tiles)
{
    SyrkJob j{};
    j.hi = hi;
    j.lo = lo;
    j.npad = npad;
    j.p = p;
    j.S = S;
    j.Tt = (int)((p + kBfTile - 1) / kBfTile);
    j.invn = (float)(1.0 / (double)n);
    j.thr = sc.thr32;
    j.scnt = sc.cnt;
    j.sidx = sc.idx;
    *tiles = (int64_t)j.Tt * (j.Tt + 1) / 2;
    return j;
}

void launch_syrk_bf16x3_grouped(const SyrkJob *tab, const int64_t *tile_off, int nd, int64_t tiles, hipStream_t s)
{
    if (tiles <= 0) return;
    const int64_t grid = tiles < 256 ? tiles : 256;
    hipLaunchKernelGGL(k_syrk_bf16x3_grouped, dim3((unsigned)grid), dim3(512), kBfLds, s, tab, tile_off, nd);
}

void launch_syrk_bf16x3(const uint16_t *hi, const uint16_t *lo, int64_t n, int64_t npad,
                        int64_t p, float *S, const Screen &sc, hipStream_t s)
{
    int Tt = (int)((p + kBfTile - 1) / kBfTile);
    int64_t ntiles = (int64_t)Tt * (Tt + 1) / 2;
    // one block per CU (LDS and registers), at most one per tile
    int64_t grid = ntiles < 256 ? ntiles : 256;
    hipLaunchKernelGGL(k_syrk_bf16x3, dim3((unsigned)grid), dim3(512), kBfLds, s, hi, lo, npad, p, S,
                       Tt, (float)(1.0 / (double)n), sc.thr32, sc.cnt, sc.idx);
}

} // namespace spmesl
