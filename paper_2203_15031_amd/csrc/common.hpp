// common.hpp -- device helpers and internal declarations shared by the
// SPMESL kernels and the host orchestration.  gfx950 only: wave64, MFMA.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace spmesl {

constexpr int kWave = 64;
// Largest working set of one regression (matches SPMESL_MAX_WORKING_SET).
constexpr int kWMax = 128;
// Violators one KKT pass may hand to the next round of a column.
constexpr int kPendMax = 64;
// Near-threshold candidates a float solve records for the double polish.
constexpr int kBandMax = 32;
// Support slots always written (padded with (k, 0)) so the row-tiled KKT pass
// can load them without waiting for the count.
constexpr int kSuppPad = 4;

// Per-solve counters, accumulated with 64-bit atomics.
enum Counter : int {
    kCntOuter = 0,
    kCntSweeps,
    kCntUpdates,
    kCntRounds,
    kCntMaxW,
    kCntMaxOuter,
    kCntNoconv,
    kCntEscalated,
    kCntPolishChecks,
    kCntPolishAdded,
    kCntBandOverflow,
    kCntSumW,
    kCntDense,
    kNumCounters
};

// Column status codes written by the kernels (mirror the public codes).
enum ColStatus : int {
    kColDenseQ = 3,     // handed to the dense tier (working set beyond 128)
    kColWarm = 2,       // state set by a warm start, not yet solved
    kColDeferred = 1,   // first solve done, KKT check left to the row-tiled pass
    kColOk = 0,
    kColDegenerate = -4,
    kColNoconv = -5,
    kColWorkset = -8,
};

// ---------------------------------------------------------------------------
// wave-level primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ float bcast(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ double bcast(double v, int lane)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int bcast(int v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Cross-lane moves by DPP (register to register, no LDS round trip).  Lanes
// that a pattern does not write (rows outside ROWS) take `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float old, float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double old, double v)
{
    const long long o = __double_as_longlong(old), b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Reduction over the 64 lanes: pairs and quads (quad permutes), half rows
// and rows of 16 (mirrors), then the four rows (broadcasts of lane 15 into
// rows 1 and 3, and of lane 31 into rows 2 and 3); lane 63 ends with the
// total, which every lane then reads.
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T identity, Op op)
{
    v = op(v, dpp_move<0xB1, 0xF>(identity, v));   // quad_perm [1, 0, 3, 2]
    v = op(v, dpp_move<0x4E, 0xF>(identity, v));   // quad_perm [2, 3, 0, 1]
    v = op(v, dpp_move<0x141, 0xF>(identity, v));  // row_half_mirror
    v = op(v, dpp_move<0x140, 0xF>(identity, v));  // row_mirror
    v = op(v, dpp_move<0x142, 0xA>(identity, v));  // row_bcast:15
    v = op(v, dpp_move<0x143, 0xC>(identity, v));  // row_bcast:31
    return bcast(v, 63);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    return wave_reduce(v, T(0), [](T a, T b) { return a + b; });
}
template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    return wave_reduce(v, -__builtin_huge_valf(), [](T a, T b) { return b > a ? b : a; });
}

// Start of column k's list of `cnt` entries in the per-column list arrays:
// slot k * kWMax, or (more than kWMax entries, from the dense tier) the pool
// after the p slots, at w_off[k].
__device__ __forceinline__ int64_t list_base(const int *w_off, int64_t p, int64_t k, int cnt)
{
    return cnt > kWMax ? p * (int64_t)kWMax + w_off[k] : k * (int64_t)kWMax;
}

// Soft_lambda(a) = sign(a) (|a| - lambda)_+ ; 0 at |a| == lambda.
template <typename T>
__device__ __forceinline__ T soft_threshold(T a, T lam)
{
    return a > lam ? a - lam : (a < -lam ? a + lam : T(0));
}

// ---------------------------------------------------------------------------
// launcher declarations (definitions live in the .hip files)
// ---------------------------------------------------------------------------

// Standardisation.  X: n x p row-major (ld = ldx).  partial: workspace of
// 2 * rchunks * p doubles.  flags[0] |= 1 on a non-finite value, |= 2 on a
// zero-variance column.
void launch_colstats(const double *X, int64_t n, int64_t p, int64_t ldx, double *partial,
                     int rchunks, double *mean, double *scale, int *flags, int *zero_cnt, hipStream_t s);
int colstats_rchunks(int64_t n, int64_t p);
// Xa (n x (p + m), row-major, contiguous) = [X | Y] for the scaled lassos of
// the m responses Y on the design X.
void launch_pack_columns(const double *X, int64_t n, int64_t p, int64_t ldx, const double *Y, int64_t m,
                         int64_t ldy, double *Xa, hipStream_t s);

// Xs = (X - mean) * scale, n x p row-major (ld p), double.
void launch_standardize_f64(const double *X, int64_t n, int64_t p, int64_t ldx,
                            const double *mean, const double *scale, double *Xs, hipStream_t s);
// float copy of the standardised data, n x p row-major.
void launch_standardize_f32(const double *X, int64_t n, int64_t p, int64_t ldx,
                            const double *mean, const double *scale, float *Xs, hipStream_t s);
// Transposed standardised data for the mixed form: Xt (p x n double) and
// the two-term bfloat16 split hi/lo of float(x), p x npad (npad = n padded
// to a multiple of 32, zero-filled).
// Mixed form: column statistics and the split in one kernel (X read once).
// Returns false (nothing launched) when a strip of n samples does not fit
// the kernel's LDS budget; the caller then takes the two-kernel path.
bool launch_stats_split(const double *X, int64_t n, int64_t p, int64_t ldx, double *mean,
                        double *scale, double *Xt, uint16_t *hi, uint16_t *lo, int64_t npad,
                        int *flags, int *zero_cnt, hipStream_t s);
void launch_standardize_split(const double *X, int64_t n, int64_t p, int64_t ldx,
                              const double *mean, const double *scale, double *Xt,
                              uint16_t *hi, uint16_t *lo, int64_t npad, hipStream_t s);

// S = Xs^T Xs / n with unit diagonal (p x p row-major, full).
// Screen of the first solves, done where S is written: for every column k
// the entries j != k with |s_jk| > thr (lambda0 + tol in S's precision, the
// KKT test at beta = 0) are appended to cnt[k] / idx[k * kPendMax + ...]
// (cnt counts past kPendMax; cnt zeroed beforehand).  cnt == nullptr: none.
struct Screen {
    double thr64 = 0.0;
    float thr32 = 0.0f;
    int *cnt = nullptr;
    int *idx = nullptr;
    int64_t pv = 0;  // candidates j < pv only (0: all; the bf16-split kernel takes all)
};
void launch_syrk_f64(const double *Xs, int64_t n, int64_t p, double *S, const Screen &sc, hipStream_t s);
void launch_syrk_f32(const float *Xs, int64_t n, int64_t p, float *S, const Screen &sc, hipStream_t s);
void launch_syrk_bf16x3(const uint16_t *hi, const uint16_t *lo, int64_t n, int64_t npad,
                        int64_t p, float *S, const Screen &sc, hipStream_t s);

// ---------------------------------------------------------------------------
// Grouped launches: one launch runs the same step of many problems (the
// batched entry point).  Work items of problem d are g in [off[d], off[d+1])
// (off has nd + 1 entries); a block or wave finds its problem by bisection.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int group_of(const int64_t *off, int nd, int64_t g)
{
    int lo = 0, hi = nd;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// off[0] = 0, off[d + 1] = off[d] + max(0, cnt[d * stride]) for d < nd: the
// offsets of work lists whose lengths are device counts (one per problem).
void launch_group_offsets(const int *cnt, int64_t stride, int nd, int64_t *off, hipStream_t s);

// One problem's covariance tiles (the mixed form's kernel).
struct SyrkJob {
    const uint16_t *hi, *lo;
    int64_t npad, p;
    float *S;
    int Tt;
    float invn, thr;
    int *scnt, *sidx;
};
// One problem's covariance tiles (the double and float forms' kernel).
template <typename T>
struct SyrkJobT {
    const T *Xs;
    int64_t n, p;
    T *S;
    int Tt;
    T invn, thr;
    int64_t pv;
    int *scnt, *sidx;
};
// Tiles of `edge` (the double form: 128 or 64, see syrk_f64_edge; float: 64).
int syrk_f64_edge(int64_t p);
template <typename T>
SyrkJobT<T> syrk_job_mfma(const T *Xs, int64_t n, int64_t p, T *S, const Screen &sc, int edge, int64_t *tiles);
template <typename T>
void launch_syrk_mfma_grouped(const SyrkJobT<T> *tab, const int64_t *tile_off, int nd, int64_t tiles, int edge,
                              hipStream_t s);
SyrkJob syrk_job_bf16x3(const uint16_t *hi, const uint16_t *lo, int64_t n, int64_t npad, int64_t p, float *S,
                        const Screen &sc, int64_t *tiles);
void launch_syrk_bf16x3_grouped(const SyrkJob *tab, const int64_t *tile_off, int nd, int64_t tiles,
                                hipStream_t s);

// Per-column working-set scaled lasso (see colsolve.hip).
template <typename T>
struct ColArgs {
    const T *S;          // p x p row-major, symmetric, unit diagonal
    int64_t p;
    T lambda0;
    T tol;               // delta: inner stop on max |change|, outer on |d sigma|
    T kkt_tol;           // a variable outside the working set violates when |g| > lambda + kkt_tol
    T band;              // record j off the support with |g| > lambda - band (0: off)
    int max_outer, max_sweeps, max_rounds;
    int mode;            // 0: fresh (screen + solve); 1: resume from the stored state
    int64_t k0;          // fresh mode: the columns k0 .. p-1 are solved (0: all)
    int64_t pv;          // candidate variables j < pv (p: all; smaller when the
                         // last columns are responses only, not predictors)
    int defer_kkt;       // fresh mode: stop after the first solve (the row-tiled pass checks)
    int screened;        // fresh mode: pend_cnt / pend_idx hold the screen (see Screen)
    int warm;            // the stored state holds a warm start (launch_warm_start)
    const int *work_list;// resume mode: columns work_list[0 .. *work_cnt)
    const int *work_cnt;
    int *w_cnt;          // [p]
    int *w_idx;          // [p * kWMax], ascending
    T *w_beta;           // [p * kWMax]
    double *sigma;       // [p]
    double *lam_used;    // [p] lambda the stored coefficients solve
    int *col_status;     // [p]
    int *supp_cnt;       // [p] support of the stored coefficients, slot-major:
    int *supp_idx;       // supp_idx[q * p + k], q < supp_cnt[k]
    T *supp_val;
    int *pend_cnt;       // [p] violators handed between phases
    int *pend_idx;       // [p * kPendMax]
    int *band_cnt;       // [p] or null
    int *band_idx;       // [p * kBandMax] or null
    int *esc_cnt;        // escalation queue (32 -> 128 working set)
    int *esc_list;       // [p]
    int *dense_cnt;      // escalation queue (128 -> the dense tier)
    int *dense_list;     // [p]
    int *colinfo;        // [p * 4] per column: sigma updates, sweeps, updates, rounds
    unsigned long long *counters;
    const int *flags;    // nonzero: bad input, every wave exits at once
};
// tier: 0 = 32-wide working sets (escalating), 1 = 128-wide
template <typename T>
void launch_colsolve(const ColArgs<T> &a, int tier, hipStream_t s);
// The first solves of many problems (columns off[d] .. off[d+1] - 1 are the
// columns of problem d), and the list-driven solves (re-solves: tier 0;
// escalations: tier 1) whose lists' offsets off are device prefix sums.
template <typename T>
void launch_colsolve_first_grouped(const ColArgs<T> *tab, const int64_t *off, int nd, int64_t total,
                                   hipStream_t s);
template <typename T>
void launch_colsolve_list_grouped(const ColArgs<T> *tab, const int64_t *off, int nd, int tier, hipStream_t s);

// Columns whose working sets outgrow the 128-coordinate LDS tier (see
// dense.hip): where their start comes from ...
template <typename TS>
struct DenseSrc {
    const int *cnt;       // [p] start-list lengths (> kWMax: the list is in the pool at off[k]);
                          // null: every column starts from beta = 0 (and sigma = 1 without `sigma`)
    const int *idx;       // lists: column k at k * kWMax, or at p * kWMax + off[k]
    const TS *beta;
    const int *off;       // [p] pool offsets (read only for lists longer than kWMax)
    const double *sigma;  // [p] start sigma
    const int *pend_cnt;  // [p] extra candidates (kPendMax per column), or null
    const int *pend_idx;
};
// ... and what the tier needs and writes.
template <typename T>
struct DenseArgs {
    const T *S;           // p x p covariance (S source), or null with ...
    const double *Xt;     // ... p x n standardised data (data source; T = double)
    int64_t n, p;
    int64_t pv;           // candidate variables j < pv (p for SPMESL)
    T lambda0, tol, kkt_tol;
    int max_outer, max_sweeps, max_rounds;
    int block;            // b: rows per block of the delayed update (16 .. 64)
    const int *queue;     // columns queue[0 .. *qcnt), or (null) the columns 0 .. ncols - 1
    const int *qcnt;
    int64_t ncols;
    int *w_cnt, *w_idx;   // results: nonzeros in ascending order, at k * kWMax,
    T *w_beta;            // or (more than kWMax) at p * kWMax + w_off[k] in the pool
    int *w_off;
    double *sigma, *lam_used;
    int *col_status;
    int *pool_cnt;        // entries of the pool taken
    int64_t pool_cap;
    int *band_cnt;        // null, or set to kBandMax + 1 (the polish takes its full pass)
    int *info;            // per-column counters (stride 4: outer, sweeps, updates,
    int info_stride;      // KKT passes; stride 8 adds the rows added), accumulated
    // workspace, one slice per workgroup (workgroup w takes the groups w,
    // w + G, ... of the G launched):
    int *mark;            // [p] per slice
    int *V, *Vold;        // [vcap] per slice
    T *R, *Bd, *Bp, *sk;  // [vcap * 16] per slice
    int64_t vcap;         // the most rows V may hold (a group beyond it fails)
    double *Svv;          // [svv_cap^2] per slice (data source)
    int64_t svv_cap;
    double *E;            // [16 * n] per slice (data source)
    unsigned long long *counters;
    const int *flags;
};
template <typename T, typename TS>
void launch_dense(const DenseArgs<T> &a, const DenseSrc<TS> &src, hipStream_t s, int blocks = 1);

// Warm start of the column solves from a caller's B0 (p x p row-major,
// column k = beta of response k) and sigma0 (p), on the standardised scale or
// (original != 0) on the data's scale, mapped by Proposition 1 with scale
// c: b_jk = b0_jk c_k / c_j, sigma_k = sigma0_k c_k.  Writes each column's
// stored state: the nonzeros of column k of B0 off the diagonal in ascending
// j (at most kWMax), sigma (1 where sigma0 is null or not a positive finite
// number), lambda = sigma lambda0, and the status kColWarm.  Either pointer
// may be null.
template <typename T>
void launch_warm_start(const double *B0, const double *sigma0, int64_t p, const double *scale,
                       int original, double lambda0, int *w_cnt, int *w_idx, T *w_beta, double *sigma,
                       double *lam_used, int *col_status, hipStream_t s);

// Row-tiled KKT pass over every column: stage rows of S in LDS once, check
// g_jk = s_jk - sum_l S_jl beta_lk for all (j, k) (see kkt.hip).
template <typename T>
struct KktArgs {
    const T *S;
    int64_t p;
    T kkt_tol, band;
    const double *lam_used;
    const int *col_status;
    const int *w_cnt, *w_idx;
    const int *supp_cnt, *supp_idx;
    const T *supp_val;
    int *pend_cnt, *pend_idx;
    int *dirty_cnt, *dirty_list;
    int *band_cnt, *band_idx;
    const int *flags;
};
// rows per block that fit `lds_budget` bytes, 0 if one row does not fit
int kkt_rows_per_block(int64_t p, size_t elem, size_t lds_budget);
template <typename T>
void launch_kkt_rows(const KktArgs<T> &a, int rj, hipStream_t s);
// One problem's share of a grouped row-tiled pass: its arguments, rows per
// block and tile stride; kkt_job also gives the problem's block count.
template <typename T>
struct KktJob {
    KktArgs<T> a;
    int64_t rpb, bstride;
};
template <typename T>
KktJob<T> kkt_job(const KktArgs<T> &a, int rj, int64_t *blocks);
template <typename T>
void launch_kkt_rows_grouped(const KktJob<T> *tab, const int64_t *off, int nd, int64_t blocks, int rj,
                             int64_t pmax, hipStream_t s);

// Double-precision polish of the float solution (mixed form).
struct PolishArgs {
    const double *Xt;       // p x n standardised data (double)
    const float *S32;       // p x p float covariance (for full KKT passes)
    int64_t n, p;
    double lambda0, tol;
    int max_outer, max_sweeps, max_rounds;
    float band;             // band the float solve recorded
    const int *w_cnt32;     // float solution
    const int *w_idx32;
    const float *w_beta32;
    const double *sigma32;
    const double *lam32;
    const int *band_cnt;
    const int *band_idx;
    const int *col_status32;
    double eps;             // bound on |g32 - g64| per unit of (1 + ||beta||_1)
    int *esc_cnt;           // escalation queue (32 -> 128 working set)
    int *esc_list;
    int *dense_cnt;         // escalation queue (128 -> the dense tier)
    int *dense_list;
    int *w_cnt;             // double solution (output)
    int *w_idx;
    double *w_beta;
    double *sigma;
    double *lam_used;
    int *col_status;
    int *polinfo;           // [p * 8] per column: sigma updates, sweeps, updates, checks, added
    const int *flags;
    int full_kkt;           // 1: every column takes the full KKT pass (no band bound)
};
void launch_polish(const PolishArgs &a, hipStream_t s);
// The polish of many problems: every column (tier2 = 0; off: the problems'
// column offsets, total: all columns), or the escalated columns (tier2 = 1;
// off: device prefix sums of the problems' escalation counts, total: an upper
// bound, which sets the grid).
void launch_polish_grouped(const PolishArgs *tab, const int64_t *off, int nd, int64_t total, int tier2,
                           hipStream_t s);

// Reduce the per-column counters and final statuses of one solve into the
// control block: counters[kNumCounters] and status bits (1 no convergence,
// 2 degenerate, 4 working set overflow).
void launch_reduce_stats(int64_t p, const int *colinfo, const int *polinfo, const int *w_cnt,
                         const int *col_status, unsigned long long *counters, int *status_bits,
                         hipStream_t s);

// Zero n 32-bit words (a kernel, so it is safe inside captured graphs).
void launch_zero_words(uint32_t *a, int64_t n, hipStream_t s);

// Outputs.
void launch_fill_zero(double *A, int64_t count, hipStream_t s, int max_blocks = 64);
template <typename T>
void launch_scatter_outputs(int64_t p, const int *w_cnt, const int *w_idx, const T *w_beta, const int *w_off,
                            const double *sigma, const double *scale, int original_scale,
                            double *B, double *sig_out, double *Omega, const int *flags,
                            hipStream_t s);
void launch_symmetrize_dense(int64_t p, const double *Om1, double *Om, hipStream_t s);
template <typename T>
void launch_scatter_lasso(int64_t k0, int64_t m, const int *w_cnt, const int *w_idx, const T *w_beta,
                          const int *w_off, const double *sigma, const double *scale, int original_scale,
                          const int *colinfo, double *beta, double *sig_out, int *outer,
                          const int *flags, hipStream_t s);

} // namespace spmesl
