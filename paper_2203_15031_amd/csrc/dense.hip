// dense.hip -- the regressions whose working sets outgrow the LDS tiers.
//
// A column whose working set would exceed the 128 coordinates an LDS tier
// holds is finished here.  Algorithm 1 puts no bound on the support, so
// neither does this tier: it runs the paper's row-wise PCD (Proposition 2,
// Algorithm 3) in covariance form on a group of up to 16 such columns at
// once, restricted to the union V of their working sets:
//
//   R = S[V, K] - S[V, V] B[V, K]          (gradients of the group's columns K)
//   for each block J of b consecutive rows of V (ascending):
//       every column sweeps J in order on its own: a = R_j + B_j,
//       B_j <- Soft_lambda(a), R_J -= S[J, j] delta_j  (in-wave, S[J, J] in LDS)
//       R -= S[V, J] dB[J, K]                 (the delayed rank-b update,
//                                              on the matrix cores)
//
// Within a column this is the cyclic order of Algorithm 1 exactly (the rows
// of V are visited in ascending order and every coordinate sees every
// earlier change), so the iterates are the same as coordinate descent on V;
// only the gradients of rows outside the current block are brought up to
// date once per block.  Each column keeps its own inner stop (largest
// change of a sweep < tol), noise update sigma^2 = 1 - B'(s + R) (Eq.
// (eq:sigma) from S) and outer stop; columns that are done stay in the group
// with zero changes.  When every column is done, one pass over all p rows
// computes the full gradient g = s_k - S[:, V] B[V, k] (again on the matrix
// cores) and every j outside V with |g_j| > lambda + tol joins V; the group
// repeats until no column has a violator.
//
// Two sources of S:
//   * the covariance S itself (double or float forms, and the float stage of
//     the mixed form): entries are gathered from S;
//   * the standardised data Xt (p x n, double) for the double polish of the
//     mixed form: S[V, V] and s are formed once per V on the matrix cores, and
//     the full gradient is taken in the data form of Algorithm 3,
//     E = x_K - X_V B[V, K] and g = X^T E / n (so no double S is needed).
//
// One workgroup of 16 waves (wave c works for column c of the group) takes
// the groups one after another; the tier is rare (none of the benchmark's
// columns reach it) and its groups are small.
#include "colsolve_dev.hpp"

namespace spmesl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct DAcc;
template <> struct DAcc<double> { typedef d4 type; };
template <> struct DAcc<float> { typedef f4 type; };

__device__ __forceinline__ d4 dmfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 dmfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of accumulator element r of `lane` in a 16 x 16 block: D[4r + l/16]
// for the double MFMA, D[4(l/16) + r] for the float one (lane l holds
// column l % 16; it supplies row l % 16 of A and column l % 16 of B at
// k-block l / 16).
template <typename T> __device__ __forceinline__ int drow(int lane, int r);
template <> __device__ __forceinline__ int drow<double>(int lane, int r) { return 4 * r + (lane >> 4); }
template <> __device__ __forceinline__ int drow<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

// acc += A (16 x K) B (K x 16); fa(r, k) and fb(k, c) give the operands
// (only called with 0 <= k < K).  U k-steps per round, loads first.
template <typename T, int U = 2, typename FA, typename FB>
__device__ __forceinline__ typename DAcc<T>::type tile_mma(typename DAcc<T>::type acc, int64_t K, FA fa, FB fb)
{
    const int l = lane_id();
    const int r = l & 15, kq = l >> 4;
    for (int64_t k0 = 0; k0 < K; k0 += 4 * U) {
        T a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + 4 * u + kq;
            const bool in = k < K;
            a[u] = in ? fa(r, k) : T(0);
            b[u] = in ? fb(k, r) : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc = dmfma(a[u], b[u], acc);
    }
    return acc;
}

constexpr int kDW = 16;      // columns per group (the MFMA tile's 16 columns)
constexpr int kNW = 8;       // waves per workgroup; wave w works for columns w and w + 8
constexpr int kCPW = kDW / kNW;
constexpr int kDT = kWave * kNW;
constexpr int kBMax = 64;    // rows per block at most (one lane each)

enum : int { kDSweep = 0, kDDone = 1, kDFail = 2 };

template <typename T>
struct DenseSm {
    T sjj[kBMax][kBMax + 1];  // S[J, J] of the current block
    T db[kBMax][kDW];         // the block's changes, column by column
    int ck[kDW];              // the group's columns
    T sig[kDW], lam[kDW];
    int state[kDW], status[kDW];
    int outer[kDW], sweeps[kDW], lsweeps[kDW], updates[kDW], checks[kDW], added[kDW];
    int have[kDW];            // secant step: the last update was a fresh one ...
    T sp[kDW], hp[kDW];       // ... at sigma sp, giving h(sp) = hp (B then in Bp)
    int viol;                 // bit c: column c has a violator
    int scan[kNW];
    int nv;
    int refresh;              // some column updated sigma: recompute R
};

// Block-wide compaction of the rows marked in `mark` (in ascending order)
// into V; every marked row becomes 1.  Returns |V|.
template <typename T>
__device__ int build_v(const DenseArgs<T> &A, DenseSm<T> &sm)
{
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    int base = 0;
    for (int64_t j0 = 0; j0 < A.p; j0 += kDT) {
        const int64_t j = j0 + tid;
        const bool f = j < A.p && A.mark[j] != 0;
        const unsigned long long m = __ballot(f);
        if (lane == 0) sm.scan[wv] = __popcll(m);
        __syncthreads();
        int off = base, tot = 0;
        for (int w = 0; w < kNW; ++w) {
            off += w < wv ? sm.scan[w] : 0;
            tot += sm.scan[w];
        }
        if (f) {
            A.V[off + lanes_below(m)] = (int)j;
            A.mark[j] = 1;
        }
        base += tot;
        __syncthreads();
    }
    return base;
}

// position of row j in V[0 .. nv) (j is in V)
__device__ __forceinline__ int v_pos(const int *V, int nv, int j)
{
    int lo = 0, hi = nv;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (V[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// S[V[a], V[b]]
template <typename T, bool DATA>
__device__ __forceinline__ T s_vv(const DenseArgs<T> &A, int nv, int64_t a, int64_t b)
{
    if constexpr (DATA) return (T)A.Svv[a * nv + b];
    else return A.S[(int64_t)A.V[a] * A.p + A.V[b]];
}

// For the data source: S[V, V] and s = S[V, K] of the current V on the
// matrix cores (from Xt), unit diagonal.  For S itself: s gathered.
template <typename T, bool DATA>
__device__ void form_s(const DenseArgs<T> &A, DenseSm<T> &sm, int nv, int m)
{
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int64_t n = A.n;
    const int tv = (nv + 15) / 16;
    if constexpr (DATA) {
        const double invn = 1.0 / (double)n;
        const double *Xt = A.Xt;
        for (int t = wv; t < tv * tv; t += kNW) {
            const int a0 = (t / tv) * 16, b0 = (t % tv) * 16;
            d4 acc = {0, 0, 0, 0};
            const int ra = a0 + (lane & 15) < nv ? A.V[a0 + (lane & 15)] : 0;
            const int rb = b0 + (lane & 15) < nv ? A.V[b0 + (lane & 15)] : 0;
            acc = tile_mma<double>(acc, n, [&](int, int64_t k) { return Xt[(int64_t)ra * n + k]; },
                                   [&](int64_t k, int) { return Xt[(int64_t)rb * n + k]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = a0 + drow<double>(lane, r), b = b0 + (lane & 15);
                if (a < nv && b < nv) A.Svv[(int64_t)a * nv + b] = a == b ? 1.0 : acc[r] * invn;
            }
        }
        for (int t = wv; t < tv; t += kNW) {
            const int a0 = t * 16;
            d4 acc = {0, 0, 0, 0};
            const int ra = a0 + (lane & 15) < nv ? A.V[a0 + (lane & 15)] : 0;
            const int cc = (lane & 15) < m ? sm.ck[lane & 15] : 0;
            acc = tile_mma<double>(acc, n, [&](int, int64_t k) { return Xt[(int64_t)ra * n + k]; },
                                   [&](int64_t k, int) { return Xt[(int64_t)cc * n + k]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = a0 + drow<double>(lane, r), c = lane & 15;
                if (a < nv) A.sk[(int64_t)a * kDW + c] = (T)(c < m ? (A.V[a] == sm.ck[c] ? 1.0 : acc[r] * invn) : 0.0);
            }
        }
    } else {
        for (int64_t e = threadIdx.x; e < (int64_t)nv * kDW; e += kDT) {
            const int a = (int)(e / kDW), c = (int)(e % kDW);
            A.sk[e] = c < m ? A.S[(int64_t)A.V[a] * A.p + sm.ck[c]] : T(0);
        }
    }
}

// R = s - S[V, V] B[V, K] for all rows of V (fresh, no accumulated rounding)
template <typename T, bool DATA>
__device__ void fresh_r(const DenseArgs<T> &A, int nv)
{
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int tv = (nv + 15) / 16;
    for (int t = wv; t < tv; t += kNW) {
        const int a0 = t * 16;
        typename DAcc<T>::type acc = {0, 0, 0, 0};
        const int ra = a0 + (lane & 15);
        acc = tile_mma<T>(acc, nv, [&](int, int64_t k) { return ra < nv ? s_vv<T, DATA>(A, nv, ra, k) : T(0); },
                          [&](int64_t k, int c) { return A.Bd[k * kDW + c]; });
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = a0 + drow<T>(lane, r), c = lane & 15;
            if (a < nv) A.R[(int64_t)a * kDW + c] = A.sk[(int64_t)a * kDW + c] - acc[r];
        }
    }
}

// The full gradient over all p rows for the group's columns; every j outside
// V with |g_j| > lambda_c + kkt_tol is marked 2 and sets bit c of sm.viol.
template <typename T, bool DATA>
__device__ void kkt_all(const DenseArgs<T> &A, DenseSm<T> &sm, int nv, int m)
{
    const int lane = lane_id(), wv = threadIdx.x / kWave;
    const int64_t p = A.p;
    const int tp = (int)((p + 15) / 16);
    if constexpr (DATA) {
        // E = x_K - X_V B[V, K]  (16 x n), then g = Xt E^T / n
        const int64_t n = A.n;
        const double *Xt = A.Xt;
        const int tn = (int)((n + 15) / 16);
        for (int t = wv; t < tn; t += kNW) {
            const int64_t i0 = (int64_t)t * 16;
            d4 acc = {0, 0, 0, 0};
            const int64_t ii = i0 + (lane & 15);
            acc = tile_mma<double>(acc, nv, [&](int c, int64_t k) { return (double)A.Bd[k * kDW + c]; },
                                   [&](int64_t k, int) { return ii < n ? Xt[(int64_t)A.V[k] * n + ii] : 0.0; });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = drow<double>(lane, r);
                if (ii < n) A.E[(int64_t)c * n + ii] = c < m ? Xt[(int64_t)sm.ck[c] * n + ii] - acc[r] : 0.0;
            }
        }
        __syncthreads();
        const double invn = 1.0 / (double)n;
        for (int t = wv; t < tp; t += kNW) {
            const int64_t j0 = (int64_t)t * 16;
            const int64_t jr = j0 + (lane & 15) < p ? j0 + (lane & 15) : p - 1;
            d4 acc = {0, 0, 0, 0};
            acc = tile_mma<double>(acc, n, [&](int, int64_t k) { return Xt[jr * n + k]; },
                                   [&](int64_t k, int c) { return A.E[(int64_t)c * n + k]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + drow<double>(lane, r);
                const int c = lane & 15;
                if (j < A.pv && c < m && A.mark[j] == 0 && j != sm.ck[c]) {
                    const double g = acc[r] * invn;
                    if ((g < 0.0 ? -g : g) > (double)sm.lam[c] + (double)A.kkt_tol) {
                        A.mark[j] = 2;
                        atomicOr(&sm.viol, 1 << c);
                    }
                }
            }
        }
    } else {
        for (int t = wv; t < tp; t += kNW) {
            const int64_t j0 = (int64_t)t * 16;
            const int64_t jr = j0 + (lane & 15) < p ? j0 + (lane & 15) : p - 1;
            typename DAcc<T>::type acc = {0, 0, 0, 0};
            acc = tile_mma<T>(acc, nv, [&](int, int64_t k) { return A.S[jr * p + A.V[k]]; },
                              [&](int64_t k, int c) { return A.Bd[k * kDW + c]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + drow<T>(lane, r);
                const int c = lane & 15;
                if (j < A.pv && c < m && A.mark[j] == 0 && j != sm.ck[c]) {
                    const T g = A.S[j * p + sm.ck[c]] - acc[r];
                    if ((g < T(0) ? -g : g) > sm.lam[c] + A.kkt_tol) {
                        A.mark[j] = 2;
                        atomicOr(&sm.viol, 1 << c);
                    }
                }
            }
        }
    }
}

template <typename T, typename TS, bool DATA>
__global__ __launch_bounds__(kDT) void k_dense(DenseArgs<T> A0, DenseSrc<TS> src)
{
    __shared__ DenseSm<T> sm;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    if (*A0.flags) return;
    const int64_t p = A0.p;
    // the queue, or (no queue) the columns 0 .. ncols - 1
    const int q = A0.queue ? *A0.qcnt : (int)A0.ncols;
    if (q <= 0 || (int64_t)blockIdx.x * kDW >= q) return;
    // this workgroup's slice of the workspace
    DenseArgs<T> A = A0;
    {
        const int64_t bi = blockIdx.x, vc = A0.vcap;
        A.mark += bi * p;
        A.V += bi * vc;
        A.Vold += bi * vc;
        A.R += bi * vc * kDW;
        A.Bd += bi * vc * kDW;
        A.Bp += bi * vc * kDW;
        A.sk += bi * vc * kDW;
        if (DATA) {
            A.Svv += bi * A0.svv_cap * A0.svv_cap;
            A.E += bi * (int64_t)kDW * A0.n;
        }
    }
    // V may hold vcap rows (and, from the data, svv_cap)
    const int64_t vlim = DATA && A.svv_cap < A.vcap ? A.svv_cap : A.vcap;
    for (int64_t j = tid; j < p; j += kDT) A.mark[j] = 0;
    __syncthreads();
    const int b = A.block < 16 ? 16 : (A.block > kBMax ? kBMax : A.block);
    for (int g0 = (int)blockIdx.x * kDW; g0 < q; g0 += (int)gridDim.x * kDW) {
        const int m = q - g0 < kDW ? q - g0 : kDW;
        // --- the group's columns and their start --------------------------
        if (tid < kDW) {
            const int c = tid;
            sm.ck[c] = c < m ? (A.queue ? A.queue[g0 + c] : g0 + c) : 0;
            const int64_t k = sm.ck[c];
            double sg = c < m && src.sigma ? src.sigma[k] : 1.0;
            sg = sg > 0.0 && sg < 1e300 ? sg : 1.0;
            sm.sig[c] = (T)sg;
            sm.lam[c] = (T)sg * A.lambda0;
            sm.state[c] = c < m ? kDSweep : kDDone;
            sm.status[c] = kColOk;
            sm.outer[c] = sm.sweeps[c] = sm.lsweeps[c] = sm.updates[c] = sm.checks[c] = sm.added[c] = 0;
            sm.have[c] = 0;
            sm.sp[c] = sm.hp[c] = T(0);
        }
        if (tid == 0) sm.viol = 0;
        __syncthreads();
        // mark the start lists (and pending candidates) of the group's columns
        for (int c = wv; c < m; c += kNW) {
            const int64_t k = sm.ck[c];
            int cnt = src.cnt ? src.cnt[k] : 0;
            cnt = cnt < 0 ? 0 : cnt;
            const int64_t base = cnt > kWMax ? p * (int64_t)kWMax + src.off[k] : k * (int64_t)kWMax;
            for (int i = lane; i < cnt; i += kWave) {
                const int j = src.idx[base + i];
                if (j >= 0 && j < p && j != k) A.mark[j] = 1;
            }
            if (src.pend_cnt) {
                int np = src.pend_cnt[k];
                np = np < 0 ? 0 : (np > kPendMax ? kPendMax : np);
                for (int i = lane; i < np; i += kWave) {
                    const int j = src.pend_idx[k * kPendMax + i];
                    if (j >= 0 && j < p && j != k) A.mark[j] = 1;
                }
            }
        }
        __syncthreads();
        int nv = build_v(A, sm);
        bool gfail = false;
        if ((int64_t)nv > vlim) {
            // V does not fit this workgroup's buffers: the group fails (rare)
            if (tid < m) sm.status[tid] = kColWorkset, sm.state[tid] = kDFail;
            gfail = true;
            nv = 0;
        }
        for (int64_t e = tid; e < (int64_t)nv * kDW; e += kDT) A.Bd[e] = T(0);
        __syncthreads();
        for (int c = wv; c < m && nv > 0; c += kNW) {
            const int64_t k = sm.ck[c];
            int cnt = src.cnt ? src.cnt[k] : 0;
            cnt = cnt < 0 ? 0 : cnt;
            const int64_t base = cnt > kWMax ? p * (int64_t)kWMax + src.off[k] : k * (int64_t)kWMax;
            for (int i = lane; i < cnt; i += kWave) {
                const int j = src.idx[base + i];
                if (j >= 0 && j < p && j != k) A.Bd[(int64_t)v_pos(A.V, nv, j) * kDW + c] = (T)src.beta[base + i];
            }
        }
        __syncthreads();
        int rounds = 0;
        for (;;) {
            // --- S on V, and fresh gradients ------------------------------
            form_s<T, DATA>(A, sm, nv, m);
            __syncthreads();
            fresh_r<T, DATA>(A, nv);
            __syncthreads();
            // --- sweeps until every column is done --------------------------
            for (;;) {
                bool any = false;
                for (int c = 0; c < kDW; ++c) any |= sm.state[c] == kDSweep;
                if (!any) break;
                T maxd[kCPW];
#pragma unroll
                for (int u = 0; u < kCPW; ++u) maxd[u] = T(0);
                for (int v0 = 0; v0 < nv; v0 += b) {
                    const int bb = nv - v0 < b ? nv - v0 : b;
                    for (int e = tid; e < bb * bb; e += kDT) {
                        const int i = e / bb, j = e % bb;
                        sm.sjj[i][j] = s_vv<T, DATA>(A, nv, v0 + i, v0 + j);
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; u < kCPW; ++u) {
                        const int c = wv + u * kNW;
                        T d = T(0);
                        if (c < m && sm.state[c] == kDSweep) {
                            const bool valid = lane < bb;
                            const int64_t v = v0 + lane;
                            const bool excl = !valid || A.V[valid ? v : 0] == sm.ck[c];
                            T r = valid ? A.R[v * kDW + c] : T(0);
                            T beta = valid ? A.Bd[v * kDW + c] : T(0);
                            const T lam = sm.lam[c];
                            int pos = 0;
                            int nupd = 0;
                            for (;;) {
                                const T nb = excl ? beta : soft_threshold(r + beta, lam);
                                const bool ch = valid && lane >= pos && nb != beta;
                                const unsigned long long mk = __ballot(ch);
                                if (!mk) break;
                                const int j = __builtin_ffsll((long long)mk) - 1;
                                const T dd = bcast(nb - beta, j);
                                if (lane == j) {
                                    beta = nb;
                                    d = dd;
                                }
                                r -= (valid ? sm.sjj[lane][j] : T(0)) * dd;
                                const T ad = dd < T(0) ? -dd : dd;
                                maxd[u] = ad > maxd[u] ? ad : maxd[u];
                                ++nupd;
                                pos = j + 1;
                            }
                            if (valid && d != T(0)) A.Bd[v * kDW + c] = beta;
                            if (lane == 0) sm.updates[c] += nupd;
                        }
                        if (lane < kBMax) sm.db[lane][c] = lane < bb ? d : T(0);
                    }
                    __syncthreads();
                    // delayed rank-b update of every row of V
                    {
                        const int tv = (nv + 15) / 16;
                        for (int t = wv; t < tv; t += kNW) {
                            const int a0 = t * 16;
                            typename DAcc<T>::type acc;
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int a = a0 + drow<T>(lane, r);
                                acc[r] = a < nv ? A.R[(int64_t)a * kDW + (lane & 15)] : T(0);
                            }
                            const int ra = a0 + (lane & 15);
                            acc = tile_mma<T>(acc, bb,
                                              [&](int, int64_t k) {
                                                  return ra < nv ? -s_vv<T, DATA>(A, nv, ra, v0 + k) : T(0);
                                              },
                                              [&](int64_t k, int c) { return sm.db[k][c]; });
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int a = a0 + drow<T>(lane, r);
                                if (a < nv) A.R[(int64_t)a * kDW + (lane & 15)] = acc[r];
                            }
                        }
                    }
                    __syncthreads();
                }
                // --- per column: inner stop, noise update, outer stop -------
                // Algorithm 1's noise update, with the secant step of the LDS
                // tiers: two fresh updates on one support and one sign
                // pattern give the fixed point of the affine model
                // h(sigma)^2 = C0 + C2 sigma^2, and B moves along its affine
                // path to it (the stopping test stays the plain one).  Every
                // lane of the column's wave takes the same decisions; lane 0
                // records them.
                if (tid == 0) sm.refresh = 0;
                __syncthreads();
#pragma unroll
                for (int u = 0; u < kCPW; ++u) {
                    const int c = wv + u * kNW;
                    if (!(c < m && sm.state[c] == kDSweep)) continue;
                    const bool inner = maxd[u] < A.tol;
                    T s2 = T(1);
                    bool same = false;
                    if (inner) {
                        T part = T(0);
                        bool diff = false;
                        for (int v = lane; v < nv; v += kWave) {
                            const int64_t e = (int64_t)v * kDW + c;
                            const T bv = A.Bd[e], pv = A.Bp[e];
                            part += bv * (A.sk[e] + A.R[e]);
                            diff |= (bv > T(0)) != (pv > T(0)) || (bv < T(0)) != (pv < T(0));
                        }
                        s2 = T(1) - wave_sum(part);
                        same = __ballot(diff) == 0ull;
                    }
                    const T so = sm.sig[c];
                    const int ls = sm.lsweeps[c] + 1;
                    const int outer = sm.outer[c] + (inner ? 1 : 0);
                    int state = kDSweep, status = kColOk;
                    T sig = so, f = T(0);
                    bool next = false;  // a new lasso at a new sigma follows
                    if (inner) {
                        if (!(s2 > DegenerateFloor<T>::v)) {
                            sig = s2 > T(0) ? sqrt(s2) : T(0);
                            status = kColDegenerate;
                            state = kDFail;
                        } else {
                            const T sn = sqrt(s2);
                            T ds = sn - so;
                            ds = ds < T(0) ? -ds : ds;
                            sig = sn;
                            if (ds < A.tol) {
                                state = kDDone;
                            } else if (outer >= A.max_outer) {
                                status = kColNoconv;
                                state = kDFail;
                            } else {
                                next = true;
                                if (sm.have[c] && same) {
                                    const T spv = sm.sp[c], hpv = sm.hp[c];
                                    const T c2 = (sn * sn - hpv * hpv) / (so * so - spv * spv);
                                    const T c0 = sn * sn - c2 * so * so;
                                    T dsp = so - spv;
                                    dsp = dsp < T(0) ? -dsp : dsp;
                                    if (dsp > T(64) * Eps<T>::v * so && c2 >= T(0) && c2 < T(1) && c0 > T(0)) {
                                        const T ss = sqrt(c0 / (T(1) - c2));
                                        T jump = ss - sn;
                                        jump = jump < T(0) ? -jump : jump;
                                        if (jump <= T(16) * ds) {
                                            f = (ss - so) / (so - spv);
                                            sig = ss;
                                        }
                                    }
                                }
                            }
                        }
                    } else if (ls >= A.max_sweeps) {
                        status = kColNoconv;
                        state = kDFail;
                    }
                    if (next) {
                        // the step (when taken), then B is the next update's Bp
                        for (int v = lane; v < nv; v += kWave) {
                            const int64_t e = (int64_t)v * kDW + c;
                            T bv = A.Bd[e];
                            if (f != T(0)) {
                                bv += f * (bv - A.Bp[e]);
                                A.Bd[e] = bv;
                            }
                            A.Bp[e] = bv;
                        }
                    }
                    if (lane == 0) {
                        ++sm.sweeps[c];
                        sm.lsweeps[c] = inner ? 0 : ls;
                        sm.outer[c] = outer;
                        sm.sig[c] = sig;
                        sm.state[c] = state;
                        sm.status[c] = status;
                        if (next) {
                            sm.lam[c] = sig * A.lambda0;
                            sm.have[c] = f == T(0);
                            sm.sp[c] = so;
                            sm.hp[c] = sqrt(s2);
                            sm.refresh = 1;
                        }
                    }
                }
                __syncthreads();
                // new lambdas: gradients recomputed from scratch (no drift)
                if (sm.refresh) {
                    fresh_r<T, DATA>(A, nv);
                    __syncthreads();
                }
            }
            // --- KKT over all p rows -----------------------------------------
            bool any_done = false;
            for (int c = 0; c < m; ++c) any_done |= sm.state[c] == kDDone;
            if (!any_done || gfail) break;
            if (tid == 0) sm.viol = 0;
            __syncthreads();
            kkt_all<T, DATA>(A, sm, nv, m);
            __syncthreads();
            const int viol = sm.viol;
            if (tid < m && sm.state[tid] == kDDone) {
                ++sm.checks[tid];
                if (viol & (1 << tid)) {
                    if (rounds >= A.max_rounds) {
                        sm.status[tid] = kColNoconv;
                        sm.state[tid] = kDFail;
                    } else {
                        sm.state[tid] = kDSweep;
                    }
                }
            }
            __syncthreads();
            if (!viol || rounds >= A.max_rounds) {
                // rows marked 2 were not taken: clear them
                for (int64_t j = tid; j < p; j += kDT)
                    if (A.mark[j] == 2) A.mark[j] = 0;
                __syncthreads();
                break;
            }
            ++rounds;
            // --- V grows: move B to the new row positions ---------------------
            // (R, rebuilt below, holds the old B meanwhile; Vold the old V)
            const int nv_old = nv;
            for (int64_t e = tid; e < (int64_t)nv_old * kDW; e += kDT) A.R[e] = A.Bd[e];
            for (int64_t e = tid; e < (int64_t)nv_old; e += kDT) A.Vold[e] = A.V[e];
            __syncthreads();
            nv = build_v(A, sm);
            if (tid < m) {
                sm.added[tid] += nv - nv_old;
                sm.have[tid] = 0;  // B moved: the secant needs two fresh updates again
            }
            if ((int64_t)nv > vlim) {
                if (tid < m) sm.status[tid] = kColWorkset, sm.state[tid] = kDFail;
                gfail = true;
                nv = 0;
            }
            for (int64_t e = tid; e < (int64_t)nv * kDW; e += kDT) A.Bd[e] = T(0);
            __syncthreads();
            for (int64_t e = tid; e < (int64_t)nv_old * kDW && nv > 0; e += kDT) {
                const int a = (int)(e / kDW), c = (int)(e % kDW);
                const T v = A.R[e];
                if (v != T(0)) A.Bd[(int64_t)v_pos(A.V, nv, A.Vold[a]) * kDW + c] = v;
            }
            __syncthreads();
            if (gfail) break;
        }
        // --- results: the nonzeros of each column, ascending ---------------
        for (int c = wv; c < m; c += kNW) {
            const int64_t k = sm.ck[c];
            int cnt = 0;
            for (int v0 = 0; v0 < nv; v0 += kWave) {
                const int v = v0 + lane;
                const bool nz = v < nv && A.Bd[(int64_t)v * kDW + c] != T(0);
                cnt += __popcll(__ballot(nz));
            }
            int status = sm.status[c];
            int64_t base = k * (int64_t)kWMax;
            if (cnt > kWMax) {
                int off = 0;
                if (lane == 0) off = atomicAdd(A.pool_cnt, cnt);
                off = __shfl(off, 0);
                if ((int64_t)off + cnt > A.pool_cap) {
                    status = kColWorkset;
                    cnt = kWMax;
                } else {
                    base = p * (int64_t)kWMax + off;
                    if (lane == 0) A.w_off[k] = off;
                }
            }
            int pos = 0;
            for (int v0 = 0; v0 < nv && pos < cnt; v0 += kWave) {
                const int v = v0 + lane;
                const T bv = v < nv ? A.Bd[(int64_t)v * kDW + c] : T(0);
                const bool nz = bv != T(0);
                const unsigned long long mk = __ballot(nz);
                const int at = pos + lanes_below(mk);
                if (nz && at < cnt) {
                    A.w_idx[base + at] = A.V[v];
                    A.w_beta[base + at] = bv;
                }
                pos += __popcll(mk);
            }
            if (lane == 0) {
                A.w_cnt[k] = cnt;
                A.sigma[k] = (double)sm.sig[c];
                A.lam_used[k] = (double)sm.lam[c];
                A.col_status[k] = status;
                if (A.band_cnt) A.band_cnt[k] = kBandMax + 1;
                int *ci = A.info + k * A.info_stride;
                if (A.info_stride == 4) {
                    ci[0] += sm.outer[c];
                    ci[1] += sm.sweeps[c];
                    ci[2] += sm.updates[c];
                    ci[3] += sm.checks[c];
                } else {
                    ci[0] += sm.outer[c];
                    ci[1] += sm.sweeps[c];
                    ci[2] += sm.updates[c];
                    ci[3] += sm.checks[c];
                    ci[4] += sm.added[c];
                }
                atomicAdd(&A.counters[kCntDense], 1ull);
            }
        }
        // clear the marks of V for the next group
        for (int64_t e = tid; e < (int64_t)nv; e += kDT) A.mark[A.V[e]] = 0;
        __syncthreads();
    }
}

} // namespace

template <typename T, typename TS>
void launch_dense(const DenseArgs<T> &a, const DenseSrc<TS> &src, hipStream_t s, int blocks)
{
    if constexpr (sizeof(T) == 8) {
        if (a.Xt) {
            hipLaunchKernelGGL((k_dense<T, TS, true>), dim3(blocks), dim3(kDT), 0, s, a, src);
            return;
        }
    }
    hipLaunchKernelGGL((k_dense<T, TS, false>), dim3(blocks), dim3(kDT), 0, s, a, src);
}

template void launch_dense<double, double>(const DenseArgs<double> &, const DenseSrc<double> &, hipStream_t, int);
template void launch_dense<float, float>(const DenseArgs<float> &, const DenseSrc<float> &, hipStream_t, int);
template void launch_dense<double, float>(const DenseArgs<double> &, const DenseSrc<float> &, hipStream_t, int);

} // namespace spmesl
