// colsolve_dev.hpp -- device routines of the per-column scaled-lasso solver,
// shared by the float/double solve and the double-precision polish.
#pragma once
#include "common.hpp"

namespace spmesl {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename T> struct DegenerateFloor;
template <> struct DegenerateFloor<double> { static constexpr double v = 1e-12; };
template <> struct DegenerateFloor<float> { static constexpr float v = 1e-6f; };
template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 0x1p-52; };
template <> struct Eps<float> { static constexpr float v = 0x1p-23f; };

// LDS of one wave.
template <typename T, int LW>
struct WaveSm {
    T sww[LW * LW];      // sww[q * LW + i] = S[W_i][W_q]
    int widx[LW];        // W, ascending
    T wbeta[LW];
    int tidx[LW];        // merge scratch
    T tbeta[LW];
    int sidx[LW];        // support (nonzero beta), ascending
    T sval[LW];
    int pend[kPendMax];  // violators found by the last KKT pass, ascending
};

template <typename T, int LW>
struct ColState {
    static constexpr int NS = (LW + kWave - 1) / kWave;  // slots per lane
    // working sets of up to 32 keep lane i's row of S_WW in registers,
    // indexed by the (wave-uniform) coordinate being updated
    static constexpr bool kRegRows = LW <= 32;
    static constexpr int kRows = kRegRows ? LW : 1;
    static constexpr int kRowsHi = (kRegRows && sizeof(T) == 8) ? LW : 1;
    T g[NS], b[NS], sv[NS];
    int w;
    T sigma, lam_used;
};

// Copy lane i's row of S_WW from LDS into registers (zero beyond w).
// Register rows: lane i's row of S_WW, indexed by a wave-uniform coordinate.
// The row is held as raw 32-bit words (two arrays for doubles: low and high
// halves) declared directly in the caller; the compiler keeps such arrays in
// registers and indexes them with s_set_gpr_idx, where an array inside a
// struct, or an array of 64-bit elements, goes to scratch.
template <typename T> __device__ __forceinline__ T row_get(const unsigned *lo, const unsigned *hi, int q);
template <> __device__ __forceinline__ float row_get<float>(const unsigned *lo, const unsigned *, int q)
{
    return __uint_as_float(lo[q]);
}
template <> __device__ __forceinline__ double row_get<double>(const unsigned *lo, const unsigned *hi, int q)
{
    return __longlong_as_double(((long long)hi[q] << 32) | (unsigned long long)lo[q]);
}
__device__ __forceinline__ void row_set(unsigned *lo, unsigned *, int q, float x) { lo[q] = __float_as_uint(x); }
__device__ __forceinline__ void row_set(unsigned *lo, unsigned *hi, int q, double x)
{
    long long b = __double_as_longlong(x);
    lo[q] = (unsigned)(b & 0xffffffffll);
    hi[q] = (unsigned)((unsigned long long)b >> 32);
}

template <typename T, int LW>
__device__ __forceinline__ void rows_to_registers(const WaveSm<T, LW> &sm, const ColState<T, LW> &st,
                                                  unsigned *rlo, unsigned *rhi)
{
    if constexpr (ColState<T, LW>::kRegRows) {
        const int lane = lane_id();
        const bool in = lane < st.w;
#pragma unroll
        for (int q = 0; q < LW; ++q) row_set(rlo, rhi, q, (in && q < st.w) ? sm.sww[q * LW + lane] : T(0));
    }
}

// Soft_lambda(a) as a - clamp(a, -lambda, lambda): the same value as the
// branch form (a - lambda, a + lambda or exactly 0).
__device__ __forceinline__ float soft_clamp(float a, float lam)
{
    return a - __builtin_amdgcn_fmed3f(a, -lam, lam);
}
__device__ __forceinline__ double soft_clamp(double a, double lam)
{
    return a - fmax(fmin(a, lam), -lam);
}

// lower_bound over an ascending int array in LDS
__device__ __forceinline__ int lds_lower_bound(const int *a, int n, int v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// KKT pass over all p coordinates of column k.
//   g_j = s_jk - sum_{l in supp} S_jl beta_l, streamed from rows of S.
//   violators: j != k, j not in W, |g_j| > thr    -> sm.pend (ascending)
//   band     : j != k, beta_j == 0, |g_j| > bthr -> band_idx (when recording)
// Returns the number of violators (may exceed kPendMax; only the first
// kPendMax are stored).
//
// Each lane reads V consecutive entries of a row at once (one 16-byte load
// when every row of S is 16-byte aligned, i.e. p a multiple of V), CH such
// groups per trip, and U support rows at a time.
// ---------------------------------------------------------------------------
template <typename TS, int V>
__device__ __forceinline__ void load_group(const TS *__restrict__ src, TS (&x)[V])
{
    if constexpr (V == 1) {
        x[0] = *src;
    } else {
        typedef TS vt __attribute__((ext_vector_type(V)));
        const vt y = *reinterpret_cast<const vt *>(src);
#pragma unroll
        for (int e = 0; e < V; ++e) x[e] = y[e];
    }
}

// Rank of this lane's first element among the flagged elements of a chunk
// taken lane by lane (c: this lane's count, 0..7), and the chunk's total.
__device__ __forceinline__ int lane_prefix(int c, int *total)
{
    int r = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const unsigned long long m = __ballot((c >> b) & 1);
        r += lanes_below(m) << b;
        tot += __popcll(m) << b;
    }
    *total = tot;
    return r;
}

// Block-shared lists of a cooperative KKT pass: the waves of a block take
// contiguous, ascending ranges of j for one column, so the lists
// concatenated in wave order are exactly those one wave would produce.
constexpr int kCoopMax = 4;
struct KktCoop {
    int pend[kCoopMax][kPendMax];
    int npend[kCoopMax];
    int band[kCoopMax][kBandMax];
    int nband[kCoopMax];
};

template <typename TS, typename T, int LW, int V, int CHV, int UV>
__device__ int kkt_pass_v(const TS *__restrict__ S, int64_t p, int64_t jend, int64_t k, WaveSm<T, LW> &sm, int w,
                          int ns, T thr, bool record_band, T bthr, int *band_cnt, int *band_idx,
                          int part, int nparts, KktCoop *cp)
{
    constexpr int CH = V == 1 ? 8 : CHV;
    constexpr int U = V == 1 ? 4 : UV;
    constexpr int STEP = kWave * V * CH;
    const int lane = lane_id();
    const TS *Sk = S + k * p;
    int npend = 0, nband = 0;
    // this wave's violators and band entries (its own lists, or its part of
    // the block's when the pass is shared)
    int *const plist = cp ? cp->pend[part] : sm.pend;
    int *const blist = cp ? cp->band[part] : band_idx + k * kBandMax;
    const int64_t nit = (jend + STEP - 1) / STEP;
    const int64_t it0 = part * nit / nparts, it1 = (part + 1) * nit / nparts;
    for (int64_t base = it0 * STEP; base < it1 * STEP; base += STEP) {
        T acc[CH][V];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int64_t j = base + (int64_t)(c * kWave + lane) * V;
            TS x[V];
            if (j < jend) {
                load_group<TS, V>(Sk + j, x);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) x[e] = TS(0);
            }
#pragma unroll
            for (int e = 0; e < V; ++e) acc[c][e] = (T)x[e];
        }
        for (int t = 0; t < ns; t += U) {
            const TS *rows[U];
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                bool ok = t + u < ns;
                int64_t l = ok ? (int64_t)sm.sidx[t + u] : k;
                l = l < 0 ? 0 : (l >= p ? p - 1 : l);
                v[u] = ok ? sm.sval[t + u] : T(0);
                rows[u] = S + l * p;
            }
            TS x[U][CH][V];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int64_t j = base + (int64_t)(c * kWave + lane) * V;
                    if (j < jend) {
                        load_group<TS, V>(rows[u] + j, x[u][c]);
                    } else {
#pragma unroll
                        for (int e = 0; e < V; ++e) x[u][c][e] = TS(0);
                    }
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < CH; ++c)
#pragma unroll
                    for (int e = 0; e < V; ++e) acc[c][e] -= v[u] * (T)x[u][c][e];
        }
        // chunk by chunk, in ascending j: lane by lane, then element
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int64_t j0 = base + (int64_t)(c * kWave + lane) * V;
            unsigned vm = 0u, bm = 0u;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t j = j0 + e;
                const T aa = acc[c][e] < T(0) ? -acc[c][e] : acc[c][e];
                const bool live = j < jend && j != k;
                if (live && aa > thr) vm |= 1u << e;
                if (record_band && live && aa > bthr) bm |= 1u << e;
            }
            if (vm) {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if ((vm >> e) & 1u) {
                        const int j = (int)(j0 + e);
                        const int pos = lds_lower_bound(sm.widx, w, j);
                        if (pos < w && sm.widx[pos] == j) vm &= ~(1u << e);
                    }
            }
            if (bm) {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if ((bm >> e) & 1u) {
                        const int j = (int)(j0 + e);
                        const int pos = lds_lower_bound(sm.sidx, ns, j);
                        if (pos < ns && sm.sidx[pos] == j) bm &= ~(1u << e);
                    }
            }
            if (__ballot(vm != 0u)) {
                int tot;
                int pos = npend + lane_prefix(__popc(vm), &tot);
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if ((vm >> e) & 1u) {
                        if (pos < kPendMax) plist[pos] = (int)(j0 + e);
                        ++pos;
                    }
                npend += tot;
            }
            if (record_band && __ballot(bm != 0u)) {
                int tot;
                int pos = nband + lane_prefix(__popc(bm), &tot);
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if ((bm >> e) & 1u) {
                        if (pos < kBandMax) blist[pos] = (int)(j0 + e);
                        ++pos;
                    }
                nband += tot;
            }
        }
    }
    if (!cp) {
        if (record_band && lane == 0) band_cnt[k] = nband;
        wave_sync();
        return npend;
    }
    // shared pass: every wave takes the concatenated violators into its own
    // list; part 0 writes the band list of the column
    if (lane == 0) {
        cp->npend[part] = npend;
        cp->nband[part] = nband;
    }
    __syncthreads();
    int tot = 0, btot = 0;
    for (int q = 0; q < nparts; ++q) {
        const int c = cp->npend[q];
        const int cc = c < kPendMax ? c : kPendMax;
        for (int i = lane; i < cc; i += kWave)
            if (tot + i < kPendMax) sm.pend[tot + i] = cp->pend[q][i];
        tot += c;
        if (record_band && part == 0) {
            const int b = cp->nband[q];
            const int bb = b < kBandMax ? b : kBandMax;
            for (int i = lane; i < bb; i += kWave)
                if (btot + i < kBandMax) band_idx[k * kBandMax + btot + i] = cp->band[q][i];
        }
        btot += cp->nband[q];
    }
    if (record_band && part == 0 && lane == 0) band_cnt[k] = btot;
    __syncthreads();  // the shared lists are free for the next pass
    return tot;
}

// CH groups of V per lane in flight and U support rows at a time: the
// defaults keep the register use of the first solves' kernel; the resume
// kernel (few columns) takes deeper settings.
template <typename TS, typename T, int LW, int CH = 4, int U = 2>
__device__ int kkt_pass(const TS *__restrict__ S, int64_t p, int64_t jend, int64_t k, WaveSm<T, LW> &sm, int w,
                        int ns, T thr, bool record_band, T bthr, int *band_cnt, int *band_idx,
                        int part = 0, int nparts = 1, KktCoop *cp = nullptr)
{
    constexpr int V = 16 / sizeof(TS);
    // rows of S start 16-byte aligned when p is a multiple of V (S itself
    // is 256-byte aligned)
    if (p % V == 0)
        return kkt_pass_v<TS, T, LW, V, CH, U>(S, p, jend, k, sm, w, ns, thr, record_band, bthr, band_cnt,
                                              band_idx, part, nparts, cp);
    return kkt_pass_v<TS, T, LW, 1, CH, U>(S, p, jend, k, sm, w, ns, thr, record_band, bthr, band_cnt, band_idx,
                                          part, nparts, cp);
}

// Support list (nonzero coefficients, ascending) from the slot registers.
template <typename T, int LW>
__device__ __forceinline__ int build_support(WaveSm<T, LW> &sm, const ColState<T, LW> &st)
{
    const int lane = lane_id();
    int ns = 0;
#pragma unroll
    for (int s = 0; s < ColState<T, LW>::NS; ++s) {
        int q = s * kWave + lane;
        bool nz = q < st.w && st.b[s] != T(0);
        unsigned long long m = __ballot(nz);
        if (nz) {
            int pos = ns + lanes_below(m);
            sm.sidx[pos] = sm.widx[q];
            sm.sval[pos] = st.b[s];
        }
        ns += __popcll(m);
    }
    wave_sync();
    return ns;
}

// Merge the np ascending, distinct pending candidates into W (ascending),
// with coefficient 0 for the new ones; candidates already in W are dropped.
// Requires w + np <= LW.  Returns the number added.
template <typename T, int LW>
__device__ __forceinline__ int merge_pending(WaveSm<T, LW> &sm, ColState<T, LW> &st, int np)
{
    const int lane = lane_id();
    const int w = st.w;
    // drop members of W (np <= kPendMax = 64: one lane per candidate)
    int v = lane < np ? sm.pend[lane] : 0;
    bool keep = false;
    if (lane < np) {
        int pos = lds_lower_bound(sm.widx, w, v);
        keep = !(pos < w && sm.widx[pos] == v);
    }
    unsigned long long m = __ballot(keep);
    wave_sync();
    if (keep) sm.pend[lanes_below(m)] = v;
    wave_sync();
    np = __popcll(m);
#pragma unroll
    for (int s = 0; s < ColState<T, LW>::NS; ++s) {
        int q = s * kWave + lane;
        if (q < w) {
            int vv = sm.widx[q];
            int pos = q + lds_lower_bound(sm.pend, np, vv);
            sm.tidx[pos] = vv;
            sm.tbeta[pos] = st.b[s];
        }
    }
    for (int i = lane; i < np; i += kWave) {
        int vv = sm.pend[i];
        int pos = i + lds_lower_bound(sm.widx, w, vv);
        sm.tidx[pos] = vv;
        sm.tbeta[pos] = T(0);
    }
    wave_sync();
    st.w = w + np;
    for (int q = lane; q < st.w; q += kWave) {
        sm.widx[q] = sm.tidx[q];
        sm.wbeta[q] = sm.tbeta[q];
    }
    wave_sync();
    return np;
}

// Load s_W, beta (from sm.wbeta) and S_WW (LDS) for the current W from S.
template <typename T, int LW>
__device__ __forceinline__ void load_working_set(const T *__restrict__ S, int64_t p, int64_t k,
                                 WaveSm<T, LW> &sm, ColState<T, LW> &st,
                                 unsigned *rlo, unsigned *rhi)
{
    const int lane = lane_id();
    const int w = st.w;
#pragma unroll
    for (int s = 0; s < ColState<T, LW>::NS; ++s) {
        int q = s * kWave + lane;
        if (q < w) {
            int64_t j = sm.widx[q];
            j = j < 0 ? 0 : (j >= p ? p - 1 : j);
            st.sv[s] = S[k * p + j];
            st.b[s] = sm.wbeta[q];
        } else {
            st.sv[s] = T(0);
            st.b[s] = T(0);
        }
        st.g[s] = T(0);
    }
    // S is stored symmetric bit for bit: the upper triangle (with the unit
    // diagonal) is gathered and mirrored, w (w + 1) / 2 entries, one load per
    // lane for w <= 10
    const int tot = w * (w + 1) / 2;
    for (int e = lane; e < tot; e += kWave) {
        // e = qj (qj + 1) / 2 + qi, qi <= qj
        int qj = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (qj * (qj + 1) / 2 > e) --qj;
        while ((qj + 1) * (qj + 2) / 2 <= e) ++qj;
        const int qi = e - qj * (qj + 1) / 2;
        int64_t a = sm.widx[qj], b = sm.widx[qi];
        a = a < 0 ? 0 : (a >= p ? p - 1 : a);
        b = b < 0 ? 0 : (b >= p ? p - 1 : b);
        const T v = S[a * p + b];
        sm.sww[qj * LW + qi] = v;
        sm.sww[qi * LW + qj] = v;
    }
    wave_sync();
    rows_to_registers(sm, st, rlo, rhi);
}

// g = s_W - S_WW beta, from scratch.
template <typename T, int LW>
__device__ __forceinline__ void fresh_gradient(WaveSm<T, LW> &sm, ColState<T, LW> &st,
                                               const unsigned *rlo, const unsigned *rhi)
{
    constexpr int NS = ColState<T, LW>::NS;
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < NS; ++s) st.g[s] = st.sv[s];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
        unsigned long long m = __ballot(s2 * kWave + lane < st.w && st.b[s2] != T(0));
        while (m) {
            int l = __builtin_ffsll((long long)m) - 1;
            m &= m - 1;
            int qq = s2 * kWave + l;
            T bq = bcast(st.b[s2], l);
            if constexpr (ColState<T, LW>::kRegRows) {
                st.g[0] -= row_get<T>(rlo, rhi, qq) * bq;
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int q = s * kWave + lane;
                    if (q < LW) st.g[s] -= sm.sww[qq * LW + q] * bq;
                }
            }
        }
    }
}

struct SolveCounts {
    int outer, sweeps, updates;
};

// Inner loops that take this many sweeps try the closed-form fixed point of
// their support (below) before the next outer pass.
constexpr int kDirectSweeps = 12;

// The fixed point of the outer iteration for the current support A and
// signs z of beta, in closed form: with A and z fixed, the lasso solution at
// lambda = lambda0 sigma is beta_A = u - lambda v, u = S_AA^-1 s_A,
// v = S_AA^-1 z_A, and the noise update of Eq. (eq:sigma) becomes
// sigma^2 = 1 - u's_A + lambda0^2 sigma^2 z_A'v, whose fixed point is
// sigma^2 = (1 - u's_A) / (1 - lambda0^2 z_A'v).  The |A| x |A| system is
// solved by Gauss-Jordan elimination on the register rows of S_WW (one row
// per lane, pivots taken in W order; S_AA is symmetric positive definite, so
// no pivoting), which it overwrites: the caller reloads them.  On success
// (a usable system and beta_A with the signs z) beta and sigma are set and
// true is returned; the caller's next coordinate-descent pass, from that
// start, confirms the conditions on all of W (or moves on from it), so the
// minimiser reached is the one of Algorithm 1.
template <typename T, int LW>
__device__ bool direct_fixed_point(ColState<T, LW> &st, unsigned *rlo, unsigned *rhi, T lambda0)
{
    static_assert(ColState<T, LW>::kRegRows && ColState<T, LW>::NS == 1, "register rows, one coordinate per lane");
    const int lane = lane_id();
    const bool inA = lane < st.w && st.b[0] != T(0);
    const unsigned long long mA = __ballot(inA);
    if (__popcll(mA) < 2) return false;
    const T s0 = inA ? st.sv[0] : T(0);
    const T z0 = inA ? (st.b[0] > T(0) ? T(1) : T(-1)) : T(0);
    T xs = s0, xz = z0, d = T(1);
    for (unsigned long long rem = mA; rem; rem &= rem - 1) {
        const int qc = __builtin_ffsll((long long)rem) - 1;  // wave-uniform pivot
        const T pc = bcast(row_get<T>(rlo, rhi, qc), qc);
        if (!(pc > DegenerateFloor<T>::v)) return false;
        if (lane == qc) d = pc;  // later steps leave the pivot's diagonal as it is
        const T f = (inA && lane != qc) ? row_get<T>(rlo, rhi, qc) / pc : T(0);
        const T rs = bcast(xs, qc), rz = bcast(xz, qc);
        for (unsigned long long cols = mA; cols; cols &= cols - 1) {
            const int qe = __builtin_ffsll((long long)cols) - 1;
            const T pv = bcast(row_get<T>(rlo, rhi, qe), qc);  // pivot row, column qe
            row_set(rlo, rhi, qe, row_get<T>(rlo, rhi, qe) - f * pv);
        }
        xs -= f * rs;
        xz -= f * rz;
    }
    const T u = inA ? xs / d : T(0), v = inA ? xz / d : T(0);
    const T us = wave_sum(u * s0), vz = wave_sum(v * z0);
    const T c0 = T(1) - us, c2 = lambda0 * lambda0 * vz;
    if (!(c0 > DegenerateFloor<T>::v) || !(c2 < T(1))) return false;
    const T sigma = sqrt(c0 / (T(1) - c2));
    const T beta = u - lambda0 * sigma * v;
    if (__ballot(inA && !(z0 > T(0) ? beta > T(0) : beta < T(0)))) return false;
    if (inA) st.b[0] = beta;
    st.sigma = sigma;
    return true;
}

// Algorithm 1 on the working set: outer sigma loop around cyclic sweeps,
// with a secant step on the sigma update.  While the support A and the signs
// z of beta stay fixed, the lasso solution at lambda = lambda0 sigma is
// affine in sigma (S_AA beta_A = s_A - lambda0 sigma z_A), and the updated
// value h(sigma)^2 = 1 - beta'(s + g) then works out to C0 + C2 sigma^2 with
// C0 = 1 - s_A' S_AA^-1 s_A and C2 = lambda0^2 z_A' S_AA^-1 z_A.  Two updates
// on the same support and signs give C0 and C2, hence the fixed point
// sigma* = sqrt(C0 / (1 - C2)) of the outer iteration, and beta moves
// along its affine path to sigma*.  The sweeps at lambda0 sigma* and the
// stopping test |h(sigma) - sigma| < tol are those of the plain iteration,
// so the result is the same minimiser (Eq. (eq:spmesl)), reached in fewer
// outer passes; a step that fails its checks is not taken.
// Returns kColOk, kColNoconv or kColDegenerate.
template <typename T, int LW, bool kDirect = true>
__device__ __forceinline__ int scaled_lasso_W(WaveSm<T, LW> &sm, ColState<T, LW> &st,
                                              unsigned *rlo, unsigned *rhi,
                                              T lambda0, T tol, int max_outer, int max_sweeps,
                                              SolveCounts &cnt)
{
    constexpr int NS = ColState<T, LW>::NS;
    const int lane = lane_id();
    // the previous update: sigma, h(sigma), beta, support and sign masks
    bool have = false;
    T sp = T(0), hp = T(0);
    T bp[NS];
    unsigned long long pnz[NS], png[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        bp[s] = T(0);
        pnz[s] = 0ull;
        png[s] = 0ull;
    }
    for (;;) {
        if (cnt.outer >= max_outer) return kColNoconv;
        ++cnt.outer;
        const int sweeps0 = cnt.sweeps;
        const T lam = st.sigma * lambda0;
        fresh_gradient(sm, st, rlo, rhi);
        bool inner_ok = false;
        if constexpr (ColState<T, LW>::kRegRows) {
            // lanes at or beyond w hold b = g = 0 and a zero row, so their
            // change is always 0 and needs no mask
            for (int m = 0; m < max_sweeps; ++m) {
                ++cnt.sweeps;
                T maxd = T(0);
                unsigned long long live = ~0ull;   // coordinates after the last update
                for (;;) {
                    const T nb = soft_clamp(st.g[0] + st.b[0], lam);
                    const T d = nb - st.b[0];
                    const unsigned long long mk = __ballot(d != T(0)) & live;
                    if (!mk) break;
                    const int qs = __builtin_ffsll((long long)mk) - 1;
                    const T dd = bcast(d, qs);
                    if (lane == qs) st.b[0] = nb;
                    st.g[0] -= row_get<T>(rlo, rhi, qs) * dd;
                    const T ad = dd < T(0) ? -dd : dd;
                    maxd = ad > maxd ? ad : maxd;
                    live = qs >= 63 ? 0ull : (~0ull << (qs + 1));
                    ++cnt.updates;
                }
                if (maxd < tol) {
                    inner_ok = true;
                    break;
                }
            }
        } else
        for (int m = 0; m < max_sweeps; ++m) {
            ++cnt.sweeps;
            T maxd = T(0);
            int cur = -1;
            for (;;) {
                T nb[NS], d[NS];
                int qstar = -1;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int q = s * kWave + lane;
                    nb[s] = soft_clamp(st.g[s] + st.b[s], lam);
                    d[s] = nb[s] - st.b[s];
                    bool nz = q < st.w && q > cur && d[s] != T(0);
                    unsigned long long mk = __ballot(nz);
                    if (qstar < 0 && mk) qstar = s * kWave + __builtin_ffsll((long long)mk) - 1;
                }
                if (qstar < 0) break;
                const int ss = qstar / kWave, ls = qstar % kWave;
                T dd = T(0);
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (s == ss) {
                        dd = bcast(d[s], ls);
                        if (lane == ls) st.b[s] = nb[s];
                    }
                T ad = dd < T(0) ? -dd : dd;
                maxd = ad > maxd ? ad : maxd;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    int q = s * kWave + lane;
                    if (q < LW) st.g[s] -= sm.sww[qstar * LW + q] * dd;
                }
                cur = qstar;
                ++cnt.updates;
            }
            if (maxd < tol) {
                inner_ok = true;
                break;
            }
        }
        T part = T(0);
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (s * kWave + lane < st.w) part += st.b[s] * (st.sv[s] + st.g[s]);
        T dot = wave_sum(part);
        T s2 = T(1) - dot;
        st.lam_used = lam;
        if (!(s2 > DegenerateFloor<T>::v)) {
            st.sigma = s2 > T(0) ? sqrt(s2) : T(0);
            return kColDegenerate;
        }
        T sn = sqrt(s2);
        const T so = st.sigma;
        T ds = sn - so;
        ds = ds < T(0) ? -ds : ds;
        st.sigma = sn;
        if (!inner_ok) return kColNoconv;
        if (ds < tol) return kColOk;
        bool same = have;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const bool in = s * kWave + lane < st.w;
            const unsigned long long nz = __ballot(in && st.b[s] != T(0));
            const unsigned long long ng = __ballot(in && st.b[s] < T(0));
            same = same && nz == pnz[s] && ng == png[s];
            pnz[s] = nz;
            png[s] = ng;
        }
        bool jumped = false;
        if constexpr (kDirect && ColState<T, LW>::kRegRows && ColState<T, LW>::NS == 1) {
            // a slow inner loop (strongly correlated coordinates): start the
            // next pass from the closed-form fixed point of this support
            if (cnt.sweeps - sweeps0 >= kDirectSweeps) {
                jumped = direct_fixed_point(st, rlo, rhi, lambda0);
                rows_to_registers(sm, st, rlo, rhi);
            }
        }
        if (same && !jumped) {
            const T c2 = (sn * sn - hp * hp) / (so * so - sp * sp);
            const T c0 = sn * sn - c2 * so * so;
            T dsp = so - sp;
            dsp = dsp < T(0) ? -dsp : dsp;
            if (dsp > T(64) * Eps<T>::v * so && c2 >= T(0) && c2 < T(1) && c0 > T(0)) {
                const T ss = sqrt(c0 / (T(1) - c2));
                T jump = ss - sn;
                jump = jump < T(0) ? -jump : jump;
                if (jump <= T(16) * ds) {
                    const T f = (ss - so) / (so - sp);
#pragma unroll
                    for (int s = 0; s < NS; ++s) st.b[s] += f * (st.b[s] - bp[s]);
                    st.sigma = ss;
                    jumped = true;
                }
            }
        }
        // a step needs two fresh updates on one support
        have = !jumped;
        sp = so;
        hp = sn;
#pragma unroll
        for (int s = 0; s < NS; ++s) bp[s] = st.b[s];
    }
}

// In-wave sort of n <= 64 ints in LDS with duplicates removed (stable rank
// sort, then compaction).  Returns the number of distinct values.
__device__ __forceinline__ int sort_unique_small(int *a, int n)
{
    const int lane = lane_id();
    int v = lane < n ? a[lane] : 0;
    int rank = 0;
    for (int i = 0; i < n; ++i) {
        int ai = a[i];
        rank += (ai < v || (ai == v && i < lane)) ? 1 : 0;
    }
    wave_sync();
    if (lane < n) a[rank] = v;
    wave_sync();
    int u = lane < n ? a[lane] : 0;
    bool keep = lane < n && (lane == 0 || a[lane - 1] != u);
    unsigned long long m = __ballot(keep);
    wave_sync();
    if (keep) a[lanes_below(m)] = u;
    wave_sync();
    return __popcll(m);
}

// Store a column's state: working set and coefficients (k-major), sigma,
// lambda, status, and (with_support) the slot-major support list.
template <typename T, int LW>
__device__ __forceinline__ void store_column(const ColArgs<T> &A, int64_t k, const WaveSm<T, LW> &sm,
                             const ColState<T, LW> &st, int status, bool with_support)
{
    const int lane = lane_id();
    const int64_t p = A.p;
    int ns = 0;
#pragma unroll
    for (int s = 0; s < ColState<T, LW>::NS; ++s) {
        int q = s * kWave + lane;
        bool in = q < st.w;
        if (in) {
            A.w_idx[k * kWMax + q] = sm.widx[q];
            A.w_beta[k * kWMax + q] = st.b[s];
        }
        if (with_support) {
            bool nz = in && st.b[s] != T(0);
            unsigned long long m = __ballot(nz);
            if (nz) {
                int pos = ns + lanes_below(m);
                A.supp_idx[(int64_t)pos * p + k] = sm.widx[q];
                A.supp_val[(int64_t)pos * p + k] = st.b[s];
            }
            ns += __popcll(m);
        }
    }
    if (with_support && lane >= ns && lane < kSuppPad) {
        // pad the first slots so readers may load them without the count
        A.supp_idx[(int64_t)lane * p + k] = (int)k;
        A.supp_val[(int64_t)lane * p + k] = T(0);
    }
    if (lane == 0) {
        A.w_cnt[k] = st.w;
        A.sigma[k] = (double)st.sigma;
        A.lam_used[k] = (double)st.lam_used;
        A.col_status[k] = status;
        if (with_support) A.supp_cnt[k] = ns;
    }
}

} // namespace spmesl
