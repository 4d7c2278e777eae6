// polish.hip -- double-precision finish of the mixed-precision solve.
//
// The float solve (covariance from a bfloat16 split, float coordinate
// descent) stops at a float-reachable tolerance.  For each column the polish
// re-solves the scaled lasso of Eq. (eq:spmesl) in double on a small working
// set W' = (float support) U (float near-threshold band), with S restricted
// to W' formed in double directly from the standardised data, to the
// caller's tolerance.  It then proves that no coordinate outside W' violates
// the lasso KKT conditions in double:
//   for j outside the band, |g32_j| <= lambda32 - band was observed, and
//   |g64_j(beta64) - g32_j(beta32)| <= ||beta64 - beta32||_1
//                                     + (eps_S + eps_f)(1 + ||beta32||_1),
//   (|S_jl| <= 1 for a correlation matrix), so if that bound plus
//   max(0, lambda32 - lambda64) stays below the band no j outside W' can
//   violate.  Otherwise a full pass over the float S with the double
//   coefficients flags every j within the error margin of lambda64, adds
//   them to W' (where the double solve decides them exactly), and repeats.
#include "colsolve_dev.hpp"

namespace spmesl {

// S_W'W' (LDS) and s_W' (registers) in double from Xt (p x n, standardised).
__device__ __forceinline__ int64_t clamp_index(int v, int64_t p)
{
    return v < 0 ? 0 : (v >= p ? p - 1 : (int64_t)v);
}

// Small working sets: the R rows x_k, x_{W'[0]}, .., x_{W'[R-2]} are read for
// C 64-sample chunks at a time with every load of a batch in flight together,
// so the n-sample dot products take ceil(n / (64 C)) memory round trips
// rather than one per 64 samples for each group of pairs.  pr[] receives the
// R (R - 1) / 2 products of rows a < b in row-major pair order, divided by n.
template <int R, int C, int LW>
__device__ __forceinline__ void gram_rows(const double *__restrict__ Xt, int64_t n, int64_t p, int64_t k,
                                          const WaveSm<double, LW> &sm, int w, double *pr)
{
    constexpr int NP = R * (R - 1) / 2;
    const int lane = lane_id();
    const double *r[R];
    r[0] = Xt + k * n;
#pragma unroll
    for (int q = 1; q < R; ++q) r[q] = Xt + (q <= w ? clamp_index(sm.widx[q - 1], p) : k) * n;
    double acc[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) acc[u] = 0.0;
    for (int64_t i0 = 0; i0 < n; i0 += C * kWave) {
        double v[R][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int64_t i = i0 + c * kWave + lane;
#pragma unroll
            for (int q = 0; q < R; ++q) v[q][c] = (q <= w && i < n) ? r[q][i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            int u = 0;
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = a + 1; b < R; ++b) acc[u++] += v[a][c] * v[b][c];
        }
    }
    const double invn = 1.0 / (double)n;
#pragma unroll
    for (int u = 0; u < NP; ++u) pr[u] = wave_sum(acc[u]) * invn;
}

// Products of rows a < b (row 0 = x_k) into s_W' (tbeta, staged) and S_W'W'.
template <int R, int LW>
__device__ __forceinline__ void store_gram_rows(WaveSm<double, LW> &sm, int w, const double *pr)
{
    if (lane_id() != 0) return;
    int u = 0;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = a + 1; b < R; ++b, ++u) {
            if (b > w) continue;
            if (a == 0) {
                sm.tbeta[b - 1] = pr[u];
            } else {
                sm.sww[(b - 1) * LW + (a - 1)] = pr[u];
                sm.sww[(a - 1) * LW + (b - 1)] = pr[u];
            }
        }
}

constexpr int kSmallW = 3;   // four rows, four chunks per batch
constexpr int kMidW = 7;     // eight rows, two chunks per batch

// Larger working sets: the rows x_k, x_{W'[0]}, .. (R = w + 1 of them) in
// blocks of four; each pair of blocks reads its eight rows for two 64-sample
// chunks at a time (all loads of a step in flight) and accumulates the 16
// products in registers, so a row is re-read once per block rather than once
// per pair.  Products of rows a < b go to s_W' (a = 0, staged in tbeta) or to
// S_W'W' (mirrored), divided by n.
template <int LW>
__device__ void gram_blocked(const double *__restrict__ Xt, int64_t n, int64_t p, int64_t k,
                             WaveSm<double, LW> &sm, int w)
{
    const int lane = lane_id();
    const int R = w + 1;
    const int nb = (R + 3) / 4;
    const double invn = 1.0 / (double)n;
    auto row = [&](int r) -> const double * {
        return Xt + (r == 0 || r > w ? k : clamp_index(sm.widx[r - 1], p)) * n;
    };
    for (int bi = 0; bi < nb; ++bi)
        for (int bj = bi; bj < nb; ++bj) {
            const double *ra[4], *rb[4];
            bool va[4], vb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                va[u] = 4 * bi + u < R;
                vb[u] = 4 * bj + u < R;
                ra[u] = row(4 * bi + u);
                rb[u] = row(4 * bj + u);
            }
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
            for (int64_t i0 = lane; i0 < n; i0 += 2 * kWave) {
                double xa[2][4], xb[2][4];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int64_t i = i0 + c * kWave;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        xa[c][u] = (va[u] && i < n) ? ra[u][i] : 0.0;
                        xb[c][u] = (vb[u] && i < n) ? rb[u][i] : 0.0;
                    }
                }
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] += xa[c][u] * xb[c][v];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int a = 4 * bi + u, b = 4 * bj + v;
                    if (!(a < b && b < R)) continue;  // wave-uniform
                    const double val = wave_sum(acc[u][v]) * invn;
                    if (lane == 0) {
                        if (a == 0) {
                            sm.tbeta[b - 1] = val;
                        } else {
                            sm.sww[(b - 1) * LW + (a - 1)] = val;
                            sm.sww[(a - 1) * LW + (b - 1)] = val;
                        }
                    }
                }
        }
}

template <int LW>
__device__ __forceinline__ void load_working_set_xt(const double *__restrict__ Xt, int64_t n, int64_t p,
                                    int64_t k, WaveSm<double, LW> &sm, ColState<double, LW> &st,
                                    unsigned *rlo, unsigned *rhi)
{
    constexpr int NS = ColState<double, LW>::NS;
    const int lane = lane_id();
    const int w = st.w;
    if (w <= kSmallW) {
        double pr[6];
        gram_rows<4, 4>(Xt, n, p, k, sm, w, pr);
        store_gram_rows<4>(sm, w, pr);
    } else if (kMidW < LW && w <= kMidW) {
        double pr[28];
        gram_rows<8, 2>(Xt, n, p, k, sm, w, pr);
        store_gram_rows<8>(sm, w, pr);
    }
    if (w > kMidW) gram_blocked(Xt, n, p, k, sm, w);
    for (int q = lane; q < w; q += kWave) sm.sww[q * LW + q] = 1.0;
    wave_sync();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int q = s * kWave + lane;
        st.sv[s] = q < w ? sm.tbeta[q] : 0.0;
        st.b[s] = q < w ? sm.wbeta[q] : 0.0;
        st.g[s] = 0.0;
    }
    wave_sync();
}

// Direct solve of the scaled lasso on W' for the float solution's support A
// and signs z.  With A and z fixed the lasso solution at lambda = lambda0
// sigma is beta_A = u - lambda v with u = S_AA^-1 s_A, v = S_AA^-1 z_A, and
// the noise update of Eq. (eq:sigma) becomes sigma^2 = 1 - u's_A +
// lambda0^2 sigma^2 z_A'v, so the fixed point of the outer iteration is
// sigma^2 = (1 - u's_A) / (1 - lambda0^2 z_A'v).  When the resulting beta_A
// has the signs z and every other j in W' has |g_j| <= lambda (+ tol), it is
// the minimiser of Eq. (eq:spmesl) on W' exactly (the KKT conditions of
// Eq. (eqn:lasso) hold with the sigma that is its own update); otherwise
// (the support or a sign changes, or the system is degenerate) nothing is
// changed and coordinate descent runs.  The |A| x |A| system is solved by
// Gauss-Jordan elimination, one row per lane (S_AA is symmetric positive
// definite, so no pivoting).
constexpr int kDirectMax = 24;

template <int LW>
__device__ bool polish_direct(WaveSm<double, LW> &sm, ColState<double, LW> &st, double lambda0, double tol)
{
    static_assert(ColState<double, LW>::NS == 1, "one coordinate per lane");
    const int lane = lane_id();
    const int w = st.w;
    const bool inA = lane < w && st.b[0] != 0.0;
    const unsigned long long mA = __ballot(inA);
    const int m = __popcll(mA);
    if (m == 0 || m > kDirectMax) return false;
    const int r0 = lanes_below(mA);  // compact position of this lane's coordinate
    if (inA) sm.tidx[r0] = lane;
    wave_sync();
    // compact row r = lane: S_AA, s_A, z_A (rows of the lanes below m)
    const bool row = lane < m;
    const int qr = row ? sm.tidx[lane] : 0;
    double a[kDirectMax];
#pragma unroll
    for (int c = 0; c < kDirectMax; ++c) a[c] = (row && c < m) ? sm.sww[qr * LW + sm.tidx[c]] : 0.0;
    const double s0 = row ? sm.tbeta[qr] : 0.0;  // s_W' as staged by the Gram
    const double z0 = row ? (sm.wbeta[qr] > 0.0 ? 1.0 : -1.0) : 0.0;
    double xs = s0, xz = z0;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < kDirectMax; ++c) {
        // every step is unrolled (the row stays in registers); steps past m
        // and entries past m are skipped by wave-uniform tests
        if (c < m) {
            const double pc = bcast(a[c], c);
            ok = ok && pc > 1e-12;
            const double rs = bcast(xs, c), rz = bcast(xz, c);
            // lane c's own row is left as it is (f = 0), so its entries read
            // here are those of the pivot row at this step
            const double f = (row && lane != c && pc > 1e-12) ? a[c] / pc : 0.0;
#pragma unroll
            for (int e = 0; e < kDirectMax; ++e)
                if (e < m) a[e] -= f * bcast(a[e], c);
            xs -= f * rs;
            xz -= f * rz;
        }
    }
    if (!ok) return false;
    double d = 1.0;
#pragma unroll
    for (int c = 0; c < kDirectMax; ++c)
        if (c == lane) d = a[c];
    const double u = row ? xs / d : 0.0, v = row ? xz / d : 0.0;
    const double us = wave_sum(u * s0), vz = wave_sum(v * z0);
    const double c0 = 1.0 - us, c2 = lambda0 * lambda0 * vz;
    if (!(c0 > DegenerateFloor<double>::v) || !(c2 < 1.0)) return false;
    const double sigma = sqrt(c0 / (1.0 - c2));
    const double lam = lambda0 * sigma;
    const double beta = u - lam * v;
    if (__ballot(row && !(z0 > 0.0 ? beta > 0.0 : beta < 0.0))) return false;
    // gradients of the coordinates of W' outside A
    if (row) sm.sval[lane] = beta;
    wave_sync();
    double g = lane < w ? st.sv[0] : 0.0;
    for (int r = 0; r < m; ++r) g -= (lane < w ? sm.sww[lane * LW + sm.tidx[r]] : 0.0) * sm.sval[r];
    const double ag = g < 0.0 ? -g : g;
    if (__ballot(lane < w && !inA && ag > lam + tol)) return false;
    st.b[0] = inA ? sm.sval[r0] : 0.0;
    st.sigma = sigma;
    st.lam_used = lam;
    wave_sync();
    return true;
}

// beta32 of variable j in column k's float list (0 if absent)
__device__ __forceinline__ double beta32_of(const PolishArgs &A, int64_t k, int j)
{
    const int *idx = A.w_idx32 + k * kWMax;
    int w = A.w_cnt32[k];
    w = w < 0 ? 0 : (w > kWMax ? kWMax : w);
    int lo = 0, hi = w;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (idx[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < w && idx[lo] == j) ? (double)A.w_beta32[k * kWMax + lo] : 0.0;
}

template <int LW>
__device__ void polish_column(const PolishArgs &A, WaveSm<double, LW> &sm, int64_t k, int tier2);

template <int LW, int NW, int MINW = 1>
__global__ __launch_bounds__(kWave *NW) __attribute__((amdgpu_waves_per_eu(MINW))) void k_polish(PolishArgs A,
                                                                                                 int tier2)
{
    __shared__ WaveSm<double, LW> smem[NW];
    const int wv = threadIdx.x / kWave;
    WaveSm<double, LW> &sm = smem[wv];
    const int64_t gw0 = (int64_t)blockIdx.x * NW + wv;
    const int64_t nwork = tier2 ? (int64_t)*A.esc_cnt : A.p;
    for (int64_t gw = gw0; gw < nwork; gw += (int64_t)gridDim.x * NW) {
        const int64_t k = tier2 ? (int64_t)A.esc_list[gw] : gw;
        polish_column<LW>(A, sm, k, tier2);
    }
}

template <int LW>
__device__ __forceinline__ void polish_column(const PolishArgs &A, WaveSm<double, LW> &sm, int64_t k, int tier2)
{
    constexpr int NS = ColState<double, LW>::NS;
    const int lane = lane_id();
    // everything the column's set-up reads, in one round of loads: the
    // counts, the first 64 entries of the float list and the band (both
    // arrays hold kWMax >= 64 and kBandMax entries per column), sigma, lambda
    const int flagged = *A.flags;
    int w32 = A.w_cnt32[k];
    int nb = A.band_cnt[k];
    const int st32 = A.col_status32[k];
    const double sig32 = A.sigma32[k];
    const double lam32 = A.lam32[k];
    const float bfirst = A.w_beta32[k * kWMax + lane];
    const int ifirst = A.w_idx32[k * kWMax + lane];
    const int bandfirst = lane < kBandMax ? A.band_idx[k * kBandMax + lane] : 0;
    asm volatile("" ::"v"(bfirst), "v"(ifirst), "v"(bandfirst));
    if (flagged) {
        if (lane == 0) {
            A.w_cnt[k] = 0;
            A.sigma[k] = 1.0;
            A.lam_used[k] = A.lambda0;
            A.col_status[k] = kColOk;
            for (int i = 0; i < 8; ++i) A.polinfo[k * 8 + i] = 0;
        }
        return;
    }
    const int64_t p = A.p;
    ColState<double, LW> st;
    unsigned rlo[ColState<double, LW>::kRows], rhi[ColState<double, LW>::kRowsHi];
    SolveCounts cnt = {0, 0, 0};
    int status = kColOk, rounds = 0, checks = 0, added = 0;

    // a column the float stage handed to the dense tier (its state is the
    // 128-coordinate tier's last working set and pending candidates): the
    // dense tier solves it in double
    if (w32 > kWMax || st32 == kColDenseQ) {
        if (lane == 0) {
            int pos = atomicAdd(A.dense_cnt, 1);
            A.dense_list[pos] = (int)k;
        }
        return;
    }
    // --- W' = float support U float band --------------------------------
    w32 = w32 < 0 ? 0 : w32;
    nb = nb < 0 ? 0 : nb;
    bool full = A.full_kkt || nb > kBandMax || (st32 != kColOk && st32 != kColDeferred);
    if constexpr (LW < kWMax) {
        // the full pass is the wide kernel's: hand a column that will need it
        // over at once
        if (A.full_kkt) {
            if (lane == 0) {
                int pos = atomicAdd(A.esc_cnt, 1);
                A.esc_list[pos] = (int)k;
            }
            return;
        }
    }
    nb = nb < kBandMax ? nb : kBandMax;
    double norm32 = 0.0;
    int ns = 0;
    for (int q0 = 0; q0 < w32; q0 += kWave) {
        int q = q0 + lane;
        float b = q < w32 ? (q0 == 0 ? bfirst : A.w_beta32[k * kWMax + q]) : 0.0f;
        bool nz = b != 0.0f;
        unsigned long long m = __ballot(nz);
        int pos = ns + lanes_below(m);
        if (nz && pos < LW) {
            sm.widx[pos] = q0 == 0 ? ifirst : A.w_idx32[k * kWMax + q];
            sm.wbeta[pos] = (double)b;
        }
        norm32 += nz ? fabs((double)b) : 0.0;
        ns += __popcll(m);
    }
    norm32 = wave_sum(norm32);
    if (lane < nb) sm.pend[lane] = bandfirst;
    wave_sync();
    nb = sort_unique_small(sm.pend, nb);  // the row-tiled pass appends in any order
    if (ns + nb > LW) {
        // to the wide kernel, or from it to the dense tier
        if (lane == 0) {
            int pos = atomicAdd(tier2 ? A.dense_cnt : A.esc_cnt, 1);
            (tier2 ? A.dense_list : A.esc_list)[pos] = (int)k;
        }
        return;
    }
    st.w = ns;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int q = s * kWave + lane;
        st.b[s] = q < ns ? sm.wbeta[q] : 0.0;
    }
    wave_sync();
    merge_pending(sm, st, nb);
    // beta32 over W' (zero on the band), kept for the first bound check:
    // every nonzero of the float solution is in W'
    double b32[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int q = s * kWave + lane;
        st.b[s] = q < st.w ? sm.wbeta[q] : 0.0;
        b32[s] = st.b[s];
    }
    st.sigma = sig32;
    st.lam_used = lam32;

    while (status == kColOk) {
        // the direct solve first (first round, one coordinate per lane);
        // the register rows of S_W'W' are filled only for coordinate descent
        constexpr bool kTryDirect = ColState<double, LW>::NS == 1;
        const bool try_direct = kTryDirect && !full;
        load_working_set_xt(A.Xt, A.n, A.p, k, sm, st, rlo, rhi);
        bool direct = false;
        if constexpr (kTryDirect) {
            if (try_direct) direct = polish_direct(sm, st, A.lambda0, A.tol);
        }
        if (direct) {
            ++cnt.outer;
        } else {
            rows_to_registers(sm, st, rlo, rhi);
            // (the direct solve of this support was tried above)
            status = scaled_lasso_W<double, LW, false>(sm, st, rlo, rhi, A.lambda0, A.tol, A.max_outer,
                                                       A.max_sweeps, cnt);
        }
        if (status != kColOk) break;
        // bound on the change of any gradient outside W'
        double part = 0.0, nrm = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            int q = s * kWave + lane;
            if (q < st.w) {
                // after a merge W' is reordered: look the float value up
                const double f = added == 0 ? b32[s] : beta32_of(A, k, sm.widx[q]);
                part += fabs(st.b[s] - f);
                nrm += fabs(st.b[s]);
            }
        }
        double l1d = wave_sum(part);
        double norm64 = wave_sum(nrm);
        double lamdrop = lam32 - st.lam_used;
        lamdrop = lamdrop > 0.0 ? lamdrop : 0.0;
        double bound = l1d + A.eps * (1.0 + norm32) + lamdrop;
        if (!full && bound < (double)A.band) break;
        if constexpr (LW < kWMax) {
            // the full pass below is left to the wide kernel, which redoes
            // the column (rare; keeps this kernel's registers low)
            if (lane == 0) {
                int pos = atomicAdd(A.esc_cnt, 1);
                A.esc_list[pos] = (int)k;
            }
            return;
        } else {
        // full pass: every j whose float-S gradient is within the error
        // margin of lambda64 joins W'
        int nsup = build_support(sm, st);
        double margin = A.eps * (1.0 + norm64);
        ++checks;
        int npend = kkt_pass<float, double, LW>(A.S32, p, p, k, sm, st.w, nsup, st.lam_used - margin,
                                               false, 0.0, nullptr, nullptr);
        if (npend == 0) break;
        if (rounds >= A.max_rounds) {
            status = kColNoconv;
            break;
        }
        ++rounds;
        int np = npend < kPendMax ? npend : kPendMax;
        if (st.w + np > LW) {
            if (lane == 0) {
                int pos = atomicAdd(tier2 ? A.dense_cnt : A.esc_cnt, 1);
                (tier2 ? A.dense_list : A.esc_list)[pos] = (int)k;
            }
            return;
        }
        // keep the double coefficients across the merge
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            int q = s * kWave + lane;
            if (q < st.w) sm.wbeta[q] = st.b[s];
        }
        wave_sync();
        merge_pending(sm, st, np);
        added += np;
        full = true;
        }
    }
    // store the double lists
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int q = s * kWave + lane;
        if (q < st.w) {
            A.w_idx[k * kWMax + q] = sm.widx[q];
            A.w_beta[k * kWMax + q] = st.b[s];
        }
    }
    if (lane == 0) {
        A.w_cnt[k] = st.w;
        A.sigma[k] = st.sigma;
        A.lam_used[k] = st.lam_used;
        A.col_status[k] = status;
        int *pi = A.polinfo + k * 8;
        pi[0] = cnt.outer;
        pi[1] = cnt.sweeps;
        pi[2] = cnt.updates;
        pi[3] = checks;
        pi[4] = added;
    }
}

// The polish of many problems in one launch: item g is column g - off[d]
// of problem d (tier2 = 0), or entry g - off[d] of its escalation list.
template <int LW, int NW, int MINW = 1>
__global__ __launch_bounds__(kWave *NW) __attribute__((amdgpu_waves_per_eu(MINW))) void k_polish_grouped(
    const PolishArgs *__restrict__ tab, const int64_t *__restrict__ off, int nd, int tier2)
{
    __shared__ WaveSm<double, LW> smem[NW];
    const int wv = threadIdx.x / kWave;
    const int64_t total = off[nd];
    for (int64_t g = (int64_t)blockIdx.x * NW + wv; g < total; g += (int64_t)gridDim.x * NW) {
        const int d = group_of(off, nd, g);
        const PolishArgs &A = tab[d];
        const int64_t k = tier2 ? (int64_t)A.esc_list[g - off[d]] : g - off[d];
        polish_column<LW>(A, smem[wv], k, tier2);
    }
}

void launch_polish_grouped(const PolishArgs *tab, const int64_t *off, int nd, int64_t total, int tier2,
                           hipStream_t s)
{
    if (total <= 0) return;
    if (tier2 == 0)
        hipLaunchKernelGGL((k_polish_grouped<32, 1, 3>), dim3((unsigned)total), dim3(kWave), 0, s, tab, off, nd, 0);
    else
        hipLaunchKernelGGL((k_polish_grouped<kWMax, 1>), dim3((unsigned)(total < 256 ? total : 256)), dim3(kWave), 0,
                           s, tab, off, nd, 1);
}

void launch_polish(const PolishArgs &a, hipStream_t s)
{
    // one column per workgroup: a column's slot frees as soon as it is done
    constexpr int NW = 1;
    hipLaunchKernelGGL((k_polish<32, NW, 3>), dim3((unsigned)((a.p + NW - 1) / NW)),
                       dim3(kWave * NW), 0, s, a, 0);
    hipLaunchKernelGGL((k_polish<kWMax, 1>), dim3((unsigned)(a.p < 256 ? a.p : 256)), dim3(kWave), 0,
                       s, a, 1);
}

} // namespace spmesl
