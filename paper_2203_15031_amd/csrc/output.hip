// output.hip -- B, sigma and the symmetrised Omega from the per-column
// coefficient lists.
//
// Omega_1 = -B D with D = diag(sigma^-2) (Eq. (eq:relation)), then the
// min-magnitude symmetrisation of Eq. (eq:symm): for j < k both entries
// become the one of smaller magnitude, the upper entry omega_jk on a tie.
// Because an entry of Omega_1 is zero wherever the coefficient is, the
// symmetrised off-diagonal entry is nonzero only where both beta_jk and
// beta_kj are, so the dense outputs are a zero fill (the HBM-bound part) and
// a scatter of the few nonzeros.  Proposition 1 maps back to the data's
// scale: b^o_jk = (c_j / c_k) b_jk, sigma^o_k = sigma_k / c_k,
// omega^o_jk = c_j c_k omega_jk.
#include "common.hpp"

namespace spmesl {

__global__ __launch_bounds__(256) void k_zero_words(uint32_t *__restrict__ a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0u;
}

// Prefix sums of nd device counts (stride apart), by one block: the counts
// are read in parallel, summed in order by one thread from LDS.
__global__ __launch_bounds__(1024) void k_group_offsets(const int *__restrict__ cnt, int64_t stride, int nd,
                                                        int64_t *__restrict__ off)
{
    __shared__ int c[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) {
        carry = 0;
        off[0] = 0;
    }
    for (int d0 = 0; d0 < nd; d0 += 1024) {
        const int d = d0 + (int)threadIdx.x;
        __syncthreads();
        if (d < nd) {
            const int v = cnt[(int64_t)d * stride];
            c[threadIdx.x] = v > 0 ? v : 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t a = carry;
            const int m = nd - d0 < 1024 ? nd - d0 : 1024;
            for (int i = 0; i < m; ++i) {
                a += c[i];
                off[d0 + i + 1] = a;
            }
            carry = a;
        }
    }
}

void launch_group_offsets(const int *cnt, int64_t stride, int nd, int64_t *off, hipStream_t s)
{
    hipLaunchKernelGGL(k_group_offsets, dim3(1), dim3(1024), 0, s, cnt, stride, nd, off);
}

void launch_zero_words(uint32_t *a, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s, a, n);
}

// One block: sums and maxima of the per-column counters, status bits from
// the final per-column statuses.  Each thread takes four columns per pass
// with every load of the pass in flight together (16-byte loads of the
// counter records); sums are carried in double (exact below 2^53) through
// DPP wave reductions, then one LDS step across the block's waves.
__global__ __launch_bounds__(1024) void k_reduce_stats(int64_t p, const int *__restrict__ colinfo,
                                                       const int *__restrict__ polinfo,
                                                       const int *__restrict__ w_cnt,
                                                       const int *__restrict__ col_status,
                                                       unsigned long long *__restrict__ counters,
                                                       int *__restrict__ status_bits)
{
    typedef int i4 __attribute__((ext_vector_type(4)));
    constexpr int U = 4;
    // outer, sweeps, updates, rounds, polish checks, polish added, noconv,
    // final working-set sizes
    double sum[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int maxw = 0, maxo = 0, bits = 0;
    const int64_t nt = blockDim.x;
    for (int64_t k0 = threadIdx.x; k0 < p; k0 += U * nt) {
        i4 ci[U], pa[U], pb[U];
        int wc[U], cs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + u * nt;
            const bool in = k < p;
            const i4 z = {0, 0, 0, 0};
            ci[u] = in ? *reinterpret_cast<const i4 *>(colinfo + k * 4) : z;
            pa[u] = in && polinfo ? *reinterpret_cast<const i4 *>(polinfo + k * 8) : z;
            pb[u] = in && polinfo ? *reinterpret_cast<const i4 *>(polinfo + k * 8 + 4) : z;
            wc[u] = in ? w_cnt[k] : 0;
            cs[u] = in ? col_status[k] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sum[0] += (double)(unsigned)ci[u].x + (double)(unsigned)pa[u].x;
            sum[1] += (double)(unsigned)ci[u].y + (double)(unsigned)pa[u].y;
            sum[2] += (double)(unsigned)ci[u].z + (double)(unsigned)pa[u].z;
            sum[3] += (double)(unsigned)ci[u].w;
            sum[4] += (double)(unsigned)pa[u].w;
            sum[5] += (double)(unsigned)pb[u].x;
            const int o = ci[u].x + pa[u].x;
            maxo = o > maxo ? o : maxo;
            maxw = wc[u] > maxw ? wc[u] : maxw;
            sum[7] += (double)(wc[u] > 0 ? wc[u] : 0);
            if (cs[u] < 0) {
                sum[6] += 1.0;
                bits |= cs[u] == kColWorkset ? 4 : (cs[u] == kColDegenerate ? 2 : 1);
            }
        }
    }
    __shared__ double red[8][32];
    __shared__ int redi[3][32];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < 8; ++i) sum[i] = wave_sum(sum[i]);
    // maxima below 2^24 are exact in float
    const int wmaxw = (int)wave_max((float)maxw), wmaxo = (int)wave_max((float)maxo);
    const int wbits = (__ballot(bits & 1) ? 1 : 0) | (__ballot(bits & 2) ? 2 : 0) | (__ballot(bits & 4) ? 4 : 0);
    if (lane == 0) {
        for (int i = 0; i < 8; ++i) red[i][wv] = sum[i];
        redi[0][wv] = wmaxw;
        redi[1][wv] = wmaxo;
        redi[2][wv] = wbits;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (int)(blockDim.x / kWave);
        double t[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int mw = 0, mo = 0, bb = 0;
        for (int w = 0; w < nw; ++w) {
            for (int i = 0; i < 8; ++i) t[i] += red[i][w];
            mw = redi[0][w] > mw ? redi[0][w] : mw;
            mo = redi[1][w] > mo ? redi[1][w] : mo;
            bb |= redi[2][w];
        }
        counters[kCntOuter] = (unsigned long long)t[0];
        counters[kCntSweeps] = (unsigned long long)t[1];
        counters[kCntUpdates] = (unsigned long long)t[2];
        counters[kCntRounds] = (unsigned long long)t[3];
        counters[kCntPolishChecks] = (unsigned long long)t[4];
        counters[kCntPolishAdded] = (unsigned long long)t[5];
        counters[kCntNoconv] = (unsigned long long)t[6];
        counters[kCntSumW] = (unsigned long long)t[7];
        counters[kCntMaxW] = (unsigned long long)mw;
        counters[kCntMaxOuter] = (unsigned long long)mo;
        *status_bits = bb;
    }
}

void launch_reduce_stats(int64_t p, const int *colinfo, const int *polinfo, const int *w_cnt,
                         const int *col_status, unsigned long long *counters, int *status_bits,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(1024), 0, s, p, colinfo, polinfo, w_cnt,
                       col_status, counters, status_bits);
}

__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ A, int64_t count)
{
    typedef double dv2 __attribute__((ext_vector_type(2)));
    int64_t nvec = count / 2;
    dv2 *A2 = reinterpret_cast<dv2 *>(A);
    const dv2 z = {0.0, 0.0};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
        __builtin_nontemporal_store(z, &A2[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (count & 1)) A[count - 1] = 0.0;
}

void launch_fill_zero(double *A, int64_t count, hipStream_t s, int max_blocks)
{
    if (count <= 0) return;
    if (((uintptr_t)A & 15u) != 0) {
        // caller's array is only 8-byte aligned: clear one element, then the
        // rest is 16-byte aligned
        launch_zero_words((uint32_t *)A, 2, s);
        ++A;
        --count;
        if (count <= 0) return;
    }
    int64_t nvec = count / 2;
    int64_t blocks = (nvec + 255) / 256;
    // a small grid: the fill runs beside the latency-bound column solves on
    // the second stream; 64 blocks of nontemporal 16-byte stores still write
    // about 5 TB/s, and leave the solves their wave slots (with 256 blocks
    // the re-solves of flagged columns took 90 us instead of 65 at p = 5000)
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, A, count);
}

// one wave per column k; lanes walk the column's list
template <typename T>
__global__ __launch_bounds__(256) void k_scatter(int64_t p, const int *__restrict__ w_cnt,
                                                 const int *__restrict__ w_idx,
                                                 const T *__restrict__ w_beta,
                                                 const int *__restrict__ w_off,
                                                 const double *__restrict__ sigma,
                                                 const double *__restrict__ scale, int original,
                                                 double *__restrict__ B,
                                                 double *__restrict__ sig_out,
                                                 double *__restrict__ Om,
                                                 const int *__restrict__ flags)
{
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= p || *flags) return;
    int wk = w_cnt[k];
    wk = wk < 0 ? 0 : wk;
    const int64_t bk = list_base(w_off, p, k, wk);
    const double sk = sigma[k];
    const double ck = original ? scale[k] : 1.0;
    const double dk = 1.0 / (sk * sk);
    for (int q = lane; q < wk; q += kWave) {
        const int j = w_idx[bk + q];
        const double b = (double)w_beta[bk + q];
        if (b == 0.0 || j < 0 || (int64_t)j >= p) continue;
        const double cj = original ? scale[j] : 1.0;
        if (B) B[(int64_t)j * p + k] = b * (cj / ck);
        if (Om && j < k) {
            // the pair (j, k) belongs to its larger index k
            int wj = w_cnt[j];
            wj = wj < 0 ? 0 : wj;
            const int64_t bj = list_base(w_off, p, j, wj);
            const int *lj = w_idx + bj;
            int lo = 0, hi = wj;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (lj[mid] < (int)k) lo = mid + 1;
                else hi = mid;
            }
            if (lo < wj && lj[lo] == (int)k) {
                const double bkj = (double)w_beta[bj + lo];
                if (bkj != 0.0) {
                    const double sj = sigma[j];
                    const double ojk = -b * dk;               // omega_jk,1 (column k)
                    const double okj = -bkj / (sj * sj);      // omega_kj,1 (column j)
                    double v = fabs(ojk) <= fabs(okj) ? ojk : okj;
                    v *= cj * ck;
                    Om[(int64_t)j * p + k] = v;
                    Om[k * p + j] = v;
                }
            }
        }
    }
    if (lane == 0) {
        if (Om) Om[k * p + k] = dk * ck * ck;
        if (sig_out) sig_out[k] = sk / ck;
    }
}

template <typename T>
void launch_scatter_outputs(int64_t p, const int *w_cnt, const int *w_idx, const T *w_beta, const int *w_off,
                            const double *sigma, const double *scale, int original_scale,
                            double *B, double *sig_out, double *Omega, const int *flags,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)((p + 3) / 4)), dim3(256), 0, s, p, w_cnt,
                       w_idx, w_beta, w_off, sigma, scale, original_scale, B, sig_out, Omega, flags);
}

template void launch_scatter_outputs<double>(int64_t, const int *, const int *, const double *, const int *,
                                             const double *, const double *, int, double *,
                                             double *, double *, const int *, hipStream_t);
template void launch_scatter_outputs<float>(int64_t, const int *, const int *, const float *, const int *,
                                            const double *, const double *, int, double *,
                                            double *, double *, const int *, hipStream_t);

// The scaled lassos of the response columns k0 .. k0 + m - 1 (design columns
// 0 .. k0 - 1), one wave per response r: beta (k0 x m row-major, zero-filled
// beforehand) takes the nonzero coefficients of column k0 + r, with
// Proposition 1's factor c_j / c_k when `original`, and sigma the noise level
// sigma_k / c_k (sigma_k when not); outer (may be null) the column's count of
// sigma updates.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_lasso(int64_t k0, int64_t m, const int *__restrict__ w_cnt,
                                                       const int *__restrict__ w_idx,
                                                       const T *__restrict__ w_beta,
                                                       const int *__restrict__ w_off,
                                                       const double *__restrict__ sigma,
                                                       const double *__restrict__ scale, int original,
                                                       const int *__restrict__ colinfo,
                                                       double *__restrict__ beta,
                                                       double *__restrict__ sig_out, int *__restrict__ outer,
                                                       const int *__restrict__ flags)
{
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m || *flags) return;
    const int64_t k = k0 + r;
    int wk = w_cnt[k];
    wk = wk < 0 ? 0 : wk;
    const int64_t bk = list_base(w_off, k0 + m, k, wk);
    const double ck = original ? scale[k] : 1.0;
    for (int q = lane; q < wk; q += kWave) {
        const int j = w_idx[bk + q];
        const double b = (double)w_beta[bk + q];
        if (b == 0.0 || j < 0 || (int64_t)j >= k0) continue;
        const double cj = original ? scale[j] : 1.0;
        beta[(int64_t)j * m + r] = b * (cj / ck);
    }
    if (lane == 0) {
        sig_out[r] = sigma[k] / ck;
        if (outer) outer[r] = colinfo[k * 4];
    }
}

template <typename T>
void launch_scatter_lasso(int64_t k0, int64_t m, const int *w_cnt, const int *w_idx, const T *w_beta,
                          const int *w_off, const double *sigma, const double *scale, int original_scale,
                          const int *colinfo, double *beta, double *sig_out, int *outer,
                          const int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter_lasso<T>, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, k0, m, w_cnt,
                       w_idx, w_beta, w_off, sigma, scale, original_scale, colinfo, beta, sig_out, outer, flags);
}

template void launch_scatter_lasso<double>(int64_t, int64_t, const int *, const int *, const double *,
                                           const int *, const double *, const double *, int, const int *,
                                           double *, double *, int *, const int *, hipStream_t);

// Dense symmetrisation of a given Omega_1 (32 x 32 tiles; the partner tile
// is read transposed through LDS so both reads are coalesced).
__global__ __launch_bounds__(256) void k_symmetrize_dense(int64_t p, const double *__restrict__ M,
                                                          double *__restrict__ O)
{
    __shared__ double tr[32][33];
    const int64_t tj = blockIdx.y, tk = blockIdx.x;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // partner tile (tk, tj), stored transposed: tr[c][r] = M[tk*32 + r][tj*32 + c]
    for (int r = ty; r < 32; r += 8) {
        int64_t row = tk * 32 + r, col = tj * 32 + tx;
        tr[tx][r] = (row < p && col < p) ? M[row * p + col] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int64_t j = tj * 32 + r, k = tk * 32 + tx;
        if (j >= p || k >= p) continue;
        double a = M[j * p + k];   // omega_jk,1
        double b = tr[r][tx];      // omega_kj,1
        double v;
        if (j < k) v = fabs(a) <= fabs(b) ? a : b;
        else if (j > k) v = fabs(b) <= fabs(a) ? b : a;
        else v = a;
        O[j * p + k] = v;
    }
}

void launch_symmetrize_dense(int64_t p, const double *Om1, double *Om, hipStream_t s)
{
    unsigned t = (unsigned)((p + 31) / 32);
    hipLaunchKernelGGL(k_symmetrize_dense, dim3(t, t), dim3(256), 0, s, p, Om1, Om);
}

} // namespace spmesl
