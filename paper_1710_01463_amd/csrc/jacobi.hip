// Block one-sided Jacobi SVD (Hestenes), used for
//   - the small SVD of B = Q^T A in Alg. RSVD step 4 (paper Sec. II.B; the
//     paper uses LAPACK GESVD there, any backward-stable SVD serves), and
//   - the full SVD of Alg. TSVD (Sec. II.A), the deterministic baseline.
//
// The vectors being orthogonalised are the R rows of X (R x C, R <= C); the
// left rotations are accumulated in P (R x R), so that P X_in = X_out with
// mutually orthogonal rows.  Rows are grouped in blocks of 16.  One launch is
// one round of the round-robin schedule over the nb blocks: each workgroup
// takes one block pair (32 rows), forms their 32 x 32 Gram matrix with FP64
// MFMA, checks the relative off-diagonal |h_ij| <= tol sqrt(h_ii h_jj), and
// if needed diagonalises it by cyclic two-sided Jacobi in LDS, then applies
// the accumulated 32 x 32 rotation to the 32 rows of X and of P with FP64
// MFMA.  A sweep is nb - 1 rounds; a problem is converged after a sweep in
// which no block pair needed a rotation.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

constexpr int JR = 2 * JAC_B;  // rows per block pair
constexpr int JCH = 128;       // column chunk staged through LDS
constexpr int JPF = JR * JCH / 256;  // prefetched doubles per thread

__device__ __forceinline__ int rr_block(int pos, int round, int nb)
{
    return pos == 0 ? 0 : ((pos - 1 + round) % (nb - 1)) + 1;
}

// Rotation (c, s) that zeroes the (p, q) entry of a symmetric 2 x 2 block
// [a g; g b] under x_p <- c x_p - s x_q, x_q <- s x_p + c x_q (the classical
// Hestenes/Jacobi formula).  Identity when |g| <= tol sqrt(a b).
__device__ __forceinline__ void jac_rotation(double a, double b, double g, double tol, double& cs, double& sn)
{
    cs = 1.0;
    sn = 0.0;
    if (a > 0.0 && b > 0.0 && g * g > tol * tol * a * b) {
        const double zeta = (b - a) / (2.0 * g);
        double t;
        if (fabs(zeta) > 1e150)
            t = 0.5 / zeta;
        else
            t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        cs = rsqrt(1.0 + t * t);
        sn = cs * t;
    }
}

// Loads the 32 x JCH chunk (rows via rowmap, columns c0..) of M into registers.
__device__ __forceinline__ void load_chunk(double (&pre)[JPF], const double* __restrict__ M, int64_t ldm,
                                           int ncols, int c0, const int* rowmap)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < JPF; ++i) {
        const int e = tid + 256 * i;
        const int a = e / JCH, cc = e % JCH;
        const int gr = rowmap[a], gc = c0 + cc;
        pre[i] = (gr >= 0 && gc < ncols) ? M[(int64_t)gr * ldm + gc] : 0.0;
    }
}
__device__ __forceinline__ void store_chunk(const double (&pre)[JPF], double (*Xs)[JCH + 1])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < JPF; ++i) {
        const int e = tid + 256 * i;
        Xs[e / JCH][e % JCH] = pre[i];
    }
}

// rows of M (32 of them, via rowmap) <- Ps (32 x 32) * rows of M, in place;
// the next chunk is prefetched into registers while the current one is used.
__device__ void apply_rotation(double* __restrict__ M, int64_t ldm, int ncols, const int* rowmap,
                               double (*Ps)[JR + 1], double (*Xs)[JCH + 1])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    double pre[JPF];
    load_chunk(pre, M, ldm, ncols, 0, rowmap);
    for (int c0 = 0; c0 < ncols; c0 += JCH) {
        store_chunk(pre, Xs);
        __syncthreads();
        if (c0 + JCH < ncols) load_chunk(pre, M, ldm, ncols, c0 + JCH, rowmap);
        // 2 row tiles x (JCH / 16) column tiles; wave w takes column tiles w, w + 4, ...
#pragma unroll
        for (int tj = wave; tj < JCH / 16; tj += 4) {
            dbl4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < JR; kk += 4) {
                const double bv = Xs[kk + lq][tj * 16 + l16];
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ps[l16][kk + lq], bv, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ps[16 + l16][kk + lq], bv, acc1, 0, 0, 0);
            }
            const int gc = c0 + tj * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int g0 = rowmap[lq + 4 * r], g1 = rowmap[16 + lq + 4 * r];
                if (gc < ncols) {
                    if (g0 >= 0) M[(int64_t)g0 * ldm + gc] = acc0[r];
                    if (g1 >= 0) M[(int64_t)g1 * ldm + gc] = acc1[r];
                }
            }
        }
        __syncthreads();
    }
}

constexpr int JAC_INNER_SWEEPS = 1;

__global__ __launch_bounds__(256) void jacobi_round_kernel(const JacDesc* __restrict__ descs,
                                                           const int* __restrict__ pair_begin, int nprob,
                                                           int sweep, int round)
{
    __shared__ double Xs[JR][JCH + 1];
    __shared__ double Hbuf[2][JR][JR + 1];
    __shared__ double Ps[JR][JR + 1];
    __shared__ int rowmap[JR];
    __shared__ int any_rot;

    const int t = blockIdx.x;
    const int b = find_problem(pair_begin, nprob, t);
    const JacDesc& d = descs[b];
    const int nb = d.nb;
    if (round >= nb - 1) return;
    if (sweep > 0 && d.rot[sweep - 1] == 0) return;
    const int pi = t - pair_begin[b];
    const int I = rr_block(pi, round, nb);
    const int J = rr_block(nb - 1 - pi, round, nb);
    const int R = d.R, C = d.C;
    const double tol = d.tol;
    double* __restrict__ X = d.X;
    const int64_t ldx = d.ldx;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    if (tid < JR) {
        const int gr = (tid < JAC_B) ? I * JAC_B + tid : J * JAC_B + (tid - JAC_B);
        rowmap[tid] = (gr < R) ? gr : -1;
    }
    if (tid == 0) any_rot = 0;
    __syncthreads();

    // ---- Gram matrix of the 32 rows (FP64 MFMA), one 16 x 16 tile per wave
    {
        const int wi = wave >> 1, wj = wave & 1;
        dbl4 acc = {0, 0, 0, 0};
        double pre[JPF];
        load_chunk(pre, X, ldx, C, 0, rowmap);
        for (int c0 = 0; c0 < C; c0 += JCH) {
            store_chunk(pre, Xs);
            __syncthreads();
            if (c0 + JCH < C) load_chunk(pre, X, ldx, C, c0 + JCH, rowmap);
#pragma unroll 8
            for (int kk = 0; kk < JCH; kk += 4) {
                const double av = Xs[wi * 16 + l16][kk + lq];
                const double bv = Xs[wj * 16 + l16][kk + lq];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Hbuf[0][wi * 16 + lq + 4 * r][wj * 16 + l16] = acc[r];
    }
    __syncthreads();
    // symmetrise from the upper triangle, identity for P
    for (int e = tid; e < JR * JR; e += 256) {
        const int i = e / JR, j = e % JR;
        if (i > j) Hbuf[0][i][j] = Hbuf[0][j][i];
        Ps[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < JR * JR; e += 256) {
        const int i = e / JR, j = e % JR;
        if (i < j) {
            const double a = Hbuf[0][i][i], c = Hbuf[0][j][j], g = Hbuf[0][i][j];
            if (a > 0.0 && c > 0.0 && g * g > tol * tol * a * c) any_rot = 1;
        }
    }
    __syncthreads();
    if (!any_rot) return;
    if (tid == 0) d.rot[sweep] = 1;

    // ---- inner cyclic Jacobi on the 32 x 32 Gram matrix, parallel order.
    // Thread (pi_, pj_) owns the 2 x 2 block (pair pi_ rows) x (pair pj_ cols)
    // of H and the 2 x 2 block (pair pi_ rows) x (columns 2 pj_, 2 pj_ + 1) of
    // P.  H is double-buffered so one barrier per step suffices.
    const int pr_i = tid >> 4, pr_j = tid & 15;
    int cur = 0;
    for (int isw = 0; isw < JAC_INNER_SWEEPS; ++isw) {
        for (int step = 0; step < JR - 1; ++step) {
            const int p_i = rr_block(pr_i, step, JR), q_i = rr_block(JR - 1 - pr_i, step, JR);
            const int p_j = rr_block(pr_j, step, JR), q_j = rr_block(JR - 1 - pr_j, step, JR);
            double (*H)[JR + 1] = Hbuf[cur];
            double (*Hn)[JR + 1] = Hbuf[cur ^ 1];
            double ci, si, cj, sj;
            jac_rotation(H[p_i][p_i], H[q_i][q_i], H[p_i][q_i], tol, ci, si);
            jac_rotation(H[p_j][p_j], H[q_j][q_j], H[p_j][q_j], tol, cj, sj);
            const double b00 = H[p_i][p_j], b01 = H[p_i][q_j], b10 = H[q_i][p_j], b11 = H[q_i][q_j];
            const double t00 = ci * b00 - si * b10, t01 = ci * b01 - si * b11;
            const double t10 = si * b00 + ci * b10, t11 = si * b01 + ci * b11;
            Hn[p_i][p_j] = t00 * cj - t01 * sj;
            Hn[p_i][q_j] = t00 * sj + t01 * cj;
            Hn[q_i][p_j] = t10 * cj - t11 * sj;
            Hn[q_i][q_j] = t10 * sj + t11 * cj;
            if (si != 0.0) {
                const int c0 = 2 * pr_j, c1 = 2 * pr_j + 1;
                const double x0 = Ps[p_i][c0], x1 = Ps[p_i][c1], y0 = Ps[q_i][c0], y1 = Ps[q_i][c1];
                Ps[p_i][c0] = ci * x0 - si * y0;
                Ps[p_i][c1] = ci * x1 - si * y1;
                Ps[q_i][c0] = si * x0 + ci * y0;
                Ps[q_i][c1] = si * x1 + ci * y1;
            }
            cur ^= 1;
            __syncthreads();
        }
    }

    // ---- apply the accumulated rotation to the rows of X and of P
    apply_rotation(X, ldx, C, rowmap, Ps, Xs);
    if (d.P) apply_rotation(d.P, d.ldp, R, rowmap, Ps, Xs);
}

hipError_t launch_jacobi_round(const JacDesc* d, const int* pair_begin, int nprob, int total_pairs,
                               int sweep, int round, hipStream_t s)
{
    if (total_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(jacobi_round_kernel, dim3(total_pairs), dim3(256), 0, s, d, pair_begin, nprob,
                       sweep, round);
    return hipGetLastError();
}

// ---------------------------------------------------------------- finishing
constexpr int FIN_MAXR = 2048;

template <typename TO>
__global__ __launch_bounds__(256) void finish_kernel(const FinDesc* __restrict__ descs)
{
    __shared__ double sig[FIN_MAXR];
    __shared__ double tail[FIN_MAXR + 1];
    __shared__ int perm_s[FIN_MAXR];
    __shared__ int kk_s;
    const FinDesc& d = descs[blockIdx.x];
    const int R = d.R, C = d.C;
    const double* __restrict__ X = d.X;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int i = wave; i < R; i += 4) {
        double s = 0.0;
        for (int t = lane; t < C; t += 64) {
            const double x = X[(int64_t)i * d.ldx + t];
            s = fma(x, x, s);
        }
        s = wave_sum(s);
        if (lane == 0) sig[i] = sqrt(s);
    }
    __syncthreads();
    // Stable descending rank sort on a total order: NaN (only from non-finite
    // input) sorts last and equal keys keep index order, so the ranks always
    // form a permutation of 0..R-1 (perm is later used as a gather index).
    for (int i = tid; i < R; i += 256) {
        const double si = (sig[i] == sig[i]) ? sig[i] : -1.0;
        int rank = 0;
        for (int j = 0; j < R; ++j) {
            const double sj = (sig[j] == sig[j]) ? sig[j] : -1.0;
            rank += (sj > si) || (sj == si && j < i);
        }
        perm_s[rank] = i;
    }
    __syncthreads();
    for (int j = tid; j < R; j += 256) {
        d.sig[j] = sig[perm_s[j]];
        d.perm[j] = perm_s[j];
    }
    if (tid == 0) {
        const double normA2 = *d.normA2;
        const int k = d.k;
        int info = 0;
        int kk = 0;
        double w = 0.0;
        if (!(normA2 < INFINITY)) {
            info = -4;  // non-finite input
            kk = 0;
            w = normA2;
        } else if (normA2 == 0.0) {
            kk = 0;
            w = 0.0;
        } else {
            // tail[k'] = discarded weight when keeping k' triplets, k' = 0..k
            if (d.mode == 0) {
                double s = normA2, c = 0.0;  // Neumaier-compensated ||A||^2 - sum sigma^2
                tail[0] = normA2;
                for (int j = 1; j <= k; ++j) {
                    const double sj = sig[perm_s[j - 1]];
                    const double x = -sj * sj;
                    const double tsum = s + x;
                    if (fabs(s) >= fabs(x)) c += (s - tsum) + x; else c += (x - tsum) + s;
                    s = tsum;
                    const double v = s + c;
                    tail[j] = v > 0.0 ? v : 0.0;
                }
            } else {
                double s = 0.0, c = 0.0;  // sum of the smallest sigma^2 first
                for (int j = R - 1; j >= 0; --j) {
                    const double sj = sig[perm_s[j]];
                    const double x = sj * sj;
                    const double tsum = s + x;
                    if (fabs(s) >= fabs(x)) c += (s - tsum) + x; else c += (x - tsum) + s;
                    s = tsum;
                    if (j <= k) tail[j] = s + c;
                }
                if (R <= k) tail[R] = 0.0;
            }
            kk = k;
            if (d.delta != 0.0) {
                for (int j = 1; j <= k; ++j)
                    if (tail[j] <= d.delta * normA2) {
                        kk = j;
                        break;
                    }
            }
            w = tail[kk];
        }
        if (info == 0 && d.rot && d.rot[d.max_sweeps - 1] != 0) info = -5;  // sweep cap reached
        kk_s = kk;
        *d.w_out = w;
        *d.kkept_out = kk;
        *d.info_out = info;
    }
    __syncthreads();
    const int kk = kk_s;
    const int k = d.k;
    TO* __restrict__ S = (TO*)d.S;
    TO* __restrict__ U = (TO*)d.U;
    TO* __restrict__ VT = (TO*)d.VT;
    for (int j = tid; j < k; j += 256) S[j] = (j < kk) ? (TO)sig[perm_s[j]] : (TO)0;
    const int n = d.n, m = d.m;
    // right vectors
    for (int j = 0; j < k; ++j) {
        const int src = (j < kk) ? perm_s[j] : -1;
        const double sj = (j < kk) ? sig[src] : 0.0;
        const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
        if (d.mode == 0 || d.mode == 1) {
            for (int t = tid; t < n; t += 256)
                VT[(int64_t)j * d.ldvt + t] = (src >= 0) ? (TO)(X[(int64_t)src * d.ldx + t] * inv) : (TO)0;
        } else {
            for (int t = tid; t < n; t += 256)
                VT[(int64_t)j * d.ldvt + t] = (src >= 0) ? (TO)d.P[(int64_t)src * d.ldp + t] : (TO)0;
        }
        if (d.mode == 1) {
            for (int i = tid; i < m; i += 256)
                U[(int64_t)i * d.ldu + j] = (src >= 0) ? (TO)d.P[(int64_t)src * d.ldp + i] : (TO)0;
        } else if (d.mode == 2) {
            for (int i = tid; i < m; i += 256)
                U[(int64_t)i * d.ldu + j] = (src >= 0) ? (TO)(X[(int64_t)src * d.ldx + i] * inv) : (TO)0;
        }
    }
}

hipError_t launch_finish(const FinDesc* d, int nprob, int out_f64, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    if (out_f64)
        hipLaunchKernelGGL(finish_kernel<double>, dim3(nprob), dim3(256), 0, s, d);
    else
        hipLaunchKernelGGL(finish_kernel<float>, dim3(nprob), dim3(256), 0, s, d);
    return hipGetLastError();
}

template <typename TO>
__global__ __launch_bounds__(64) void signfix_kernel(const FinDesc* __restrict__ descs,
                                                     const int* __restrict__ col_begin, int nprob)
{
    const int t = blockIdx.x;
    const int b = find_problem(col_begin, nprob, t);
    const FinDesc& d = descs[b];
    const int j = t - col_begin[b];
    const int lane = threadIdx.x;
    const int64_t kk = *d.kkept_out;
    TO* __restrict__ U = (TO*)d.U;
    TO* __restrict__ VT = (TO*)d.VT;
    const int m = d.m, n = d.n;
    if (j >= kk) {
        for (int i = lane; i < m; i += 64) U[(int64_t)i * d.ldu + j] = (TO)0;
        return;
    }
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < m; i += 64) {
        const double a = fabs((double)U[(int64_t)i * d.ldu + j]);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    if (bi >= m) return;  // no finite entry: leave the column as it is
    const bool flip = (double)U[(int64_t)bi * d.ldu + j] < 0.0;
    if (flip) {
        for (int i = lane; i < m; i += 64) U[(int64_t)i * d.ldu + j] = -U[(int64_t)i * d.ldu + j];
        for (int x = lane; x < n; x += 64) VT[(int64_t)j * d.ldvt + x] = -VT[(int64_t)j * d.ldvt + x];
    }
}

hipError_t launch_signfix(const FinDesc* d, const int* col_begin, int nprob, int total_cols, int out_f64,
                          hipStream_t s)
{
    if (total_cols <= 0) return hipSuccess;
    if (out_f64)
        hipLaunchKernelGGL(signfix_kernel<double>, dim3(total_cols), dim3(64), 0, s, d, col_begin, nprob);
    else
        hipLaunchKernelGGL(signfix_kernel<float>, dim3(total_cols), dim3(64), 0, s, d, col_begin, nprob);
    return hipGetLastError();
}

}  // namespace rsvd
