// Orthonormalisation of the sample matrices (paper Sec. II.B, Alg. RSVD step 3,
// and the re-orthonormalisation after every product of the power iteration).
//
// Cholesky QR: with the Gram matrix G = M^T M computed in FP64 by the batched
// GEMM, factor G = L L^T and form Q = M L^-T.  Two passes (CholQR2) give an
// orthonormal Q to working precision when M is not too ill conditioned.  A
// pivot that falls below a relative threshold flags the problem, and the
// Householder kernel recomputes that problem's Q from the original M.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

constexpr int CHOL_W = 16;
// A pivot d_j of the Cholesky factorisation equals ||m_j||^2 sin^2 of the angle
// between column j and the previous columns; below this fraction of ||m_j||^2
// the factor no longer yields an orthonormal Q and Householder takes over.
constexpr double CHOL_PIVOT_REL = 1e-13;

template <typename T> __device__ __forceinline__ double ld_any(const void* p, int64_t i)
{
    return to_f64(((const T*)p)[i]);
}
__device__ __forceinline__ double ld_elem(const void* p, int elem, int64_t i)
{
    if (elem == E_F64) return ld_any<double>(p, i);
    if (elem == E_F32) return ld_any<float>(p, i);
    return ld_any<__bf16>(p, i);
}

// ---------------------------------------------------------------- Cholesky
// One workgroup per problem; blocked left-looking, 16-column panels kept in LDS.
__global__ __launch_bounds__(256) void chol_kernel(const QrDesc* __restrict__ descs)
{
    extern __shared__ double smem[];
    __shared__ double T[CHOL_W][64 + 1];
    __shared__ int bad;
    const QrDesc& d = descs[blockIdx.x];
    if (d.Qout == nullptr || *d.flag) return;
    const int l = d.l;
    const double* __restrict__ G = d.G;
    double* __restrict__ L = d.L;
    double* Pn = smem;  // (l) x CHOL_W panel, row r = global row J + r
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;

    for (int J = 0; J < l; J += CHOL_W) {
        const int w = min(CHOL_W, l - J);
        const int rows = l - J;
        for (int e = tid; e < rows * CHOL_W; e += 256) {
            const int r = e / CHOL_W, c = e % CHOL_W;
            Pn[e] = (c < w) ? G[(int64_t)(J + r) * l + J + c] : 0.0;
        }
        __syncthreads();
        // left-looking update with the already factored columns 0..J-1
        for (int t0 = 0; t0 < J; t0 += 64) {
            const int tw = min(64, J - t0);
            for (int e = tid; e < CHOL_W * 64; e += 256) {
                const int c = e / 64, tt = e % 64;
                T[c][tt] = (c < w && tt < tw) ? L[(int64_t)(J + c) * l + t0 + tt] : 0.0;
            }
            __syncthreads();
            for (int e = tid; e < rows * CHOL_W; e += 256) {
                const int r = e / CHOL_W, c = e % CHOL_W;
                if (c < w && r >= c) {
                    const double* __restrict__ Lr = L + (int64_t)(J + r) * l + t0;
                    double s = 0.0;
                    for (int tt = 0; tt < tw; ++tt) s = fma(Lr[tt], T[c][tt], s);
                    Pn[e] -= s;
                }
            }
            __syncthreads();
        }
        // factor the panel column by column
        for (int c = 0; c < w; ++c) {
            if (tid == 0) {
                const double d0 = Pn[c * CHOL_W + c];
                const double gjj = G[(int64_t)(J + c) * l + J + c];
                if (!(d0 > CHOL_PIVOT_REL * gjj) || !(d0 < INFINITY)) bad = 1;
                Pn[c * CHOL_W + c] = bad ? 1.0 : sqrt(d0);
            }
            __syncthreads();
            if (bad) break;
            const double piv = Pn[c * CHOL_W + c];
            for (int r = c + 1 + tid; r < rows; r += 256) Pn[r * CHOL_W + c] /= piv;
            __syncthreads();
            for (int e = tid; e < rows * CHOL_W; e += 256) {
                const int r = e / CHOL_W, cc = e % CHOL_W;
                if (cc > c && cc < w && r >= cc) Pn[e] -= Pn[r * CHOL_W + c] * Pn[cc * CHOL_W + c];
            }
            __syncthreads();
        }
        if (bad) break;
        for (int e = tid; e < rows * CHOL_W; e += 256) {
            const int r = e / CHOL_W, c = e % CHOL_W;
            if (c < w) L[(int64_t)(J + r) * l + J + c] = (r >= c) ? Pn[e] : 0.0;
        }
        __syncthreads();
    }
    __syncthreads();
    if (tid == 0 && bad) *d.flag = 1;
}

// ---------------------------------------------------------------- Q = M L^-T
// Each workgroup owns 16 rows of M and runs a blocked forward substitution
// L q^T = m^T for its rows (no explicit inverse).
__global__ __launch_bounds__(256) void trsm_kernel(const QrDesc* __restrict__ descs,
                                                   const int* __restrict__ row_begin, int nprob,
                                                   int from_min)
{
    extern __shared__ double smem[];
    __shared__ double Ld[16][17];
    const int t = blockIdx.x;
    const int b = find_problem(row_begin, nprob, t);
    const QrDesc& d = descs[b];
    if (d.Qout == nullptr || *d.flag) return;
    const int l = d.l, rows = d.rows;
    const int ldq = l + 1;
    const int r0 = (t - row_begin[b]) * 16;
    const int nr = min(16, rows - r0);
    const double* __restrict__ L = d.L;
    double* Qs = smem;  // 16 x ldq
    const int tid = threadIdx.x;

    for (int e = tid; e < 16 * l; e += 256) {
        const int r = e / l, c = e % l;
        double v = 0.0;
        if (r < nr) {
            const int64_t gi = (int64_t)(r0 + r) * l + c;
            v = from_min ? ld_elem(d.Min, d.min_elem, gi) : d.Qout[gi];
        }
        Qs[r * ldq + c] = v;
    }
    __syncthreads();
    for (int C0 = 0; C0 < l; C0 += 16) {
        const int w = min(16, l - C0);
        {
            const int i = tid >> 4, j = tid & 15;
            Ld[i][j] = (i < w && j < w) ? L[(int64_t)(C0 + i) * l + C0 + j] : 0.0;
        }
        {
            const int r = tid >> 4, c = tid & 15;
            if (r < nr && c < w && C0 > 0) {
                const double* __restrict__ Lr = L + (int64_t)(C0 + c) * l;
                const double* Qr = Qs + r * ldq;
                double s = 0.0;
                for (int t2 = 0; t2 < C0; ++t2) s = fma(Lr[t2], Qr[t2], s);
                Qs[r * ldq + C0 + c] -= s;
            }
        }
        __syncthreads();
        if (tid < nr) {
            double* Qr = Qs + tid * ldq + C0;
            for (int c = 0; c < w; ++c) {
                double s = Qr[c];
                for (int t2 = 0; t2 < c; ++t2) s -= Ld[c][t2] * Qr[t2];
                Qr[c] = s / Ld[c][c];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < nr * l; e += 256) {
        const int r = e / l, c = e % l;
        d.Qout[(int64_t)(r0 + r) * l + c] = Qs[r * ldq + c];
    }
}

// ---------------------------------------------------------------- Householder
// One workgroup per flagged problem: in-place Householder QR of a copy of M in
// Qout, then the explicit thin Q formed in place from the reflectors, and the
// sign convention diag(R) >= 0.  Always orthonormal, also for rank-deficient M.
constexpr int HH_MAXL = 2048;

__device__ __forceinline__ double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = (red[0] + red[1]) + (red[2] + red[3]);
    return s;
}

__global__ __launch_bounds__(256) void householder_kernel(const QrDesc* __restrict__ descs)
{
    __shared__ double tau_s[HH_MAXL];
    __shared__ double beta_s[HH_MAXL];
    __shared__ double red[4];
    const QrDesc& d = descs[blockIdx.x];
    if (d.Qout == nullptr || !*d.flag) return;
    const int rows = d.rows, l = d.l;
    double* __restrict__ A = d.Qout;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int64_t e = tid; e < (int64_t)rows * l; e += 256) A[e] = ld_elem(d.Min, d.min_elem, e);
    __syncthreads();

    for (int j = 0; j < l; ++j) {
        double p = 0.0;
        for (int i = j + 1 + tid; i < rows; i += 256) {
            const double x = A[(int64_t)i * l + j];
            p = fma(x, x, p);
        }
        const double xn2 = block_sum(p, red);
        const double alpha = A[(int64_t)j * l + j];
        double tau = 0.0, beta = alpha;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            const double scal = 1.0 / (alpha - beta);
            for (int i = j + 1 + tid; i < rows; i += 256) A[(int64_t)i * l + j] *= scal;
        }
        __syncthreads();
        if (tid == 0) {
            A[(int64_t)j * l + j] = beta;
            tau_s[j] = tau;
            beta_s[j] = beta;
        }
        __syncthreads();
        if (tau != 0.0) {
            for (int c = j + 1 + wave; c < l; c += 4) {
                double s = (lane == 0) ? A[(int64_t)j * l + c] : 0.0;
                for (int i = j + 1 + lane; i < rows; i += 64) s = fma(A[(int64_t)i * l + j], A[(int64_t)i * l + c], s);
                s = wave_sum(s) * tau;
                if (lane == 0) A[(int64_t)j * l + c] -= s;
                for (int i = j + 1 + lane; i < rows; i += 64) A[(int64_t)i * l + c] -= s * A[(int64_t)i * l + j];
            }
        }
        __syncthreads();
    }
    // form Q in place from the reflectors, last one first
    for (int j = l - 1; j >= 0; --j) {
        const double tau = tau_s[j];
        if (tau != 0.0) {
            for (int c = j + 1 + wave; c < l; c += 4) {
                double s = (lane == 0) ? A[(int64_t)j * l + c] : 0.0;
                for (int i = j + 1 + lane; i < rows; i += 64) s = fma(A[(int64_t)i * l + j], A[(int64_t)i * l + c], s);
                s = wave_sum(s) * tau;
                if (lane == 0) A[(int64_t)j * l + c] -= s;
                for (int i = j + 1 + lane; i < rows; i += 64) A[(int64_t)i * l + c] -= s * A[(int64_t)i * l + j];
            }
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < rows; i += 256) A[(int64_t)i * l + j] *= -tau;
        if (tid == 0) A[(int64_t)j * l + j] = 1.0 - tau;
        for (int i = tid; i < j; i += 256) A[(int64_t)i * l + j] = 0.0;
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)rows * l; e += 256) {
        const int c = (int)(e % l);
        if (beta_s[c] < 0.0) A[e] = -A[e];
    }
}

hipError_t launch_chol(const QrDesc* d, int nprob, int max_l, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    const size_t lds = (size_t)max_l * CHOL_W * sizeof(double);
    hipLaunchKernelGGL(chol_kernel, dim3(nprob), dim3(256), lds, s, d);
    return hipGetLastError();
}

hipError_t launch_trsm(const QrDesc* d, const int* row_begin, int nprob, int total_blocks,
                           int from_min, int max_l, hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    const size_t lds = (size_t)16 * (max_l + 1) * sizeof(double);
    hipLaunchKernelGGL(trsm_kernel, dim3(total_blocks), dim3(256), lds, s, d, row_begin, nprob, from_min);
    return hipGetLastError();
}

hipError_t init_qr_kernels()
{
    hipError_t e = hipFuncSetAttribute((const void*)chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       CHOL_MAX_L * CHOL_W * (int)sizeof(double));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)trsm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               16 * (CHOL_MAX_L + 1) * (int)sizeof(double));
}

hipError_t launch_householder(const QrDesc* d, int nprob, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(householder_kernel, dim3(nprob), dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace rsvd
