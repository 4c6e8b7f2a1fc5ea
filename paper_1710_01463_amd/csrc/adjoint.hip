// Elementwise kernels of the reverse (adjoint) pass of the RSVD with the
// Gaussian test matrix held fixed.  The paper gives no derivative; the
// formulas are the standard ones: the SVD adjoint of a wide matrix with
// orthonormal factors (Townsend 2016; Seeger et al. 2017), with optional
// Lorentzian broadening of 1/(s_j^2 - s_i^2), and the thin-QR adjoint
// (Walter & Lehmann 2018), chained through the products of Alg. RSVD
// (Sec. II.B).  Every product of the reverse pass is an FP64 MFMA GEMM of
// gemm.hip; these kernels stage cotangents and form the small l x l matrices.
//
// Notation for one problem: B = Q^T A (l x n) = Utilde diag(s) Vtilde^T, the
// forward keeps the rotated rows X = P B (row perm[j] = s_j v_j^T) and the
// rotations P (row perm[j] = u_j^T); outputs U = Q Utilde, V^T = Vtilde^T
// with the canonical signs sgn_j, truncated to k_kept.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

template <typename T> __device__ __forceinline__ double ldc(const void* p, int64_t i)
{
    return to_f64(((const GLB T*)p)[i]);
}

int64_t bw_prep_elems(int m, int n, int l) { return (int64_t)m * l + (int64_t)l * n + (int64_t)l * l + l; }
int64_t bw_core_elems(int n, int l) { return (int64_t)l * l + (int64_t)l * n; }
int64_t bw_sym_elems(int l) { return (int64_t)l * l; }

// Cotangent staging and sorted factors, one flat index space per problem:
//   [0, m l)          Ub[i][j]  = sgn_j dU[i][j]            (j < k, zero else)
//   [m l, + l n)      Vbt[j][t] = sgn_j dVT[j][t]           (j < k, zero else)
//                     Vts[j][t] = X[perm_j][t] / s_j        (zero when s_j = 0)
//   [.., + l l)       Ut[r][j]  = P[perm_j][r]
//   [.., + l)         sb[j]     = dS[j] if sgn_j != 0       (j < k, zero else)
// sgn_j = 0 marks the triplets the truncation dropped: their outputs are
// constant zeros, so their cotangents do not enter.
template <typename TE>
__global__ __launch_bounds__(256) void bw_prep_kernel(const BwDesc* __restrict__ descs,
                                                      const int* __restrict__ blk_begin, int nprob)
{
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(blk_begin, t);
    const int b = wi_.x;
    const BwDesc& d = descs[b];
    const int64_t m = d.m, n = d.n, l = d.l, k = d.k;
    const int64_t e1 = m * l, e2 = e1 + l * n, e3 = e2 + l * l, e4 = e3 + l;
    const GLB double* __restrict__ sgn = to_glb(d.sgn);
    const int64_t base = (int64_t)wi_.y * BW_ELEMS_PER_BLOCK + threadIdx.x;
#pragma unroll
    for (int u = 0; u < BW_ELEMS_PER_BLOCK / 256; ++u) {
        const int64_t e = base + 256 * u;
        if (e >= e4) break;
        if (e < e1) {
            const int64_t i = e / l, j = e % l;
            double v = 0.0;
            if (j < k) v = sgn[j] * ldc<TE>(d.dU, i * d.ldu + j);
            to_glb(d.Ub)[e] = v;
        } else if (e < e2) {
            const int64_t f = e - e1;
            const int64_t j = f / n, c = f % n;
            double v = 0.0;
            if (j < k) v = sgn[j] * ldc<TE>(d.dVT, j * d.ldvt + c);
            to_glb(d.Vbt)[f] = v;
            const double sj = to_glb(d.sig)[j];
            const int src = to_glb(d.perm)[j];
            to_glb(d.Vts)[f] = (sj > 0.0) ? to_glb(d.X)[(int64_t)src * n + c] / sj : 0.0;
        } else if (e < e3) {
            const int64_t f = e - e2;
            const int64_t r = f / l, j = f % l;
            const int src = to_glb(d.perm)[j];
            to_glb(d.Ut)[f] = to_glb(d.P)[(int64_t)src * l + r];
        } else {
            const int64_t j = e - e3;
            double v = 0.0;
            if (j < k && sgn[j] != 0.0) v = ldc<TE>(d.dS, j);
            to_glb(d.sb)[j] = v;
        }
    }
}

// 1 / (s_j^2 - s_i^2) (i != j), or its Lorentzian broadening d / (d^2 + eps).
__device__ __forceinline__ double bw_f(double si, double sj, double eps)
{
    const double dd = sj * sj - si * si;
    if (eps > 0.0) return dd / (dd * dd + eps);
    return dd != 0.0 ? 1.0 / dd : 0.0;
}

// Core of the SVD adjoint, written so that the whole of N = Kp Vtilde^T +
// Sigma^-1 Vbar^T takes one GEMM:
//   Kp[i][j] = delta_ij sb_i + F_ij (EU_ij - EU_ji) s_j + s_i F_ij (EV_ij - EV_ji)
//              - EV_ji / s_i                    (the projector term; 0 if s_i = 0)
//   Vbt[i][:] *= 1 / s_i                        (0 if s_i = 0)
// so that Bbar = Utilde N.
__global__ __launch_bounds__(256) void bw_core_kernel(const BwDesc* __restrict__ descs,
                                                      const int* __restrict__ blk_begin, int nprob)
{
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(blk_begin, t);
    const int b = wi_.x;
    const BwDesc& d = descs[b];
    const int64_t n = d.n, l = d.l;
    const int64_t e1 = l * l, e2 = e1 + l * n;
    const GLB double* __restrict__ s = to_glb(d.sig);
    const double s1 = s[0];
    const double eps = d.broad * (s1 * s1) * (s1 * s1);
    const int64_t base = (int64_t)wi_.y * BW_ELEMS_PER_BLOCK + threadIdx.x;
#pragma unroll
    for (int u = 0; u < BW_ELEMS_PER_BLOCK / 256; ++u) {
        const int64_t e = base + 256 * u;
        if (e >= e2) break;
        if (e < e1) {
            const int64_t i = e / l, j = e % l;
            const double si = s[i], sj = s[j];
            const double eu_ij = to_glb(d.EU)[i * l + j], eu_ji = to_glb(d.EU)[j * l + i];
            const double ev_ij = to_glb(d.EV)[i * l + j], ev_ji = to_glb(d.EV)[j * l + i];
            double v;
            if (i == j) {
                v = to_glb(d.sb)[i];
            } else {
                const double f = bw_f(si, sj, eps);
                v = f * (eu_ij - eu_ji) * sj + si * (f * (ev_ij - ev_ji));
            }
            if (si > 0.0) v -= ev_ji / si;
            to_glb(d.Kp)[e] = v;
        } else {
            const int64_t f = e - e1;
            const double si = s[f / n];
            GLB double* V = to_glb(d.Vbt);
            V[f] = (si > 0.0) ? V[f] / si : 0.0;
        }
    }
}

// S = -copyltu(C), copyltu(C) = tril(C) + tril(C, -1)^T.
__global__ __launch_bounds__(256) void bw_sym_kernel(const BwDesc* __restrict__ descs,
                                                     const int* __restrict__ blk_begin, int nprob)
{
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(blk_begin, t);
    const int b = wi_.x;
    const BwDesc& d = descs[b];
    const int64_t l = d.l;
    const int64_t base = (int64_t)wi_.y * BW_ELEMS_PER_BLOCK + threadIdx.x;
#pragma unroll
    for (int u = 0; u < BW_ELEMS_PER_BLOCK / 256; ++u) {
        const int64_t e = base + 256 * u;
        if (e >= l * l) break;
        const int64_t i = e / l, j = e % l;
        to_glb(d.S)[e] = -((i >= j) ? to_glb(d.C)[e] : to_glb(d.C)[j * l + i]);
    }
}

hipError_t launch_bw_prep(const BwDesc* d, const int* blk_begin, int nprob, int total, int cot_f64,
                          hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    if (cot_f64)
        hipLaunchKernelGGL(bw_prep_kernel<double>, dim3(total), dim3(256), 0, s, d, blk_begin, nprob);
    else
        hipLaunchKernelGGL(bw_prep_kernel<float>, dim3(total), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

hipError_t launch_bw_core(const BwDesc* d, const int* blk_begin, int nprob, int total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(bw_core_kernel, dim3(total), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

hipError_t launch_bw_sym(const BwDesc* d, const int* blk_begin, int nprob, int total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(bw_sym_kernel, dim3(total), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

}  // namespace rsvd
