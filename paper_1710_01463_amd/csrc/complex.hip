// Complex matrices (the paper's simulations run in complex double, Sec. IV):
// the RSVD of Alg. RSVD and the full-SVD truncation of Alg. TSVD are run on
// the real embedding At = [[Ar, -Ai], [Ai, Ar]] of A, whose singular values
// are A's, each twice, with left vectors [u_r; u_i] and [-u_i; u_r] (the
// embedding of u and of i u) and right vectors likewise.  The sketch uses
// the embedding of a complex Gaussian test matrix, so every product of the
// range finder is the embedding of the corresponding complex product with
// A^H in place of A^T, and the computed subspaces are the embeddings of the
// complex ones.  This file turns the real triplets back into complex ones.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

constexpr int CF_T = 256;
constexpr int CF_MAXK2 = 2048;  // 2k real values per problem at most

// Block-wide sum of a complex value (all CF_T threads call it).
__device__ __forceinline__ void block_csum(double& re, double& im, double* red)
{
    re = wave_sum(re);
    im = wave_sum(im);
    const int tid = threadIdx.x, wv = tid >> 6;
    __syncthreads();
    if ((tid & 63) == 0) {
        red[2 * wv] = re;
        red[2 * wv + 1] = im;
    }
    __syncthreads();
    re = (red[0] + red[2]) + (red[4] + red[6]);
    im = (red[1] + red[3]) + (red[5] + red[7]);
}

// One workgroup per problem: the complex vectors from the sorted real
// triplets, then the truncation rule, the discarded weight and S.
//
// The real triplets come in pairs (x, Jx) per complex value (J: multiplication
// by i).  Candidates are taken in sorted order; each is made orthogonal, in
// the complex inner product, to the vectors already kept whose singular
// values lie within CPLX_MIX_REL sigma_1 of its own (classical Gram-Schmidt,
// twice, eight vectors per pass), and kept if a unit fraction of it remains.
// The partner of a kept vector leaves nothing and is dropped; a degenerate
// cluster yields an orthonormal basis of its span; and the real Jacobi's
// mixing of close values, of order u sigma_1 / |sigma_i - sigma_j|, is removed
// wherever it exceeds u / CPLX_MIX_REL, while values further apart are left
// untouched.  The same combinations are applied to the right vectors, so
// A v = sigma u holds.  Kept vectors go to U (columns) and VT (rows, not yet
// conjugated); the gather kernel applies the canonical phases.
constexpr int CF_GS = 8;
__global__ __launch_bounds__(CF_T) void complex_select_kernel(const CFinDesc* __restrict__ descs)
{
    __shared__ double sr[CF_MAXK2];
    __shared__ double red[2 * CF_GS * (CF_T / 64)];
    __shared__ double coef[2 * CF_GS];
    const CFinDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = d.m, n = d.n, k = d.k, k2 = 2 * k;
    const GLB double* __restrict__ Sr = to_glb(d.Sr);
    for (int t = tid; t < k2; t += CF_T) sr[t] = Sr[t];
    __syncthreads();
    const GLB double* __restrict__ Ur = to_glb(d.Ur);
    const GLB double* __restrict__ VTr = to_glb(d.VTr);
    GLB double* __restrict__ U = to_glb(d.U);
    GLB double* __restrict__ VT = to_glb(d.VT);
    GLB double* __restrict__ sig = to_glb(d.sig);
    const int64_t ldu = d.ldu, ldv = d.ldvt;
    const double s1 = k2 > 0 ? sr[0] : 0.0;
    int j = 0;     // vectors kept
    int p0 = 0;    // first kept vector inside the current candidate's window
    for (int r = 0; r < k2 && j < k; ++r) {
        // candidate into slot j
        for (int i = tid; i < m; i += CF_T) {
            U[2 * ((int64_t)i * ldu + j)] = Ur[(int64_t)i * k2 + r];
            U[2 * ((int64_t)i * ldu + j) + 1] = Ur[(int64_t)(m + i) * k2 + r];
        }
        for (int c = tid; c < n; c += CF_T) {
            VT[2 * ((int64_t)j * ldv + c)] = VTr[(int64_t)r * 2 * n + c];
            VT[2 * ((int64_t)j * ldv + c) + 1] = VTr[(int64_t)r * 2 * n + n + c];
        }
        while (p0 < j && sig[p0] - sr[r] > CPLX_MIX_REL * s1) ++p0;  // uniform
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int pb = p0; pb < j; pb += CF_GS) {
                const int np = min(CF_GS, j - pb);
                // coef_p = <u_p, u> = sum_i conj(u_p[i]) u[i], p = pb .. pb + np - 1
                double acc[2 * CF_GS];
#pragma unroll
                for (int q = 0; q < 2 * CF_GS; ++q) acc[q] = 0.0;
                for (int i = tid; i < m; i += CF_T) {
                    const GLB double* row = U + 2 * (int64_t)i * ldu;
                    const double ur = row[2 * j], ui = row[2 * j + 1];
#pragma unroll
                    for (int q = 0; q < CF_GS; ++q) {
                        if (q < np) {
                            const double pr = row[2 * (pb + q)], pi = row[2 * (pb + q) + 1];
                            acc[2 * q] = fma(pr, ur, fma(pi, ui, acc[2 * q]));
                            acc[2 * q + 1] = fma(pr, ui, fma(-pi, ur, acc[2 * q + 1]));
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < 2 * CF_GS; ++q) {
                    const double v = wave_sum(acc[q]);
                    if (lane == 0) red[wv * 2 * CF_GS + q] = v;
                }
                __syncthreads();
                if (tid < 2 * CF_GS) {
                    double t2 = 0.0;
                    for (int w = 0; w < CF_T / 64; ++w) t2 += red[w * 2 * CF_GS + tid];
                    coef[tid] = t2;
                }
                __syncthreads();
                // u -= sum_p coef_p u_p, v -= sum_p coef_p v_p
                for (int i = tid; i < m; i += CF_T) {
                    GLB double* row = U + 2 * (int64_t)i * ldu;
                    double ur = row[2 * j], ui = row[2 * j + 1];
                    for (int q = 0; q < np; ++q) {
                        const double pr = row[2 * (pb + q)], pi = row[2 * (pb + q) + 1];
                        const double cr = coef[2 * q], ci = coef[2 * q + 1];
                        ur -= cr * pr - ci * pi;
                        ui -= cr * pi + ci * pr;
                    }
                    row[2 * j] = ur;
                    row[2 * j + 1] = ui;
                }
                for (int q = 0; q < np; ++q) {
                    const double cr = coef[2 * q], ci = coef[2 * q + 1];
                    for (int c = tid; c < n; c += CF_T) {
                        const int64_t a = 2 * ((int64_t)(pb + q) * ldv + c), b = 2 * ((int64_t)j * ldv + c);
                        const double pr = VT[a], pi = VT[a + 1];
                        VT[b] -= cr * pr - ci * pi;
                        VT[b + 1] -= cr * pi + ci * pr;
                    }
                }
                __syncthreads();
            }
        }
        double nr = 0.0, dummy = 0.0;
        for (int i = tid; i < m; i += CF_T) {
            const int64_t b = 2 * ((int64_t)i * ldu + j);
            nr = fma(U[b], U[b], fma(U[b + 1], U[b + 1], nr));
        }
        block_csum(nr, dummy, red);
        if (nr > 0.25) {  // a new direction: keep it, normalised (v scaled alike)
            const double sc = 1.0 / sqrt(nr);
            for (int i = tid; i < m; i += CF_T) {
                const int64_t b = 2 * ((int64_t)i * ldu + j);
                U[b] *= sc;
                U[b + 1] *= sc;
            }
            for (int c = tid; c < n; c += CF_T) {
                const int64_t b = 2 * ((int64_t)j * ldv + c);
                VT[b] *= sc;
                VT[b + 1] *= sc;
            }
            if (tid == 0) sig[j] = sr[r];
            ++j;
        }
        __syncthreads();
    }
    // triplets the 2k real ones could not supply (rank deficiency): zero
    for (int jj = j + tid; jj < k; jj += CF_T) sig[jj] = -1.0;
    __syncthreads();
    if (tid == 0) {
        // truncation on the complex values, as for the real RSVD / full SVD
        const double a2 = *to_glb(d.normA2) * 0.5;
        int info = *to_glb(d.info_in);
        int kk = 0;
        double w = 0.0;
        auto sg = [&](int q) { return fmax(sig[q], 0.0); };
        if (!(a2 < INFINITY)) {
            info = -4;
            w = a2;
        } else if (a2 == 0.0) {
            kk = 0;
        } else {
            auto weight = [&](int kp) {
                double s = 0.0, c = 0.0;
                if (d.full) {
                    // tail: the embedded problem's weight beyond its 2k values, halved, plus sigma_j^2, j >= kp
                    s = *to_glb(d.wr) * 0.5;
                    for (int q = kp; q < k; ++q) {
                        const double x = sg(q) * sg(q);
                        const double t2 = s + x;
                        c += (fabs(s) >= fabs(x)) ? (s - t2) + x : (x - t2) + s;
                        s = t2;
                    }
                } else {
                    s = a2;
                    for (int q = 0; q < kp; ++q) {
                        const double x = -sg(q) * sg(q);
                        const double t2 = s + x;
                        c += (fabs(s) >= fabs(x)) ? (s - t2) + x : (x - t2) + s;
                        s = t2;
                    }
                }
                return fmax(0.0, s + c);
            };
            kk = j;  // at most the vectors found
            if (d.delta > 0.0) {
                for (int kp = 1; kp <= j; ++kp)
                    if (weight(kp) <= d.delta * a2) {
                        kk = kp;
                        break;
                    }
            }
            w = weight(kk);
        }
        if (info == -4) kk = 0;
        *to_glb(d.w_out) = w;
        *to_glb(d.kkept_out) = kk;
        *to_glb(d.info_out) = info;
    }
    __syncthreads();
    const int kk = (int)*to_glb(d.kkept_out);
    for (int q = tid; q < k; q += CF_T) to_glb(d.S)[q] = q < kk ? sig[q] : 0.0;
}

// One wave per (problem, triplet j): the complex vectors of triplet j with the
// canonical phase (the entry of u of largest modulus, lowest index on ties,
// made real and positive; the row of V^H takes the conjugate phase), written
// interleaved; zero beyond k_kept.
__global__ __launch_bounds__(64) void complex_gather_kernel(const CFinDesc* __restrict__ descs,
                                                            const int* __restrict__ col_map, int nprob)
{
    const int2 wi_ = wg_item(col_map, blockIdx.x);
    const CFinDesc& d = descs[wi_.x];
    const int j = wi_.y, lane = threadIdx.x;
    const int m = d.m, n = d.n;
    const int kk = (int)*to_glb(d.kkept_out);
    GLB double* __restrict__ U = to_glb(d.U);
    GLB double* __restrict__ VT = to_glb(d.VT);
    if (j >= kk) {
        for (int i = lane; i < m; i += 64) {
            U[2 * ((int64_t)i * d.ldu + j)] = 0.0;
            U[2 * ((int64_t)i * d.ldu + j) + 1] = 0.0;
        }
        for (int c = lane; c < n; c += 64) {
            VT[2 * ((int64_t)j * d.ldvt + c)] = 0.0;
            VT[2 * ((int64_t)j * d.ldvt + c) + 1] = 0.0;
        }
        return;
    }
    auto u_at = [&](int i, double& re, double& im) {
        re = U[2 * ((int64_t)i * d.ldu + j)];
        im = U[2 * ((int64_t)i * d.ldu + j) + 1];
    };
    // largest modulus, first index on ties
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < m; i += 64) {
        double re, im;
        u_at(i, re, im);
        const double a = fma(re, re, im * im);
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
    double pr, pi;
    u_at(bi, pr, pi);
    const double mag = sqrt(fma(pr, pr, pi * pi));
    const double cr = mag > 0.0 ? pr / mag : 1.0, ci = mag > 0.0 ? pi / mag : 0.0;  // ph = u[big] / |u[big]|
    // U[:, j] = u conj(ph); all reads of this column happen before any write
    double ure[32], uim[32];
    for (int i0 = 0; i0 < m; i0 += 64 * 32) {
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int i = i0 + lane + 64 * q;
            if (i < m) u_at(i, ure[q], uim[q]);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int i = i0 + lane + 64 * q;
            if (i < m) {
                U[2 * ((int64_t)i * d.ldu + j)] = ure[q] * cr + uim[q] * ci;
                U[2 * ((int64_t)i * d.ldu + j) + 1] = uim[q] * cr - ure[q] * ci;
            }
        }
    }
    // VT[j, :] = conj(v) ph
    for (int c = lane; c < n; c += 64) {
        const double vr = VT[2 * ((int64_t)j * d.ldvt + c)];
        const double vi = VT[2 * ((int64_t)j * d.ldvt + c) + 1];
        VT[2 * ((int64_t)j * d.ldvt + c)] = vr * cr + vi * ci;
        VT[2 * ((int64_t)j * d.ldvt + c) + 1] = vr * ci - vi * cr;
    }
}

hipError_t launch_complex_finish(const CFinDesc* d, int nprob, const int* col_map, int col_total, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(complex_select_kernel, dim3(nprob), dim3(CF_T), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || col_total <= 0) return e;
    hipLaunchKernelGGL(complex_gather_kernel, dim3(col_total), dim3(64), 0, s, d, col_map, nprob);
    return hipGetLastError();
}

}  // namespace rsvd
