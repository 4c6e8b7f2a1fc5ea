// Batched, descriptor-driven MFMA GEMM for the skinny products of the RSVD
// (paper Sec. II.B: the sample Y = A Omega, the power-iteration products A^T Q
// and A Z, the projection B = Q^T A, and the back-projection Q Utilde), plus
// the Gram matrices Y^T Y of the Cholesky-QR orthonormalisation.
//
// One launch covers every problem of a batch: the grid is the concatenation
// of all problems' 64 x 64 output tiles, and each workgroup finds its problem
// by binary search in the tile prefix sums.  Workgroup = 4 waves in a 2 x 2
// arrangement, each wave owning a 32 x 32 sub-tile = 2 x 2 MFMA 16 x 16
// accumulators.  Operand tiles are staged through LDS k-contiguous so every
// MFMA operand read is a single (or 16-byte for bf16) LDS load per lane.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

template <int GK> struct GemmCfg;
template <> struct GemmCfg<GK_F64> {
    typedef double OpT;
    typedef dbl4 Acc4;
    static constexpr int BK = 16;
    static constexpr int PAD = 1;
};
template <> struct GemmCfg<GK_F32> {
    typedef float OpT;
    typedef flt4 Acc4;
    static constexpr int BK = 16;
    static constexpr int PAD = 1;
};
template <> struct GemmCfg<GK_BF16> {
    typedef __bf16 OpT;
    typedef flt4 Acc4;
    static constexpr int BK = 32;
    static constexpr int PAD = 8;
};

template <typename OpT> struct OpConv;
template <> struct OpConv<double> {
    template <typename T> __device__ static double cvt(T x) { return to_f64(x); }
};
template <> struct OpConv<float> {
    template <typename T> __device__ static float cvt(T x) { return to_f32(x); }
};
template <> struct OpConv<__bf16> {
    __device__ static __bf16 cvt(double x) { return from_f64<__bf16>(x); }
    __device__ static __bf16 cvt(float x) { return from_f32<__bf16>(x); }
    __device__ static __bf16 cvt(__bf16 x) { return x; }
};

template <typename TC> __device__ __forceinline__ TC store_cvt(double x) { return from_f64<TC>(x); }

template <int GK, typename TA, typename TX, typename TC>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                    const int* __restrict__ tile_begin, int nprob)
{
    typedef typename GemmCfg<GK>::OpT OpT;
    typedef typename GemmCfg<GK>::Acc4 Acc4;
    constexpr int BK = GemmCfg<GK>::BK;
    constexpr int LDK = BK + GemmCfg<GK>::PAD;
    constexpr int BM = GEMM_BM, BN = GEMM_BN;
    __shared__ __attribute__((aligned(16))) OpT As[BM * LDK];
    __shared__ __attribute__((aligned(16))) OpT Xs[BN * LDK];

    const int t = blockIdx.x;
    const int2 wi_ = wg_item(tile_begin, t);
    const int b = wi_.x;
    const GemmDesc& d = descs[b];
    if (d.skip && *to_glb(d.skip)) return;
    const int local = wi_.y;
    const int m0 = (local / d.tiles_n) * BM;
    const int n0 = (local % d.tiles_n) * BN;
    const int M = d.M, N = d.N, K = d.K;
    const int64_t lda = d.lda, ldx = d.ldx;
    const int transA = d.transA, transX = d.transX;
    const GLB TA* __restrict__ A = (const GLB TA*)d.A;
    const GLB TX* __restrict__ X = (const GLB TX*)d.X;
    const GLB int* __restrict__ gather = to_glb(d.gather);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * 32;
    const int wn = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lq = lane >> 4;

    Acc4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = Acc4{0, 0, 0, 0};

    for (int k0 = 0; k0 < K; k0 += BK) {
        // ---- stage op(A) tile (BM x BK) as As[i][kk]
        for (int e = tid; e < BM * BK; e += 256) {
            int i, kk;
            if (!transA) {
                i = e / BK;
                kk = e % BK;
            } else {
                kk = e / BM;
                i = e % BM;
            }
            const int gi = m0 + i, gk = k0 + kk;
            OpT v = OpConv<OpT>::cvt((TA)0);
            if (gi < M && gk < K)
                v = OpConv<OpT>::cvt(transA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]);
            As[i * LDK + kk] = v;
        }
        // ---- stage op(X) tile (BK x BN) as Xs[j][kk]
        for (int e = tid; e < BK * BN; e += 256) {
            int j, kk;
            if (!transX) {
                kk = e / BN;
                j = e % BN;
            } else {
                j = e / BK;
                kk = e % BK;
            }
            const int gj = n0 + j, gk = k0 + kk;
            OpT v = OpConv<OpT>::cvt((TX)0);
            if (gj < N && gk < K) {
                if (!transX) {
                    v = OpConv<OpT>::cvt(X[(int64_t)gk * ldx + gj]);
                } else {
                    const int row = gather ? gather[gj] : gj;
                    v = OpConv<OpT>::cvt(X[(int64_t)row * ldx + gk]);
                }
            }
            Xs[j * LDK + kk] = v;
        }
        __syncthreads();

        if constexpr (GK == GK_F64) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                double av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = As[(wm + a * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int c = 0; c < 2; ++c) bv[c] = Xs[(wn + c * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
            }
        } else if constexpr (GK == GK_F32) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = As[(wm + a * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int c = 0; c < 2; ++c) bv[c] = Xs[(wn + c * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[c], acc[a][c], 0, 0, 0);
            }
        } else {
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                av[a] = *reinterpret_cast<const bf16x8*>(&As[(wm + a * 16 + l16) * LDK + 8 * lq]);
#pragma unroll
            for (int c = 0; c < 2; ++c)
                bv[c] = *reinterpret_cast<const bf16x8*>(&Xs[(wn + c * 16 + l16) * LDK + 8 * lq]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
        }
        __syncthreads();
    }

    // ---- epilogue
    GLB TC* __restrict__ C = (GLB TC*)d.C;
    const int64_t ldc = d.ldc;
    const int transC = d.transC, accumulate = d.accumulate;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int i, j;
                if constexpr (GK == GK_F64) {
                    i = wm + a * 16 + lq + 4 * r;  // f64 16x16x4 output: row = lane/16 + 4r
                } else {
                    i = wm + a * 16 + 4 * lq + r;  // f32 accumulators: row = 4(lane/16) + r
                }
                j = wn + c * 16 + l16;
                const int gi = m0 + i, gj = n0 + j;
                if (gi < M && gj < N) {
                    const int64_t idx = transC ? (int64_t)gj * ldc + gi : (int64_t)gi * ldc + gj;
                    double v = (double)acc[a][c][r];
                    if (accumulate) v += to_f64(C[idx]);
                    C[idx] = store_cvt<TC>(v);
                }
            }
}

template <int GK, typename TA, typename TX, typename TC>
static hipError_t launch_t(const GemmDesc* descs, const int* tile_begin, int nprob, int total,
                           hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_kernel<GK, TA, TX, TC>), dim3(total), dim3(256), 0, s, descs, tile_begin,
                       nprob);
    return hipGetLastError();
}

template <int GK, typename TA, typename TX>
static hipError_t launch_c(Elem ec, const GemmDesc* d, const int* tb, int np, int tot, hipStream_t s)
{
    switch (ec) {
    case E_F64: return launch_t<GK, TA, TX, double>(d, tb, np, tot, s);
    case E_F32: return launch_t<GK, TA, TX, float>(d, tb, np, tot, s);
    default: return hipErrorInvalidValue;
    }
}

template <int GK, typename TA>
static hipError_t launch_x(Elem ex, Elem ec, const GemmDesc* d, const int* tb, int np, int tot,
                           hipStream_t s)
{
    switch (ex) {
    case E_F64: return launch_c<GK, TA, double>(ec, d, tb, np, tot, s);
    case E_F32: return launch_c<GK, TA, float>(ec, d, tb, np, tot, s);
    case E_BF16: return launch_c<GK, TA, __bf16>(ec, d, tb, np, tot, s);
    }
    return hipErrorInvalidValue;
}

template <int GK>
static hipError_t launch_a(Elem ea, Elem ex, Elem ec, const GemmDesc* d, const int* tb, int np, int tot,
                           hipStream_t s)
{
    switch (ea) {
    case E_F64: return launch_x<GK, double>(ex, ec, d, tb, np, tot, s);
    case E_F32: return launch_x<GK, float>(ex, ec, d, tb, np, tot, s);
    case E_BF16: return launch_x<GK, __bf16>(ex, ec, d, tb, np, tot, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gemm(GemmKind kind, Elem ea, Elem ex, Elem ec, const GemmDesc* descs,
                       const int* tile_begin, int nprob, int total_tiles, hipStream_t stream)
{
    switch (kind) {
    case GK_F64: return launch_a<GK_F64>(ea, ex, ec, descs, tile_begin, nprob, total_tiles, stream);
    case GK_F32: return launch_a<GK_F32>(ea, ex, ec, descs, tile_begin, nprob, total_tiles, stream);
    case GK_BF16: return launch_a<GK_BF16>(ea, ex, ec, descs, tile_begin, nprob, total_tiles, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace rsvd
