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

#include <type_traits>

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

template <int GK, typename TA, typename TX, typename TC, int BM, int BN, bool GATHER>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                    const int* __restrict__ tile_begin, int nprob)
{
    typedef typename GemmCfg<GK>::OpT OpT;
    typedef typename GemmCfg<GK>::Acc4 Acc4;
    constexpr int BK = GemmCfg<GK>::BK;
    constexpr int LDK = BK + GemmCfg<GK>::PAD;
    // 2 x 2 waves, each owning a WTM x WTN sub-tile of FM x FN MFMA 16 x 16 tiles
    constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
    __shared__ __attribute__((aligned(16))) OpT As[BM * LDK];
    __shared__ __attribute__((aligned(16))) OpT Xs[BN * LDK];

    const int t = blockIdx.x;
    const int2 wi_ = wg_item(tile_begin, t);
    const int b = wi_.x;
    const GemmDesc& d = descs[b];
    if (d.skip && *to_glb(d.skip)) return;
    const int local = wi_.y;
    int tm = local / d.tiles_n, tn = local % d.tiles_n;
    if (d.lower) {
        // local = tm (tm + 1) / 2 + tn, tn <= tm
        tm = (int)((__builtin_sqrtf(8.0f * (float)local + 1.0f) - 1.0f) * 0.5f);
        while (tm > 0 && tm * (tm + 1) / 2 > local) --tm;
        while ((tm + 1) * (tm + 2) / 2 <= local) ++tm;
        tn = local - tm * (tm + 1) / 2;
    }
    const int m0 = tm * BM;
    const int n0 = tn * BN;
    const int M = d.M, N = d.N, K = d.K;
    const int64_t lda = d.lda, ldx = d.ldx;
    const int transA = d.transA, transX = d.transX;
    const GLB TA* __restrict__ A = (const GLB TA*)d.A;
    const GLB TX* __restrict__ X = (const GLB TX*)d.X;
    const GLB int* __restrict__ gather = to_glb(d.gather);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * WTM;
    const int wn = (wave & 1) * WTN;
    const int l16 = lane & 15;
    const int lq = lane >> 4;

    const bool wave_in = m0 + wm < d.M && n0 + wn < d.N;  // uniform per wave
    Acc4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c) acc[a][c] = Acc4{0, 0, 0, 0};

    // Operand tiles are loaded into registers one K step ahead (the loads of
    // step k + 1 are in flight while step k multiplies out of LDS).  Loads use
    // a clamped in-bounds address and keep their raw element type; bounds and
    // conversion are applied when the registers are written to LDS, so no
    // instruction consumes a loaded value before the multiply is issued.
    constexpr int NLA = BM * BK / 256, NLX = BK * BN / 256;
    TA ra[NLA];
    TX rx[NLX];
    uint32_t oka = 0, okx = 0;
    // Branch-free address arithmetic (transposition flags select, out-of-range
    // elements read index 0 and are masked later): every load of a step is
    // issued back to back.
    auto load_tiles = [&](int k0) {
        oka = 0;
        okx = 0;
#pragma unroll
        for (int u = 0; u < NLA; ++u) {
            const int e = tid + 256 * u;
            const int i = transA ? e % BM : e / BK, kk = transA ? e / BM : e % BK;
            const int gi = m0 + i, gk = k0 + kk;
            const bool ok = gi < M && gk < K;
            const int64_t off = transA ? (int64_t)gk * lda + gi : (int64_t)gi * lda + gk;
            ra[u] = A[ok ? off : 0];
            oka |= (uint32_t)ok << u;
        }
        int rowv[NLX];
#pragma unroll
        for (int u = 0; u < NLX; ++u) {
            const int e = tid + 256 * u;
            const int j = transX ? e / BK : e % BN;
            const int gj = n0 + j;
            rowv[u] = gj;
            if constexpr (GATHER) rowv[u] = gather[gj < N ? gj : 0];
        }
#pragma unroll
        for (int u = 0; u < NLX; ++u) {
            const int e = tid + 256 * u;
            const int j = transX ? e / BK : e % BN, kk = transX ? e % BK : e / BN;
            const int gj = n0 + j, gk = k0 + kk;
            const bool ok = gj < N && gk < K;
            const int64_t off = transX ? (int64_t)rowv[u] * ldx + gk : (int64_t)gk * ldx + gj;
            rx[u] = X[ok ? off : 0];
            okx |= (uint32_t)ok << u;
        }
    };
    load_tiles(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        // ---- registers -> LDS, k-contiguous: As[i][kk], Xs[j][kk]
#pragma unroll
        for (int u = 0; u < NLA; ++u) {
            const int e = tid + 256 * u;
            const int i = transA ? e % BM : e / BK, kk = transA ? e / BM : e % BK;
            As[i * LDK + kk] = ((oka >> u) & 1u) ? OpConv<OpT>::cvt(ra[u]) : OpConv<OpT>::cvt((TA)0);
        }
#pragma unroll
        for (int u = 0; u < NLX; ++u) {
            const int e = tid + 256 * u;
            const int j = transX ? e / BK : e % BN, kk = transX ? e % BK : e / BN;
            Xs[j * LDK + kk] = ((okx >> u) & 1u) ? OpConv<OpT>::cvt(rx[u]) : OpConv<OpT>::cvt((TX)0);
        }
        __syncthreads();
        if (k0 + BK < K) load_tiles(k0 + BK);

        // a wave whose sub-tile lies wholly outside C (the last tile row or
        // column of a size that is not a tile multiple) leaves its MFMAs out
        if (!wave_in) {
        } else if constexpr (GK == GK_F64) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                double av[FM], bv[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a) av[a] = As[(wm + a * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int c = 0; c < FN; ++c) bv[c] = Xs[(wn + c * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int c = 0; c < FN; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
            }
        } else if constexpr (GK == GK_F32) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                float av[FM], bv[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a) av[a] = As[(wm + a * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int c = 0; c < FN; ++c) bv[c] = Xs[(wn + c * 16 + l16) * LDK + kk + lq];
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int c = 0; c < FN; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[c], acc[a][c], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 32) {
                bf16x8 av[FM], bv[FN];
#pragma unroll
                for (int a = 0; a < FM; ++a)
                    av[a] = *reinterpret_cast<const bf16x8*>(&As[(wm + a * 16 + l16) * LDK + kk + 8 * lq]);
#pragma unroll
                for (int c = 0; c < FN; ++c)
                    bv[c] = *reinterpret_cast<const bf16x8*>(&Xs[(wn + c * 16 + l16) * LDK + kk + 8 * lq]);
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int c = 0; c < FN; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // ---- epilogue
    GLB TC* __restrict__ C = (GLB TC*)d.C;
    const int64_t ldc = d.ldc;
    const int transC = d.transC, accumulate = d.accumulate;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c)
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
static hipError_t launch_t(GemmTile tile, bool gather, const GemmDesc* descs, const int* tile_begin, int nprob,
                           int total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    if (gather) {
        // the gathered product (U = Q Utilde[:, perm]) is small and FP64: one tile shape
        if constexpr (GK == GK_F64 && std::is_same<TA, double>::value && std::is_same<TX, double>::value) {
            hipLaunchKernelGGL((gemm_kernel<GK, TA, TX, TC, 64, 64, true>), dim3(total), dim3(256), 0, s, descs,
                               tile_begin, nprob);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    switch (tile) {
    case GT_64x64:
        hipLaunchKernelGGL((gemm_kernel<GK, TA, TX, TC, 64, 64, false>), dim3(total), dim3(256), 0, s, descs, tile_begin, nprob);
        break;
    case GT_128x64:
        hipLaunchKernelGGL((gemm_kernel<GK, TA, TX, TC, 128, 64, false>), dim3(total), dim3(256), 0, s, descs, tile_begin, nprob);
        break;
    case GT_64x128:
        hipLaunchKernelGGL((gemm_kernel<GK, TA, TX, TC, 64, 128, false>), dim3(total), dim3(256), 0, s, descs, tile_begin, nprob);
        break;
    case GT_128x128:
        hipLaunchKernelGGL((gemm_kernel<GK, TA, TX, TC, 128, 128, false>), dim3(total), dim3(256), 0, s, descs, tile_begin, nprob);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int GK, typename TA, typename TX>
static hipError_t launch_c(Elem ec, GemmTile tl, bool g, const GemmDesc* d, const int* tb, int np, int tot, hipStream_t s)
{
    switch (ec) {
    case E_F64: return launch_t<GK, TA, TX, double>(tl, g, d, tb, np, tot, s);
    case E_F32: return launch_t<GK, TA, TX, float>(tl, g, d, tb, np, tot, s);
    default: return hipErrorInvalidValue;
    }
}

template <int GK, typename TA>
static hipError_t launch_x(Elem ex, Elem ec, GemmTile tl, bool g, const GemmDesc* d, const int* tb, int np, int tot,
                           hipStream_t s)
{
    switch (ex) {
    case E_F64: return launch_c<GK, TA, double>(ec, tl, g, d, tb, np, tot, s);
    case E_F32: return launch_c<GK, TA, float>(ec, tl, g, d, tb, np, tot, s);
    case E_BF16: return launch_c<GK, TA, __bf16>(ec, tl, g, d, tb, np, tot, s);
    }
    return hipErrorInvalidValue;
}

template <int GK>
static hipError_t launch_a(Elem ea, Elem ex, Elem ec, GemmTile tl, bool g, const GemmDesc* d, const int* tb, int np,
                           int tot, hipStream_t s)
{
    switch (ea) {
    case E_F64: return launch_x<GK, double>(ex, ec, tl, g, d, tb, np, tot, s);
    case E_F32: return launch_x<GK, float>(ex, ec, tl, g, d, tb, np, tot, s);
    case E_BF16: return launch_x<GK, __bf16>(ex, ec, tl, g, d, tb, np, tot, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gemm(GemmKind kind, Elem ea, Elem ex, Elem ec, GemmTile tile, bool gather, const GemmDesc* descs,
                       const int* tile_begin, int nprob, int total_tiles, hipStream_t stream)
{
    if (gather && !(kind == GK_F64 && ea == E_F64 && ex == E_F64)) return hipErrorInvalidValue;
    if (gather) tile = GT_64x64;
    switch (kind) {
    case GK_F64: return launch_a<GK_F64>(ea, ex, ec, tile, gather, descs, tile_begin, nprob, total_tiles, stream);
    case GK_F32: return launch_a<GK_F32>(ea, ex, ec, tile, false, descs, tile_begin, nprob, total_tiles, stream);
    case GK_BF16: return launch_a<GK_BF16>(ea, ex, ec, tile, false, descs, tile_begin, nprob, total_tiles, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace rsvd
