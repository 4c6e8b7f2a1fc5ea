// Orthonormalisation of the sample matrices (paper Sec. II.B, Alg. RSVD step 3,
// and the re-orthonormalisation after every product of the power iteration).
//
// Cholesky QR: with the Gram matrix G = M^T M computed in FP64 by the batched
// GEMM, factor G = L L^T and form Q = M L^-T by block forward substitution.
// Two passes (CholQR2) give an orthonormal Q to working precision when M is
// not too ill conditioned.  A pivot that falls below a relative threshold
// flags the problem, and the Householder kernel recomputes that problem's Q
// from the original M.
#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <type_traits>

namespace rsvd {

// A pivot d_j of the Cholesky factorisation equals ||m_j||^2 sin^2 of the angle
// between column j and the previous columns; below this fraction of ||m_j||^2
// the factor no longer yields an orthonormal Q and Householder takes over.
constexpr double CHOL_PIVOT_REL = 1e-13;

template <typename T> __device__ __forceinline__ double ld_any(const void* p, int64_t i)
{
    return to_f64(((const GLB T*)p)[i]);
}
__device__ __forceinline__ double ld_elem(const void* p, int elem, int64_t i)
{
    if (elem == E_F64) return ld_any<double>(p, i);
    if (elem == E_F32) return ld_any<float>(p, i);
    return ld_any<__bf16>(p, i);
}

// Inverses of the 16 x 16 diagonal blocks of L (stored column-major: Rt[c * l
// + r] = L[r][c]), D_I = L_II^-1 zero padded, for the substitution kernels.
// The blocks are staged in LDS (lds: ceil(l/16) * 272 doubles) with their
// reciprocal diagonals; each thread forms one column of one inverse by forward
// substitution (branch free: the column is zero above its diagonal, so the
// sums run over t < r).  Called by all NT threads of the block.
template <int NT>
__device__ void diag_block_inverses(const GLB double* __restrict__ Rt, int l, GLB double* __restrict__ Dg,
                                    double* lds)
{
    const int tid = threadIdx.x;
    const int nbk = (l + 15) / 16;
    double* Pn = lds;
    double* idg = lds + nbk * 256;
    __syncthreads();
    for (int e = tid; e < nbk * 256; e += NT) {
        const int I = e / 256, i = (e / 16) % 16, j = e % 16;
        const int gi = I * 16 + i, gj = I * 16 + j;
        Pn[e] = (gi < l && gj < l && j <= i) ? Rt[(int64_t)gj * l + gi] : 0.0;
    }
    for (int e = tid; e < nbk * 16; e += NT) idg[e] = (e < l) ? 1.0 / Rt[(int64_t)e * l + e] : 0.0;
    __syncthreads();
    for (int e = tid; e < nbk * 16; e += NT) {
        const int I = e / 16, c = e % 16;
        const double* Lb = Pn + I * 256;
        const double* ib = idg + I * 16;
        double col[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double s0 = 0.0;
#pragma unroll
            for (int t2 = 0; t2 < r; ++t2) s0 = fma(Lb[r * 16 + t2], col[t2], s0);
            const double v = (r == c) ? ib[r] : -s0 * ib[r];
            col[r] = (r < c) ? 0.0 : v;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Dg[(int64_t)I * 256 + r * 16 + c] = col[r];
    }
}

// ---------------------------------------------------------------- right-looking Cholesky
__device__ __forceinline__ double readlane_f64(double v, int src)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 1 / sqrt(x) to working precision: hardware estimate and two Newton steps
// (each written as three dependent operations).
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = x * y;
        const double e = fma(-h, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// One workgroup per problem: G (l x l, FP64, lower triangle used) = L L^T,
// right-looking by 16-column panels with a lookahead of one panel.  Wave 0
// factors the 16 x 16 diagonal blocks in registers (lane r holds row r; the
// column entries travel by readlane, so the 16 sequential column steps need
// no barrier or LDS round trip) and inverts them by forward substitution on
// all 16 right-hand sides at once.  Per panel J: (1) the panel below the
// diagonal block, L_iJ = G_iJ L_JJ^-T, is formed by FP64 MFMA tiles into d.L
// and into an LDS copy; (2) wave 0 applies the update of this panel to the
// next diagonal block first and factors it, while the other waves update the
// remaining lower tiles G_IK -= L_IJ L_KJ^T of the trailing matrix (operands
// from the LDS copy of the panel; each wave loads the G tiles of a group
// before multiplying them, so that memory latency is paid once per group).
// Two barriers per panel.  A pivot that falls below CHOL_PIVOT_REL times the
// original diagonal entry sets the breakdown flag.  Writes L column-major
// into d.L and the diagonal-block inverses into d.D.
constexpr int CHOL_GRP = 4;  // trailing tiles per wave and load group

// Wave 0: factor the diagonal block held in Dt (w x w, identity padded),
// invert it, publish L_JJ (Lb), L_JJ^-1 (Li) and the breakdown flag, write
// the inverse to Dg.
__device__ __forceinline__ void chol_factor_diag(double (*Dt)[17], double (*Lb)[17], double (*Li)[17],
                                                 const double* g0, int J, int w, int* bad_s,
                                                 GLB double* __restrict__ Dg)
{
    const int lane = threadIdx.x & 63, r = lane & 15, lq = lane >> 4;
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = (r < w && c < w && c <= r) ? Dt[r][c] : (r == c ? 1.0 : 0.0);
    bool bad = false;
    double dinv = 1.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const double pc = readlane_f64(a[c], c);
        const double gref = (c < w) ? g0[J + c] : 1.0;
        bad = bad || !(pc > CHOL_PIVOT_REL * gref) || !(pc < INFINITY);
        const double inv = rsqrt_f64(pc);
        const double lrc = (r == c) ? pc * inv : a[c] * inv;
        a[c] = lrc;
        if (r == c) dinv = inv;
#pragma unroll
        for (int k = c + 1; k < 16; ++k) {
            const double lkc = readlane_f64(lrc, k);
            if (r >= k) a[k] = fma(-lrc, lkc, a[k]);
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Lb[r][c] = (c <= r) ? a[c] : 0.0;
    }
    if (lane == 0) *bad_s = bad ? 1 : 0;
    // lane (r, q) holds row r of columns 4 q .. 4 q + 3 of the inverse; step t
    // takes x_t = s_t / L_tt from lane (t, q) and updates the rows below it
    double sv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) sv[j] = (r == 4 * lq + j) ? 1.0 : 0.0;
#pragma unroll
    for (int t2 = 0; t2 < 16; ++t2) {
        const double it = readlane_f64(dinv, t2);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double xt = __shfl(sv[j], t2 + 16 * lq, 64) * it;
            if (r > t2) sv[j] = fma(-a[t2], xt, sv[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = 4 * lq + j;
        const double x = (c <= r) ? sv[j] * dinv : 0.0;
        Li[r][c] = x;
        Dg[(int64_t)(J / 16) * 256 + r * 16 + c] = (r < w && c < w) ? x : 0.0;
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void chol_rl_kernel(const QrDesc* __restrict__ descs, int min_l)
{
    constexpr int NW = NT / 64;
    static_assert(NW >= 2, "wave 0 factors while the others update");
    extern __shared__ double dyn[];  // g0 (l), then the panel copy Lp (16 ceil((l - J - 16) / 16) < l rows x 17)
    __shared__ double Lb[16][17];
    __shared__ double Li[16][17];
    __shared__ double Dt[16][17];
    __shared__ int bad_s;
    const QrDesc& d = descs[blockIdx.x];
    if (d.Qout == nullptr || d.l < min_l || *to_glb(d.flag)) return;
    const int l = d.l;
    double* g0 = dyn;
    double(*Lp)[17] = reinterpret_cast<double(*)[17]>(dyn + ((l + 1) & ~1));
    GLB double* __restrict__ G = to_glb(d.G);
    GLB double* __restrict__ Rt = to_glb(d.L);  // Rt[c * l + r] = L[r][c]
    GLB double* __restrict__ Dg = to_glb(d.D);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    for (int i = tid; i < l; i += NT) g0[i] = G[(int64_t)i * l + i];
    if (tid < 256) {
        const int r = tid >> 4, c = tid & 15;
        Dt[r][c] = ld_or0(G, (int64_t)r * l + c, r < l && c < l);
    }
    __syncthreads();
    if (wave == 0) chol_factor_diag(Dt, Lb, Li, g0, 0, min(16, l), &bad_s, Dg);
    __syncthreads();

    for (int J = 0; J < l; J += 16) {
        const int w = min(16, l - J);
        if (bad_s) {
            if (tid == 0) *to_glb(d.flag) = 1;
            return;
        }
        for (int e = tid; e < 256; e += NT) {
            const int r = e >> 4, c = e & 15;
            if (r < w && c < w) Rt[(int64_t)(J + c) * l + J + r] = (c <= r) ? Lb[r][c] : 0.0;
        }
        // (1) panel below the diagonal block: L_iJ = G_iJ L_JJ^-T (row i - J - 16 of Lp)
        const int nrt = (l - J - 16 + 15) / 16;
        for (int t = wave; t < nrt; t += NW) {
            const int I0 = J + 16 + 16 * t;
            double av[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int k = 4 * s4 + lq;
                av[s4] = ld_or0(G, (int64_t)(I0 + l16) * l + J + k, I0 + l16 < l && k < w);
            }
            dbl4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], Li[l16][4 * s4 + lq], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I0 + lq + 4 * r;
                const double v = (i < l && l16 < w) ? acc[r] : 0.0;
                Lp[16 * t + lq + 4 * r][l16] = v;
                if (i < l && l16 < w) Rt[(int64_t)(J + l16) * l + i] = v;
            }
        }
        __syncthreads();
        if (nrt == 0) break;
        const int ntile = nrt * (nrt + 1) / 2;
        if (wave == 0) {
            // (2a) lookahead: the next diagonal block (tile 0) first, then its factorisation
            const int I0 = J + 16;
            dbl4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I0 + lq + 4 * r, j = I0 + l16;
                acc[r] = ld_or0(G, (int64_t)i * l + j, i < l && j < l);
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int k = 4 * s4 + lq;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Lp[l16][k], Lp[l16][k], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Dt[lq + 4 * r][l16] = acc[r];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            chol_factor_diag(Dt, Lb, Li, g0, I0, min(16, l - I0), &bad_s, Dg);
        } else {
            // (2b) the other lower tiles of the trailing matrix: G_IK -= L_IJ L_KJ^T
            for (int t0 = 1 + (wave - 1) * CHOL_GRP; t0 < ntile; t0 += (NW - 1) * CHOL_GRP) {
                int ti[CHOL_GRP], tk[CHOL_GRP];
                dbl4 acc[CHOL_GRP];
#pragma unroll
                for (int g = 0; g < CHOL_GRP; ++g) {
                    const int t = t0 + g;
                    int a = 0, rem = (t < ntile) ? t : 0;
                    while (rem > a) {
                        rem -= a + 1;
                        ++a;
                    }
                    ti[g] = (t < ntile) ? a : -1;
                    tk[g] = rem;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = J + 16 + 16 * a + lq + 4 * r, j = J + 16 + 16 * rem + l16;
                        acc[g][r] = ld_or0(G, (int64_t)i * l + j, t < ntile && i < l && j < l);
                    }
                }
#pragma unroll
                for (int g = 0; g < CHOL_GRP; ++g) {
                    if (ti[g] < 0) continue;
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int k = 4 * s4 + lq;
                        acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(-Lp[16 * ti[g] + l16][k],
                                                                      Lp[16 * tk[g] + l16][k], acc[g], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int g = 0; g < CHOL_GRP; ++g) {
                    if (ti[g] < 0) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = J + 16 + 16 * ti[g] + lq + 4 * r, j = J + 16 + 16 * tk[g] + l16;
                        if (i < l && j < l) G[(int64_t)i * l + j] = acc[g][r];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- register-resident Cholesky
// For l <= 288 the lower triangle of G fits in the registers of one workgroup
// of 12 waves as 16 x 16 MFMA accumulator tiles: waves 1..11 hold the tiles
// (diagonal ones included; column-major order, round robin, so that every
// panel's remaining tiles are spread evenly), so the trailing updates never go
// back to memory, and wave 0 runs the dependent chain of the method.  Each
// tile is held transposed, T_IK = G_IK^T, which makes it the B operand of the
// panel product and the output of the update:
//   panel     L_IJ^T = L_JJ^-1 T_IJ          (then copied to LDS and to d.L)
//   update    T_IK  -= L_KJ L_IJ^T            (operands from the LDS panel copy)
// Right-looking by 16-column panels.  The chain of panel J (sub-diagonal tile
// J + 1, then diagonal block J + 1 updated and factored) is wave 0's: the
// owners of those two tiles copy them to LDS after their last update in the
// previous panel, and wave 0 forms the sub-diagonal block of L, updates and
// factors diagonal block J + 1 while the other waves form the rest of panel
// J and update their tiles.  Two barriers per panel, ordering LDS only:
// nothing the kernel writes to global memory is read back in it.  Same
// outputs as the kernel above (L column-major in d.L, the diagonal-block
// inverses in d.D, the breakdown flag); G is only read.
constexpr int CHR_T = 18;                                                 // tile rows: l <= 288
constexpr int CHR_NT = 768;                                               // 12 waves
constexpr int CHR_OW = CHR_NT / 64 - 1;                                   // waves holding tiles
constexpr int CHR_NPW = (CHR_T * (CHR_T + 1) / 2 + CHR_OW - 1) / CHR_OW;  // tiles per such wave

struct ChrLds {
    double Lp[CHR_T * 16][17];  // column panel J of L, by absolute row (staging tiles at the start)
    double Lb[16][17], Li[16][17], Dt[16][17];
    double Ts[16][17], Td[16][17];  // the next sub-diagonal and diagonal tiles (transposed)
    double g0[CHR_T * 16];          // diagonal of G (pivot reference)
    int bad;
};

// Workgroup barrier ordering LDS only (the global stores stay in flight).
__device__ __forceinline__ void chr_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Lane T of every row of 16 lanes, broadcast to its row (one 64-bit DPP
// row_newbcast move).
template <int T> __device__ __forceinline__ double row_bcast16(double v)
{
    const long long u = __builtin_bit_cast(long long, v);
    return __builtin_bit_cast(double, (long long)__builtin_amdgcn_mov_dpp(u, 0x150 + T, 0xF, 0xF, false));
}

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// The diagonal block factorisation of the register-resident kernel: the same
// arithmetic as chol_factor_diag (so the same L and inverse to the bit), laid
// out for latency, since every dependent FP64 operation costs tens of cycles.
// Lane (r, q) holds row r of the block and the column values travel by row
// broadcasts; every lane updates its whole row (the entries above the
// diagonal become garbage that is never read: the lower triangle depends on
// lower entries only); the pivot test is off the dependent chain; and each
// column's inverse pivot is kept apart, so that the substitution for the
// inverse (its step t needs column t of L only) can run beside the later
// columns of the factorisation.
__device__ __forceinline__ void chr_factor_diag(double (*Dt)[17], double (*Lb)[17], double (*Li)[17],
                                                const double* g0, int J0, int w, int* bad_s,
                                                GLB double* __restrict__ Dg)
{
    const int lane = threadIdx.x & 63, r = lane & 15, lq = lane >> 4;
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const double v = Dt[r][c];
        a[c] = (r < w && c < w) ? v : (r == c ? 1.0 : 0.0);
    }
    const double gv = g0[J0 + (r < w ? r : 0)];
    const double gref = (r < w) ? gv : 1.0;
    double piv = 1.0;
    // lane (r, q) holds row r of columns 4 q .. 4 q + 3 of the inverse; step t
    // takes x_t = s_t / L_tt from row t of its column group
    double sv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) sv[j] = (r == 4 * lq + j) ? 1.0 : 0.0;
    double dinv = 1.0, inv_prev = 1.0;
    // (rows r <= t keep their value: they add -0 x_t, which changes no value)
    auto inverse_step = [&](auto T_, double it) {
        constexpr int T = decltype(T_)::value;
        const double na = (r > T) ? -a[T] : -0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double xt = row_bcast16<T>(sv[j]) * it;
            sv[j] = fma(na, xt, sv[j]);
        }
    };
    // column C of the factorisation beside step C - 1 of the substitution
    static_for<0, 16>([&](auto C_) {
        constexpr int C = decltype(C_)::value;
        const double pc = row_bcast16<C>(a[C]);
        const double inv = rsqrt_f64(pc);
        const double lrc = a[C] * inv;
        a[C] = lrc;
        static_for<C + 1, 16>([&](auto K_) {
            constexpr int K = decltype(K_)::value;
            a[K] = fma(-lrc, row_bcast16<K>(lrc), a[K]);
        });
        piv = (r == C) ? pc : piv;
        dinv = (r == C) ? inv : dinv;
        if constexpr (C > 0) inverse_step(std::integral_constant<int, C - 1>{}, inv_prev);
        inv_prev = inv;
        __builtin_amdgcn_sched_barrier(0);
    });
    inverse_step(std::integral_constant<int, 15>{}, inv_prev);
    const bool bad = __any(!(piv > CHOL_PIVOT_REL * gref) || !(piv < INFINITY));
    if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Lb[r][c] = (c <= r) ? a[c] : 0.0;
    }
    if (lane == 0) *bad_s = bad ? 1 : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = 4 * lq + j;
        const double x = (c <= r) ? sv[j] * dinv : 0.0;
        Li[r][c] = x;
        Dg[(int64_t)(J0 / 16) * 256 + r * 16 + c] = (r < w && c < w) ? x : 0.0;
    }
}

// A tile coordinate the compiler must re-read in every pass: without it the
// per-tile addresses (loop invariant) are hoisted out of the panel loop and
// spilled.
__device__ __forceinline__ int chr_opaque(int t)
{
    asm volatile("" : "+s"(t));
    return t;
}

// Tile (I, K) of G into an LDS block: dst[l16][lq + 4 r] = G[16 I + l16][16 K + lq + 4 r]
// (trans = false: the tile as it is) or dst[lq + 4 r][l16] = the same value
// (trans = true: the transposed tile T_IK in accumulator layout).
__device__ __forceinline__ void chr_load_tile(double (*dst)[17], const GLB double* __restrict__ G, int l, int I, int K,
                                              int l16, int lq, bool trans)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + l16, j = 16 * K + lq + 4 * r;
        const double v = ld_or0(G, (int64_t)i * l + j, i < l && j < l);
        if (trans)
            dst[lq + 4 * r][l16] = v;
        else
            dst[l16][lq + 4 * r] = v;
    }
}

// wave 0: per panel J, the sub-diagonal block of L, diagonal block J + 1
// updated and factored; the diagonal blocks of L are written out during the
// next panel pass
__device__ __forceinline__ void chr_chain_path(ChrLds& s, const GLB double* __restrict__ G,
                                               GLB double* __restrict__ Rt, GLB double* __restrict__ Dg,
                                               GLB int* __restrict__ flag, int l, int T)
{
    const int lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
    __builtin_amdgcn_s_setprio(3);  // the dependent chain first on this SIMD
    // the pivot references, diagonal block 0 and the first sub-diagonal and
    // diagonal tiles, loaded here so that block 0 is factored while the other
    // waves load their tiles
    for (int i = lane; i < l; i += 64) s.g0[i] = G[(int64_t)i * l + i];
    chr_load_tile(s.Dt, G, l, 0, 0, l16, lq, false);
    if (T > 1) {
        chr_load_tile(s.Ts, G, l, 1, 0, l16, lq, true);
        chr_load_tile(s.Td, G, l, 1, 1, l16, lq, true);
    }
    wave_lds_fence();
    chr_factor_diag(s.Dt, s.Lb, s.Li, s.g0, 0, min(16, l), &s.bad, Dg);
    chr_barrier();  // tiles loaded, block 0 factored
    for (int J = 0; J < T; ++J) {
        if (s.bad) {
            if (lane == 0) *flag = 1;
            return;
        }
        const int K1 = J + 1;
        if (K1 < T) {
            // L_{J+1,J}^T = L_JJ^-1 T_{J+1,J}; o[r] = L[16 K1 + l16][16 J + lq + 4 r]
            dbl4 o = {0, 0, 0, 0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                o = __builtin_amdgcn_mfma_f64_16x16x4f64(s.Li[l16][4 * s4 + lq], s.Ts[4 * s4 + lq][l16], o, 0, 0, 0);
            const int i = 16 * K1 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = lq + 4 * r;
                const bool ok = i < l && 16 * J + c < l;
                s.Lp[i][c] = ok ? o[r] : 0.0;
                if (ok) Rt[(int64_t)(16 * J + c) * l + i] = o[r];
            }
            wave_lds_fence();
            // diagonal block J + 1 -= L_{J+1,J} L_{J+1,J}^T
            dbl4 t;
#pragma unroll
            for (int r = 0; r < 4; ++r) t[r] = s.Td[lq + 4 * r][l16];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double v = s.Lp[i][4 * s4 + lq];
                t = __builtin_amdgcn_mfma_f64_16x16x4f64(-v, v, t, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) s.Dt[l16][lq + 4 * r] = t[r];
        }
        chr_barrier();  // panel J in Lp (diagonal block J of L written out by a tile wave)
        if (K1 == T) break;
        chr_factor_diag(s.Dt, s.Lb, s.Li, s.g0, 16 * K1, min(16, l - 16 * K1), &s.bad, Dg);
        chr_barrier();  // block J + 1 factored, trailing tiles updated
    }
}

// waves 1..11: the tiles.  Tile t (column-major over the lower triangle,
// column K starting at t = K T - K (K - 1) / 2) is held by tile wave t mod
// CHR_OW in slot t / CHR_OW, so each pass finds its tiles by arithmetic.
__device__ __forceinline__ void chr_tile_path(ChrLds& s, const GLB double* __restrict__ G, GLB double* __restrict__ Rt,
                                              int l, int T, int w)
{
    const int lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
    const int ntile = T * (T + 1) / 2;
    const int nslot = w < ntile ? (ntile - w + CHR_OW - 1) / CHR_OW : 0;
    auto base = [&](int K) { return K * T - K * (K - 1) / 2; };
    auto first_slot = [&](int t) { return t > w ? (t - w + CHR_OW - 1) / CHR_OW : 0; };  // first slot with tile >= t
    int tc[CHR_NPW];  // I + 256 K; invalid tiles get K = CHR_T
    {
        int K = 0, rem = w;  // column K holds T - K tiles
#pragma unroll
        for (int g = 0; g < CHR_NPW; ++g) {
            const bool ok = g < nslot;
            while (ok && rem >= T - K) {
                rem -= T - K;
                ++K;
            }
            tc[g] = ok ? (K + rem) + 256 * K : 256 * CHR_T;
            rem += CHR_OW;
        }
    }
    // coalesced loads (tile row lq + 4 r, column l16), then a transpose through
    // this wave's 16 staging rows of Lp into T_IK[lq + 4 r][l16] = G[16 I + l16][16 K + lq + 4 r]
    dbl4 acc[CHR_NPW];
#pragma unroll
    for (int g = 0; g < CHR_NPW; ++g) {
        const int I = tc[g] & 255, K = tc[g] >> 8;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * I + lq + 4 * r, j = 16 * K + l16;
            acc[g][r] = ld_or0(G, (int64_t)i * l + j, K < T && i < l && j < l);
        }
    }
    // (one wave's LDS operations execute in order, so the staging rows are
    // reused from tile to tile without a wait)
    double(*stg)[17] = &s.Lp[16 * w];
#pragma unroll
    for (int g = 0; g < CHR_NPW; ++g) {
#pragma unroll
        for (int r = 0; r < 4; ++r) stg[lq + 4 * r][l16] = acc[g][r];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[g][r] = stg[l16][lq + 4 * r];
    }
    chr_barrier();  // tiles loaded, block 0 factored (the staging rows are free again)
    // panel product of the tile in slot G: L_IJ^T = L_JJ^-1 T_IJ; o[r] = L[16 I + l16][16 J + lq + 4 r]
    auto panel = [&](auto G_, int J) {
        constexpr int Gs = decltype(G_)::value;
        const int I = chr_opaque(tc[Gs]) & 255;
        dbl4 o = {0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            o = __builtin_amdgcn_mfma_f64_16x16x4f64(s.Li[l16][4 * s4 + lq], acc[Gs][s4], o, 0, 0, 0);
        const int i = 16 * I + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = lq + 4 * r;
            const bool ok = i < l && 16 * J + c < l;
            s.Lp[i][c] = ok ? o[r] : 0.0;
            if (ok) Rt[(int64_t)(16 * J + c) * l + i] = o[r];
        }
    };
    for (int J = 0; J < T; ++J) {
        if (s.bad) return;
        const int K1 = J + 1;
        const int bJ = base(J), bK1 = base(K1);
        const int tdiag = bK1;  // tile (J + 1, J + 1), wave 0's
        const bool more = K1 < T;
        // the sub-diagonal tile first (it feeds diagonal block J + 1)
        if (w == CHR_OW - 1) {  // diagonal block J of L, factored by wave 0
            const int wd = min(16, l - 16 * J);
            for (int e = lane; e < 256; e += 64) {
                const int r = e >> 4, c = e & 15;
                if (r < wd && c < wd) Rt[(int64_t)(16 * J + c) * l + 16 * J + r] = (c <= r) ? s.Lb[r][c] : 0.0;
            }
        }
        const int glo = first_slot(bJ + 2), ghi = first_slot(bK1);  // column J below the sub-diagonal tile
        static_for<0, CHR_NPW>([&](auto G_) {
            if (decltype(G_)::value >= glo && decltype(G_)::value < ghi) panel(G_, J);
            __builtin_amdgcn_sched_barrier(0);
        });
        const int gdiag = (more && tdiag % CHR_OW == w) ? tdiag / CHR_OW : -1;
        chr_barrier();  // panel J in Lp
        if (!more) break;
        // the trailing tiles (columns > J, diagonal block J + 1 is wave 0's):
        // T_IK -= L_KJ L_IJ^T; the next panel's sub-diagonal and diagonal
        // tiles go to LDS for wave 0 after this, their last update
        const int gfirst = first_slot(bK1);
        const int tnsub = bK1 + 1, tndiag = base(K1 + 1);  // tiles (J + 2, J + 1) and (J + 2, J + 2)
        const bool next = K1 + 1 < T;
        const int gnsub = (next && tnsub % CHR_OW == w) ? tnsub / CHR_OW : -1;
        const int gndiag = (next && tndiag % CHR_OW == w) ? tndiag / CHR_OW : -1;
#pragma unroll
        for (int g = 0; g < CHR_NPW; ++g) {
            if (g >= gfirst && g < nslot && g != gdiag) {
                const int t = chr_opaque(tc[g]);
                const int I = t & 255, K = t >> 8;
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    const int k = 4 * s4 + lq;
                    acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(-s.Lp[16 * K + l16][k], s.Lp[16 * I + l16][k],
                                                                  acc[g], 0, 0, 0);
                }
                if (g == gnsub) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) s.Ts[lq + 4 * r][l16] = acc[g][r];
                }
                if (g == gndiag) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) s.Td[lq + 4 * r][l16] = acc[g][r];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        chr_barrier();  // block J + 1 factored, trailing tiles updated
    }
}

__global__ __launch_bounds__(CHR_NT) void chol_reg_kernel(const QrDesc* __restrict__ descs)
{
    __shared__ ChrLds s;
    const QrDesc& d = descs[blockIdx.x];
    if (d.Qout == nullptr || d.l > CHR_T * 16 || *to_glb(d.flag)) return;
    const int l = d.l, T = (l + 15) / 16;
    const GLB double* __restrict__ G = to_glb((const double*)d.G);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave == 0)
        chr_chain_path(s, G, to_glb(d.L), to_glb(d.D), to_glb(d.flag), l, T);
    else
        chr_tile_path(s, G, to_glb(d.L), l, T, wave - 1);
}

// ---------------------------------------------------------------- Q = M L^-T
// One wave per 16 rows of M.  With Q^T = L^-1 M^T, block column C of Q^T is
// D_C (M^T[C] - L[C, :C] Q^T[:C]); both products are FP64 MFMA chains, the
// accumulator of the first feeding the second directly as its B operand.  The
// wave's 16 rows of Q stay in LDS; no other wave reads them.
template <typename TS>
__global__ __launch_bounds__(64) void trsm_kernel(const QrDesc* __restrict__ descs,
                                                  const int* __restrict__ row_begin, int nprob, int from_min,
                                                  int min_l)
{
    extern __shared__ double Qs[];  // 16 x (l + 1)
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(row_begin, t);
    const int b = wi_.x;
    const QrDesc& d = descs[b];
    if (d.Qout == nullptr || d.l < min_l || *to_glb(d.flag)) return;
    const int l = d.l, rows = d.rows;
    const int ldq = l + 1;
    const int r0 = wi_.y * 16;
    const int nr = min(16, rows - r0);
    const GLB double* __restrict__ Rt = to_glb((const double*)d.L);  // Rt[k * l + r] = L[r][k]
    const GLB double* __restrict__ D = to_glb((const double*)d.D);
    GLB double* __restrict__ Qout = to_glb(d.Qout);
    const int lane = threadIdx.x;
    const int l16 = lane & 15, lq = lane >> 4;

    // load the 16 rows (8 loads in flight per lane)
    for (int base = lane; base < 16 * l; base += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + 64 * u;
            const int r = e / l, c = e % l;
            const GLB TS* src = from_min ? (const GLB TS*)d.Min : (const GLB TS*)Qout;
            v[u] = to_f64(ld_or0(src, (int64_t)(r0 + r) * l + c, e < 16 * l && r < nr));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + 64 * u;
            if (e < 16 * l) Qs[(e / l) * ldq + e % l] = v[u];
        }
    }
    __syncthreads();
    for (int C0 = 0; C0 < l; C0 += 16) {
        // acc[r] = (M^T - L Q^T)[C0 + lq + 4r][l16]  (column index, row of M)
        dbl4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = C0 + lq + 4 * r;
            acc[r] = (c < l) ? Qs[l16 * ldq + c] : 0.0;
        }
        const int ra = C0 + l16;  // row of L supplying the A operand
        for (int k0 = 0; k0 < C0; k0 += 32) {
            double av[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kc = k0 + 4 * u + lq;
                const bool ok = kc < C0;
                av[u] = -ld_or0(Rt, (int64_t)kc * l + ra, ok && ra < l);
                bv[u] = ok ? Qs[l16 * ldq + kc] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
        // R = D_C * acc: accumulator register s is the B operand row 4 s + lane/16
        dbl4 res = {0, 0, 0, 0};
        const GLB double* Dc = D + (int64_t)(C0 / 16) * 256;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const double av = Dc[l16 * 16 + 4 * s2 + lq];
            res = __builtin_amdgcn_mfma_f64_16x16x4f64(av, acc[s2], res, 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = C0 + lq + 4 * r;
            if (c < l) Qs[l16 * ldq + c] = res[r];
        }
        __syncthreads();
    }
    for (int e = lane; e < nr * l; e += 64) {
        const int r = e / l, c = e % l;
        Qout[(int64_t)(r0 + r) * l + c] = Qs[r * ldq + c];
    }
}

// The same substitution for l <= 288 with the wave's 16 rows of Q held in
// registers: block C of Q^T leaves the D_C product in accumulator layout,
// res[C][r] = Q[r0 + l16][16 C + lq + 4 r], which is exactly the B operand
// layout in which the later blocks read it, so no LDS round trip (and no
// barrier) separates the blocks, and the loads for a block are issued one
// block ahead.  The products are those of trsm_kernel in the same order, up
// to exact sign changes (the same Q to the bit, up to the sign of zeros).
template <typename TS>
__global__ __launch_bounds__(64) void trsm_reg_kernel(const QrDesc* __restrict__ descs,
                                                      const int* __restrict__ row_begin, int nprob, int from_min)
{
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(row_begin, t);
    const QrDesc& d = descs[wi_.x];
    if (d.Qout == nullptr || d.l > CHR_T * 16 || *to_glb(d.flag)) return;
    const int l = d.l, rows = d.rows, T = (l + 15) / 16;
    const int r0 = wi_.y * 16;
    const GLB double* __restrict__ Rt = to_glb((const double*)d.L);  // Rt[k * l + r] = L[r][k]
    const GLB double* __restrict__ D = to_glb((const double*)d.D);
    GLB double* __restrict__ Qout = to_glb(d.Qout);
    const GLB TS* __restrict__ src = from_min ? (const GLB TS*)d.Min : (const GLB TS*)d.Qout;
    const int lane = threadIdx.x, l16 = lane & 15, lq = lane >> 4;
    const int row = r0 + l16;
    const bool row_ok = row < rows;
    dbl4 res[CHR_T];
    // the operands of block C: the 4 row values of M^T (acc init), the 4 C
    // values of L (A operand of the update) and the diagonal-block inverse;
    // double-buffered, so that block C + 1's loads are in flight while block
    // C's dependent MFMA chain runs.  They are kept as loaded (no select or
    // negation that would wait for them): out-of-range elements read an
    // in-range one, which only reaches padded rows of Q (never stored, and
    // each lane's row is independent) or padded columns (cancelled by the
    // zero-padded D_C), and the chain accumulates -(M^T - L Q^T), negated
    // back after the D_C product (sign changes are exact).
    double lv[2][4 * CHR_T];
    TS mv[2][4];
    double dv[2][4];
    auto issue = [&](auto C_, auto B_) {
        constexpr int C = decltype(C_)::value, Bf = decltype(B_)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * C + lq + 4 * r;
            mv[Bf][r] = src[(row_ok && c < l) ? (int64_t)row * l + c : 0];
        }
        const int ra = 16 * C + l16;  // row of L supplying the A operand
#pragma unroll
        for (int j = 0; j < 4 * C; ++j) lv[Bf][j] = Rt[ra < l ? (int64_t)(4 * j + lq) * l + ra : 0];
        const GLB double* Dc = D + (int64_t)C * 256;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) dv[Bf][s2] = Dc[l16 * 16 + 4 * s2 + lq];
    };
    issue(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    static_for<0, CHR_T>([&](auto C_) {
        constexpr int C = decltype(C_)::value, Bf = C % 2;
        if (C < T) {
            if constexpr (C + 1 < CHR_T) {
                if (C + 1 < T) issue(std::integral_constant<int, C + 1>{}, std::integral_constant<int, 1 - Bf>{});
            }
            __builtin_amdgcn_sched_barrier(0);
            // nacc[r] = -(M^T - L Q^T)[16 C + lq + 4 r][row]
            dbl4 nacc;
#pragma unroll
            for (int r = 0; r < 4; ++r) nacc[r] = -to_f64(mv[Bf][r]);
            static_for<0, C>([&](auto Cp_) {
                constexpr int Cp = decltype(Cp_)::value;
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    nacc = __builtin_amdgcn_mfma_f64_16x16x4f64(lv[Bf][4 * Cp + s4], res[Cp][s4], nacc, 0, 0, 0);
            });
            // res[C] = D_C acc = -(D_C nacc): accumulator register s is the B operand row 4 s + lane / 16
            dbl4 o = {0, 0, 0, 0};
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) o = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[Bf][s2], nacc[s2], o, 0, 0, 0);
            res[C] = -o;
            __builtin_amdgcn_sched_barrier(0);
        }
    });
    static_for<0, CHR_T>([&](auto C_) {
        constexpr int C = decltype(C_)::value;
        if (C < T) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = 16 * C + lq + 4 * r;
                if (row_ok && c < l) Qout[(int64_t)row * l + c] = res[C][r];
            }
        }
    });
}

// ---------------------------------------------------------------- adjoint helpers
// R (l x l, row-major) = Q^T M of a stage, computed by GEMM: zero its strictly
// lower part so that it is exactly the upper-triangular factor, and form the
// diagonal-block inverses of L = R^T for the substitution below.  (Row-major R
// is the column-major storage of L.)
__global__ __launch_bounds__(256) void tri_prep_kernel(const QrDesc* __restrict__ descs)
{
    extern __shared__ double lds[];
    const QrDesc& d = descs[blockIdx.x];
    if (d.Qout == nullptr) return;
    const int l = d.l;
    GLB double* __restrict__ R = to_glb(d.L);
    for (int e = threadIdx.x; e < l * l; e += 256)
        if (e / l > e % l) R[e] = 0.0;
    diag_block_inverses<256>(R, l, to_glb(d.D), lds);
}

// Y = X L^-1 in place on the rows of X = Qout (rows x l), L lower triangular
// stored column-major (Rt[c * l + r] = L[r][c]).  Row by row y L = x, i.e.
// backward substitution: with Y^T = L^-T X^T, block column C of Y^T is
// D_C^T (X^T[C] - L[>C, C]^T Y^T[>C]), C from the last block to the first;
// both products are FP64 MFMA chains as in trsm_kernel.
__global__ __launch_bounds__(64) void trsm_upper_kernel(const QrDesc* __restrict__ descs,
                                                        const int* __restrict__ row_begin, int nprob)
{
    extern __shared__ double Qs[];  // 16 x (l + 1)
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(row_begin, t);
    const int b = wi_.x;
    const QrDesc& d = descs[b];
    if (d.Qout == nullptr) return;
    const int l = d.l, rows = d.rows;
    const int ldq = l + 1;
    const int r0 = wi_.y * 16;
    const int nr = min(16, rows - r0);
    const GLB double* __restrict__ Rt = to_glb((const double*)d.L);
    const GLB double* __restrict__ D = to_glb((const double*)d.D);
    GLB double* __restrict__ Qout = to_glb(d.Qout);
    const int lane = threadIdx.x;
    const int l16 = lane & 15, lq = lane >> 4;

    for (int base = lane; base < 16 * l; base += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + 64 * u;
            const int r = e / l, c = e % l;
            v[u] = ld_or0((const GLB double*)Qout, (int64_t)(r0 + r) * l + c, e < 16 * l && r < nr);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + 64 * u;
            if (e < 16 * l) Qs[(e / l) * ldq + e % l] = v[u];
        }
    }
    __syncthreads();
    const int nbk = (l + 15) / 16;
    for (int cb = nbk - 1; cb >= 0; --cb) {
        const int C0 = cb * 16;
        dbl4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = C0 + lq + 4 * r;
            acc[r] = (c < l) ? Qs[l16 * ldq + c] : 0.0;
        }
        const int ci = C0 + l16;  // column of L supplying the A operand (A[i][k] = L[k][C0 + i])
        for (int k0 = C0 + 16; k0 < l; k0 += 32) {
            double av[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kc = k0 + 4 * u + lq;
                const bool ok = kc < l;
                av[u] = -ld_or0(Rt, (int64_t)ci * l + kc, ok && ci < l);
                bv[u] = ok ? Qs[l16 * ldq + kc] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
        // res = D_C^T acc (A operand element (i, k) = D_C[k][i])
        dbl4 res = {0, 0, 0, 0};
        const GLB double* Dc = D + (int64_t)cb * 256;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const double av = Dc[(4 * s2 + lq) * 16 + l16];
            res = __builtin_amdgcn_mfma_f64_16x16x4f64(av, acc[s2], res, 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = C0 + lq + 4 * r;
            if (c < l) Qs[l16 * ldq + c] = res[r];
        }
        __syncthreads();
    }
    for (int e = lane; e < nr * l; e += 64) {
        const int r = e / l, c = e % l;
        Qout[(int64_t)(r0 + r) * l + c] = Qs[r * ldq + c];
    }
}

hipError_t launch_tri_prep(const QrDesc* d, int nprob, int max_l, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    const size_t lds = (size_t)((max_l + 15) / 16) * 272 * sizeof(double);
    hipLaunchKernelGGL(tri_prep_kernel, dim3(nprob), dim3(256), lds, s, d);
    return hipGetLastError();
}

hipError_t launch_trsm_upper(const QrDesc* d, const int* row_begin, int nprob, int total_blocks, int max_l,
                             hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    const size_t lds = (size_t)16 * (max_l + 1) * sizeof(double);
    hipLaunchKernelGGL(trsm_upper_kernel, dim3(total_blocks), dim3(64), lds, s, d, row_begin, nprob);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Householder
// One workgroup per flagged problem: in-place Householder QR of a copy of M in
// Qout, then the explicit thin Q formed in place from the reflectors, and the
// sign convention diag(R) >= 0.  Always orthonormal, also for rank-deficient M.
//
// M is row-major, so the work of each reflector is laid out along the rows:
// for the trailing columns c > j, w_c = sum_i v_i M_ic and M_ic -= tau v_i w_c
// are computed with lanes on consecutive columns (coalesced row segments; v_i
// is one broadcast load per row) and the waves split the rows into groups
// when the trailing block is narrower than the workgroup, the groups' partial
// sums meeting in LDS.
constexpr int HH_MAXL = 2048;
constexpr int HH_T = 512;
constexpr int HH_W = HH_T / 64;

__device__ __forceinline__ double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < HH_W; ++w) s += red[w];
    return s;
}

// Applies the reflector I - tau v v^T (v = (1, A[j+1:, j])) to the columns
// c0 <= c < l of A (rows j..rows-1).  Called by all threads; part holds
// HH_W x 64 partial sums.
__device__ void hh_apply(GLB double* __restrict__ A, int rows, int l, int j, int c0, double tau, double* part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int cb = c0; cb < l; cb += 64 * HH_W) {
        const int nchunk = min(HH_W, (l - cb + 63) / 64);  // 64-column chunks in this pass
        const int groups = HH_W / nchunk;                  // row groups per chunk
        const int chunk = wave % nchunk, g = wave / nchunk;
        const int c = cb + 64 * chunk + lane;
        const bool act = g < groups && c < l;
        // row j (v_j = 1) belongs to group 0; all reads of the block precede the barrier
        double w = (act && g == 0) ? A[(int64_t)j * l + c] : 0.0;
        if (act) {
            for (int i = j + 1 + g; i < rows; i += groups) w = fma(A[(int64_t)i * l + j], A[(int64_t)i * l + c], w);
        }
        __syncthreads();  // part is free
        part[wave * 64 + lane] = w;
        __syncthreads();
        if (act) {
            // every group forms the same total (same order), so no broadcast is needed
            double tot = 0.0;
            for (int q = 0; q < groups; ++q) tot += part[(q * nchunk + chunk) * 64 + lane];
            tot *= tau;
            if (g == 0) A[(int64_t)j * l + c] -= tot;
            for (int i = j + 1 + g; i < rows; i += groups) A[(int64_t)i * l + c] -= tot * A[(int64_t)i * l + j];
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(HH_T) void householder_kernel(const QrDesc* __restrict__ descs)
{
    __shared__ double tau_s[HH_MAXL];
    __shared__ double beta_s[HH_MAXL];
    __shared__ double red[HH_W];
    __shared__ double part[HH_W * 64];
    const QrDesc& d = descs[blockIdx.x];
    if (d.Qout == nullptr || !*to_glb(d.flag)) return;
    const int rows = d.rows, l = d.l;
    GLB double* __restrict__ A = to_glb(d.Qout);
    const int tid = threadIdx.x;

    for (int64_t e = tid; e < (int64_t)rows * l; e += HH_T) A[e] = ld_elem(d.Min, d.min_elem, e);
    __syncthreads();

    for (int j = 0; j < l; ++j) {
        double p = 0.0;
        for (int i = j + 1 + tid; i < rows; i += HH_T) {
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
            for (int i = j + 1 + tid; i < rows; i += HH_T) A[(int64_t)i * l + j] *= scal;
        }
        __syncthreads();
        if (tid == 0) {
            A[(int64_t)j * l + j] = beta;
            tau_s[j] = tau;
            beta_s[j] = beta;
        }
        __syncthreads();
        if (tau != 0.0) hh_apply(A, rows, l, j, j + 1, tau, part);
    }
    // form Q in place from the reflectors, last one first
    for (int j = l - 1; j >= 0; --j) {
        const double tau = tau_s[j];
        if (tau != 0.0) hh_apply(A, rows, l, j, j + 1, tau, part);
        for (int i = j + 1 + tid; i < rows; i += HH_T) A[(int64_t)i * l + j] *= -tau;
        if (tid == 0) A[(int64_t)j * l + j] = 1.0 - tau;
        for (int i = tid; i < j; i += HH_T) A[(int64_t)i * l + j] = 0.0;
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)rows * l; e += HH_T) {
        const int c = (int)(e % l);
        if (beta_s[c] < 0.0) A[e] = -A[e];
    }
}

// ---------------------------------------------------------------- blocked Householder
// The same factorisation as householder_kernel, by panels of HB = 16 columns
// (compact WY form, Schreiber and Van Loan): the product of a panel's
// reflectors is H = H_1 ... H_bw = I - V T V^T, with V (rows x bw, unit lower
// trapezoidal, stored below the diagonal of the panel) and T (bw x bw upper
// triangular).  A panel is factored in registers by one workgroup; the rest of
// the matrix is updated by H^T (factorisation) or H (forming Q, last panel
// first) as two FP64 MFMA products per 64-column tile, W = V^T C and
// C -= V (X W) with X = T^T or T, one workgroup per tile, so the update of one
// problem spreads over many CUs and reads its columns once per panel instead of
// once per column.
//
// One launch per panel and phase (hb_kernel, blockIdx.x = tile, blockIdx.y =
// problem):
//   factor, launch J:  tiles over columns [16 J, l): J = 0 copies M in, J > 0
//                      applies panel J-1; then tile 0 factors panel J.
//   form Q, launch J (J = P-2 .. -1): tiles over columns [16 (J+1), l):
//                      tile 0 turns panel J+1 into its Q columns (E - V T V_top^T,
//                      zero above), then every tile applies panel J (J >= 0), or
//                      at J = -1 the sign convention diag(R) >= 0.
// T of panel J is kept in G (offset 256 J, row-major with stride bw), tau and
// beta in D (D[c], D[l + c]).
constexpr int HB = 16;
constexpr int HB_TW = 64;
constexpr int HB_T = 512;
constexpr int HB_G = HB_T / HB;  // row groups of the panel layout
enum { HB_FACTOR = 0, HB_QFORM = 1 };

struct HbLds {
    double wpart[4 * 64 * 4];  // W partial sums of the second row half
    double W[HB * HB_TW];      // W = V^T C, then Y = X W
    double red[HB_T / 64][HB]; // panel reductions, one row per wave
    double T[HB * HB];
    double tau[HB], beta[HB];
    double Wc[HB * HB];        // T V_top^T for the Q columns of a panel
    double scal[2];
};

// V[r][k] of the panel at column pc with bw columns (r >= pc): 1 on the
// diagonal, the stored reflector entries below, 0 above and for k >= bw.
__device__ __forceinline__ double hb_v(const GLB double* A, int64_t l, int rows, int pc, int bw, int r, int k)
{
    const int d = r - pc;
    const bool below = d > k && k < bw && r < rows;
    const double x = A[below ? (int64_t)r * l + pc + k : 0];
    return below ? x : ((d == k && k < bw) ? 1.0 : 0.0);
}

// Applies I - V X V^T to the columns [c0, c1) of rows [pc, rows), with X = T^T
// (trans) or T: W = V^T C, Y = X W, C -= V Y.  All 512 threads; the tile is at
// most 64 columns wide and lies right of the panel.
__device__ void hb_update(GLB double* __restrict__ A, int64_t l, int rows, int pc, int bw,
                          const GLB double* __restrict__ Tg, bool trans, int c0, int c1, HbLds& s)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int cb = wave & 3, h = wave >> 2;
    const int c = c0 + 16 * cb + l16;
    const bool cok = c < c1;
    // ---- W = V^T C: D[k][col] = sum_r V[r][k] C[r][col], K = rows, 4 rows per MFMA
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int rb = pc + 4 * h; rb < rows; rb += 8) {
        const int r = rb + lq;
        const double av = hb_v(A, l, rows, pc, bw, r, l16);
        const double bv = ld_or0<double>(A, (int64_t)r * l + c, r < rows && cok);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    if (h == 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s.wpart[(cb * 64 + lane) * 4 + q] = acc[q];
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s.W[(lq + 4 * q) * HB_TW + 16 * cb + l16] = acc[q] + s.wpart[(cb * 64 + lane) * 4 + q];
    }
    __syncthreads();
    // ---- Y = X W (16 x 64), two rows per thread, written over W after a barrier
    double y[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int k = 2 * wave + u;
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < HB; ++j) {
            const bool ok = k < bw && j < bw;
            const double x = Tg[ok ? (trans ? j * bw + k : k * bw + j) : 0];
            t = fma(ok ? x : 0.0, s.W[j * HB_TW + lane], t);
        }
        y[u] = t;
    }
    __syncthreads();
    s.W[(2 * wave) * HB_TW + lane] = y[0];
    s.W[(2 * wave + 1) * HB_TW + lane] = y[1];
    __syncthreads();
    // ---- C -= V Y: 16-row blocks, D[row][col] = sum_k V[row][k] Y[k][col], 4 MFMAs (K = 16)
    double bvv[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) bvv[m] = s.W[(4 * m + lq) * HB_TW + 16 * cb + l16];
    for (int rb = pc + 16 * h; rb < rows; rb += 32) {
        double av[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) av[m] = hb_v(A, l, rows, pc, bw, rb + l16, 4 * m + lq);
        dbl4 p = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < 4; ++m) p = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bvv[m], p, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rb + lq + 4 * q;
            if (r < rows && cok) A[(int64_t)r * l + c] -= p[q];
        }
    }
    __syncthreads();
}

// Sum over the 32 row groups of the panel layout (thread = group * 16 + column):
// the per-column totals meet in LDS and every thread reads the total of column
// col.  Two barriers; red is free again on return.
__device__ __forceinline__ double hb_colsum(double v, double (*red)[HB], int col)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < HB) red[wave][lane] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < HB_T / 64; ++w) t += red[w][col];
    __syncthreads();
    return t;
}

// Factors the panel at column pc (bw <= 16 columns, rows [pc, rows)) in
// registers: RPT rows per thread, rows - pc <= 32 RPT.
template <int RPT>
__device__ void hb_panel(GLB double* __restrict__ A, int64_t l, int rows, int pc, int bw, GLB double* __restrict__ Tg,
                         GLB double* __restrict__ Dg, HbLds& s)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const int c = tid & 15, g = tid >> 4;
    const bool cok = c < bw;
    double x[RPT];
#pragma unroll
    for (int i0 = 0; i0 < RPT; i0 += 16) {
#pragma unroll
        for (int i = i0; i < i0 + 16 && i < RPT; ++i) {
            const int r = pc + g + HB_G * i;
            x[i] = ld_or0<double>(A, (int64_t)r * l + pc + c, r < rows && cok);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (tid < HB * HB) s.T[tid] = 0.0;
    // Register row i of this thread is row pc + g + 32 i.  For i >= 1 that row
    // lies below the diagonal of every panel column (j < 16 < 32), so only
    // i = 0 needs the row tests; rows past the end hold zeros.
    for (int j = 0; j < bw; ++j) {
        const bool below0 = g > j, diag0 = g == j;
        // squared norm of column j below the diagonal, and the diagonal entry alpha
        double p = below0 ? x[0] * x[0] : 0.0;
#pragma unroll
        for (int i = 1; i < RPT; ++i) p = fma(x[i], x[i], p);
        p = c == j ? p : 0.0;
        if (c == j && diag0) s.scal[0] = x[0];
        const double xn2 = hb_colsum(p, s.red, j);
        const double alpha = s.scal[0];
        double tau = 0.0, beta = alpha, sc = 1.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            sc = 1.0 / (alpha - beta);
        }
        {
            const double scl = c == j ? sc : 1.0;  // x * 1.0 == x: no branch over the rows
            x[0] *= below0 ? scl : 1.0;
#pragma unroll
            for (int i = 1; i < RPT; ++i) x[i] *= scl;
        }
        // v_j at this thread's rows comes from the lane of column j in the same
        // row group (all lanes shuffle; column j itself is not changed below),
        // in chunks of 16 rows so that not every shuffle result is held at once
        double dot;
        {
            const double xv = __shfl(x[0], (lane & 48) | j, 64);
            dot = (below0 ? xv : (diag0 ? 1.0 : 0.0)) * x[0];
        }
#pragma unroll
        for (int i0 = 1; i0 < RPT; i0 += 16) {
#pragma unroll
            for (int i = i0; i < i0 + 16 && i < RPT; ++i) dot = fma(__shfl(x[i], (lane & 48) | j, 64), x[i], dot);
            __builtin_amdgcn_sched_barrier(0);
        }
        // s_c = v_j^T (column c): the reflector's dots for c > j, V^T v_j for c < j
        const double sc_tot = hb_colsum(dot, s.red, c);
        const double f = c > j ? tau * sc_tot : 0.0;
        // the same shuffles as for the dots, recomputed: an opaque source lane keeps
        // the compiler from holding all RPT shuffle results across the reduction
        int src = (lane & 48) | j;
        asm volatile("" : "+v"(src));
        {
            const double xv = __shfl(x[0], src, 64);
            x[0] = fma(-f, below0 ? xv : (diag0 ? 1.0 : 0.0), x[0]);
        }
#pragma unroll
        for (int i0 = 1; i0 < RPT; i0 += 16) {
#pragma unroll
            for (int i = i0; i < i0 + 16 && i < RPT; ++i) x[i] = fma(-f, __shfl(x[i], src, 64), x[i]);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (c == j && g == j) x[0] = beta;
        // T column j: T[j][j] = tau, T[k][j] = -tau sum_{k <= q < j} T[k][q] s_q
        if (g == 0) s.red[0][c] = sc_tot;
        __syncthreads();
        if (tid < j) {
            double t = 0.0;
            for (int q = tid; q < j; ++q) t = fma(s.T[tid * HB + q], s.red[0][q], t);
            s.T[tid * HB + j] = -tau * t;
        }
        if (tid == 0) {
            s.T[j * HB + j] = tau;
            s.tau[j] = tau;
            s.beta[j] = beta;
        }
        __syncthreads();
    }
    // opaque copies, so that the row addresses of the loads are recomputed here
    // instead of being kept live through the factorisation
    int64_t ls = l;
    int g2 = g;
    asm volatile("" : "+s"(ls), "+v"(g2));
#pragma unroll
    for (int i0 = 0; i0 < RPT; i0 += 16) {
#pragma unroll
        for (int i = i0; i < i0 + 16 && i < RPT; ++i) {
            const int r = pc + g2 + HB_G * i;
            if (r < rows && cok) A[(int64_t)r * ls + pc + c] = x[i];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (tid < bw * bw) Tg[tid] = s.T[(tid / bw) * HB + tid % bw];
    if (tid < bw) {
        Dg[pc + tid] = s.tau[tid];
        Dg[l + pc + tid] = s.beta[tid];
    }
    __syncthreads();
}

// Q columns of the panel at pc (bw columns) from its reflectors: rows < pc are
// zero, rows >= pc are E - V (T V_top^T).  One row per thread at a time: a
// row's reflector entries are read before its Q entries are written, and no
// other thread touches that row.
__device__ void hb_panel_q(GLB double* __restrict__ A, int64_t l, int rows, int pc, int bw,
                           const GLB double* __restrict__ Tg, HbLds& s)
{
    const int tid = threadIdx.x;
    if (tid < HB * HB) {
        const int k = tid >> 4, cc = tid & 15;
        double t = 0.0;
        for (int j = 0; j < HB; ++j) {
            const bool ok = k < bw && j < bw && cc < bw;
            const double tk = Tg[ok ? k * bw + j : 0];
            t = fma(ok ? tk : 0.0, ok ? hb_v(A, l, rows, pc, bw, pc + cc, j) : 0.0, t);
        }
        s.Wc[tid] = t;
    }
    __syncthreads();
    for (int r = tid; r < rows; r += HB_T) {
        double out[HB];
#pragma unroll
        for (int cc = 0; cc < HB; ++cc) out[cc] = (r - pc == cc) ? 1.0 : 0.0;
        if (r >= pc) {
            // k outermost, one reflector entry and one row of Wc at a time (a fully
            // unrolled k x cc loop would hold all of Wc in registers)
#pragma unroll 2
            for (int k = 0; k < HB; ++k) {
                const double vk = hb_v(A, l, rows, pc, bw, r, k);
#pragma unroll
                for (int cc = 0; cc < HB; ++cc) out[cc] = fma(-vk, s.Wc[k * HB + cc], out[cc]);
            }
        }
#pragma unroll
        for (int cc = 0; cc < HB; ++cc)
            if (cc < bw) A[(int64_t)r * l + pc + cc] = out[cc];
    }
    __syncthreads();
}

template <int RPT>
__global__ __launch_bounds__(HB_T) void hb_kernel(const QrDesc* __restrict__ descs, int J, int mode)
{
    __shared__ HbLds s;
    const QrDesc& d = descs[blockIdx.y];
    if (d.Qout == nullptr || !*to_glb(d.flag)) return;
    const int rows = d.rows, l = d.l;
    const int t = blockIdx.x;
    const int lo = mode == HB_FACTOR ? HB * J : HB * (J + 1);
    const int c0 = lo + HB_TW * t;
    if (c0 >= l) return;
    const int c1 = min(c0 + HB_TW, l);
    GLB double* __restrict__ A = to_glb(d.Qout);
    GLB double* __restrict__ G = to_glb(d.G);
    GLB double* __restrict__ D = to_glb(d.D);
    const int tid = threadIdx.x;
    if (mode == HB_FACTOR) {
        if (J == 0) {
            const int lane = tid & 63, wave = tid >> 6;
            for (int r = wave; r < rows; r += HB_T / 64)
                if (c0 + lane < c1) A[(int64_t)r * l + c0 + lane] = ld_elem(d.Min, d.min_elem, (int64_t)r * l + c0 + lane);
            __syncthreads();
        } else {
            hb_update(A, l, rows, HB * (J - 1), HB, G + HB * HB * (J - 1), true, c0, c1, s);
        }
        if (t == 0) hb_panel<RPT>(A, l, rows, lo, min(HB, l - lo), G + HB * HB * J, D, s);
        return;
    }
    if (t == 0) hb_panel_q(A, l, rows, lo, min(HB, l - lo), G + HB * HB * (J + 1), s);
    if (J >= 0) {
        hb_update(A, l, rows, HB * J, HB, G + HB * HB * J, false, c0, c1, s);
    } else {
        const int lane = tid & 63, wave = tid >> 6;
        const int cc = c0 + lane;
        const bool neg = cc < c1 && D[cc < c1 ? l + cc : 0] < 0.0;
        if (neg)
            for (int r = wave; r < rows; r += HB_T / 64) A[(int64_t)r * l + cc] = -A[(int64_t)r * l + cc];
    }
}

int householder_blocked_rows_max() { return HB_G * 64; }

hipError_t launch_householder_blocked(const QrDesc* d, int nprob, int max_l, int max_rows, hipStream_t s)
{
    if (nprob <= 0 || max_l <= 0) return hipSuccess;
    if (max_rows > householder_blocked_rows_max()) return hipErrorInvalidValue;
    const int P = (max_l + HB - 1) / HB;
    auto go = [&](int J, int mode) {
        const int lo = mode == HB_FACTOR ? HB * J : HB * (J + 1);
        const dim3 grid((max_l - lo + HB_TW - 1) / HB_TW, nprob);
        if (max_rows <= HB_G * 16)
            hipLaunchKernelGGL(hb_kernel<16>, grid, dim3(HB_T), 0, s, d, J, mode);
        else if (max_rows <= HB_G * 32)
            hipLaunchKernelGGL(hb_kernel<32>, grid, dim3(HB_T), 0, s, d, J, mode);
        else
            hipLaunchKernelGGL(hb_kernel<64>, grid, dim3(HB_T), 0, s, d, J, mode);
        return hipGetLastError();
    };
    hipError_t e = hipSuccess;
    for (int J = 0; J < P && e == hipSuccess; ++J) e = go(J, HB_FACTOR);
    for (int J = P - 2; J >= -1 && e == hipSuccess; --J) e = go(J, HB_QFORM);
    return e;
}

static size_t chol_lds_bytes(int max_l)
{
    return (size_t)(((max_l + 1) & ~1) + (size_t)max_l * 17) * sizeof(double);  // g0, then Lp rows < l
}

hipError_t launch_chol(const QrDesc* d, int nprob, int max_l, hipStream_t s)
{
    // problems with l <= 288 take the register-resident kernel, wider ones the
    // general one (each kernel skips the other's problems)
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(chol_reg_kernel, dim3(nprob), dim3(CHR_NT), 0, s, d);
    if (max_l <= CHR_T * 16) return hipGetLastError();
    const size_t lds = chol_lds_bytes(max_l);
    hipLaunchKernelGGL(chol_rl_kernel<512>, dim3(nprob), dim3(512), lds, s, d, CHR_T * 16 + 1);
    return hipGetLastError();
}

hipError_t launch_trsm(const QrDesc* d, const int* row_begin, int nprob, int total_blocks, int from_min,
                       int src_elem, int max_l, hipStream_t s)
{
    // row blocks of problems with l <= 288 take the register-resident kernel,
    // those of wider ones the general one (each kernel skips the other's)
    if (total_blocks <= 0) return hipSuccess;
    const bool f32 = from_min && src_elem == E_F32;
    if (!f32 && from_min && src_elem != E_F64) return hipErrorInvalidValue;
    if (f32)
        hipLaunchKernelGGL(trsm_reg_kernel<float>, dim3(total_blocks), dim3(64), 0, s, d, row_begin, nprob, from_min);
    else
        hipLaunchKernelGGL(trsm_reg_kernel<double>, dim3(total_blocks), dim3(64), 0, s, d, row_begin, nprob, from_min);
    if (max_l <= CHR_T * 16) return hipGetLastError();
    const size_t lds = (size_t)16 * (max_l + 1) * sizeof(double);
    const int min_l = CHR_T * 16 + 1;
    if (f32)
        hipLaunchKernelGGL(trsm_kernel<float>, dim3(total_blocks), dim3(64), lds, s, d, row_begin, nprob, from_min, min_l);
    else
        hipLaunchKernelGGL(trsm_kernel<double>, dim3(total_blocks), dim3(64), lds, s, d, row_begin, nprob, from_min, min_l);
    return hipGetLastError();
}

hipError_t init_qr_kernels()
{
    hipError_t e = hipFuncSetAttribute((const void*)chol_rl_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)chol_lds_bytes(CHOL_MAX_L));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)trsm_upper_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       16 * (CHOL_MAX_L + 1) * (int)sizeof(double));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)tri_prep_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (CHOL_MAX_L / 16) * 272 * (int)sizeof(double));
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)trsm_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            16 * (CHOL_MAX_L + 1) * (int)sizeof(double));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)trsm_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               16 * (CHOL_MAX_L + 1) * (int)sizeof(double));
}

hipError_t launch_householder(const QrDesc* d, int nprob, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(householder_kernel, dim3(nprob), dim3(HH_T), 0, s, d);
    return hipGetLastError();
}

}  // namespace rsvd
