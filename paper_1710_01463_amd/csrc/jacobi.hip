// Block one-sided Jacobi SVD (Hestenes), used for
//   - the small SVD of B = Q^T A in Alg. RSVD step 4 (paper Sec. II.B; the
//     paper uses LAPACK GESVD there, any backward-stable SVD serves), and
//   - the full SVD of Alg. TSVD (Sec. II.A), the deterministic baseline.
//
// The vectors being orthogonalised are the R rows of X (R x C, R <= C); the
// left rotations are accumulated in P (R x R), so that P X_in = X_out with
// mutually orthogonal rows.  Rows are grouped in blocks of JAC_B.  One launch
// is one round of the round-robin schedule over the nb blocks: each workgroup
// takes one block pair (JR = 2 JAC_B rows), forms their JR x JR Gram matrix
// with FP64 MFMA, checks the relative off-diagonal |h_ij| <= tol
// sqrt(h_ii h_jj), and if needed diagonalises it by one sweep of cyclic
// two-sided Jacobi in LDS (with many blocks, rounds 2.. of a sweep rotate only
// the row pairs across the two blocks), then applies the accumulated JR x JR
// rotation to the JR rows of X and of P with FP64 MFMA.  A sweep is nb - 1
// rounds; a problem is converged after a sweep in which no off-diagonal entry
// of any block pair was above the threshold.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

constexpr int JR = 2 * JAC_B;                    // rows per block pair
constexpr int JNP = JR / 2;                      // plane pairs per inner step
constexpr int JHB = JNP * JNP;                   // 2 x 2 blocks of the pair's Gram
constexpr int JT = (2 * JHB <= 1024) ? 2 * JHB : JHB;  // threads per workgroup
constexpr bool JSPLIT = JT == 2 * JHB;           // separate threads update P
constexpr int JCH = JR >= 64 ? 64 : JAC_CHUNK;   // column chunk staged through LDS
constexpr int JPF = JR * JCH / JT;               // prefetched doubles per thread
constexpr int JTILES = (JR / 16) * (JR / 16);    // 16 x 16 Gram tiles
constexpr int JKS = (JT / 64) / JTILES;          // waves sharing one Gram tile (k split)
static_assert(JKS >= 1 && (JT / 64) % JTILES == 0, "Gram tiling");

__device__ __forceinline__ int rr_block(int pos, int round, int nb)
{
    return pos == 0 ? 0 : ((pos - 1 + round) % (nb - 1)) + 1;
}

// |g| > tol sqrt(a b), with hardware square roots (about 2^-22 relative):
// the threshold only decides whether a rotation is worth doing.
__device__ __forceinline__ bool jac_needs(double a, double b, double g, double tol)
{
    return a > 0.0 && b > 0.0 && fabs(g) > tol * (__builtin_amdgcn_sqrt(a) * __builtin_amdgcn_sqrt(b));
}

// Rotation (c, s) that (nearly) zeroes the (p, q) entry of a symmetric 2 x 2
// block [a g; g b] under x_p <- c x_p - s x_q, x_q <- s x_p + c x_q, from the
// classical Hestenes/Jacobi formula t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// zeta = (b - a) / (2 g) (scale free).  The angle may be approximate (hardware
// reciprocal and square root): a slightly-off rotation leaves a tiny
// off-diagonal that later rotations remove.  What must hold to working
// precision is c^2 + s^2 = 1, so c = (1 + t^2)^(-1/2) is refined by two Newton
// steps.  Everything is computed unconditionally and the identity selected
// when no rotation is needed, so the threshold test is off the dependent
// chain (each dependent FP64 operation costs tens of cycles).
__device__ __forceinline__ void jac_rotation(double a, double b, double g, double tol, double& cs, double& sn)
{
    const double zeta = (b - a) * __builtin_amdgcn_rcp(2.0 * g);
    const double az = fabs(zeta);
    const double tb = copysign(__builtin_amdgcn_rcp(az + __builtin_amdgcn_sqrt(fma(zeta, zeta, 1.0))), zeta);
    const double t = (az > 1e150) ? 0.5 * __builtin_amdgcn_rcp(zeta) : tb;
    const double x = fma(t, t, 1.0);
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = x * y;
        const double e = fma(-h, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    const bool rot = jac_needs(a, b, g, tol);
    cs = rot ? y : 1.0;
    sn = rot ? y * t : 0.0;
}

// A 32 x JCH chunk in registers: slot k of lane (l16, lq) of wave w holds
// element (4 k + lq, 16 w + l16), the B operand layout of a 16 x 16 x 4 FP64
// MFMA for column tile w, so the rotation multiplies the rows where they were
// loaded (each load instruction reads four rows of 128 contiguous bytes).
constexpr int JWAVES = JT / 64;
static_assert(JCH == 16 * JWAVES && JR == 4 * JPF, "one column tile per wave, one row per slot and lane row");

// Loads the chunk (rows via rowmap, columns c0..) of M as loaded (an
// out-of-range element reads an in-range one) and returns the in-range mask,
// applied where the chunk is used: nothing consumes a loaded value before
// then, so the loads stay in flight (across the inner sweep for the rows of P).
__device__ __forceinline__ uint32_t load_chunk(double (&pre)[JPF], const GLB double* __restrict__ M, int64_t ldm,
                                               int ncols, int c0, const int* rowmap)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gc = c0 + 16 * wave + (lane & 15), lq = lane >> 4;
    uint32_t ok = 0;
#pragma unroll
    for (int k = 0; k < JPF; ++k) {
        const int gr = rowmap[4 * k + lq];
        const bool in = gr >= 0 && gc < ncols;
        pre[k] = M[in ? (int64_t)gr * ldm + gc : 0];
        ok |= (uint32_t)in << k;
    }
    return ok;
}
__device__ __forceinline__ void store_chunk(const double (&pre)[JPF], uint32_t ok, double (*Xs)[JCH + 1])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = 16 * wave + (lane & 15), lq = lane >> 4;
#pragma unroll
    for (int k = 0; k < JPF; ++k) Xs[4 * k + lq][c] = ((ok >> k) & 1u) ? pre[k] : 0.0;
}

// The augmented rows [X | P] of the pair, JCH columns at a time: chunk ci < ncx
// is columns ci*JCH.. of X, later chunks are columns of P.
struct ChunkSeq {
    GLB double* X;
    GLB double* P;
    int64_t ldx, ldp;
    int C, R, ncx, nct;
    __device__ void select(int ci, GLB double*& M, int64_t& ldm, int& ncols, int& c0) const
    {
        const bool in_x = ci < ncx;
        M = in_x ? X : P;
        ldm = in_x ? ldx : ldp;
        ncols = in_x ? C : R;
        c0 = (in_x ? ci : ci - ncx) * JCH;
    }
    __device__ uint32_t load(double (&pre)[JPF], int ci, const int* rowmap) const
    {
        GLB double* M;
        int64_t ldm;
        int ncols, c0;
        select(ci, M, ldm, ncols, c0);
        return load_chunk(pre, M, ldm, ncols, c0, rowmap);
    }
};

// The rotation phase: rows <- Ps (JR x JR) * rows, chunk by chunk, straight
// from the registers the chunk was loaded into: wave w forms both 16-row
// tiles of column tile w (two interleaved MFMA chains over the same B
// operands, the A operands being all of Ps, loaded once per phase), and the
// destination rows come from registers; no LDS staging and no barrier.  A
// column tile wholly outside the matrix is left out.  Each output element is
// the same k-ordered sum as one 16 x 16 x JR product.
constexpr int JRT = JR / 16;  // row tiles
static_assert(JRT == 2, "two row tiles per pair");

struct RotLane {
    double pa[JRT][JR / 4];  // A operands: Ps rows of each row tile
    int grow[JRT][4];        // destination rows of the lane's outputs (-1: padding)
};

__device__ __forceinline__ void rot_lane_init(RotLane& rl, const double (*Ps)[JR + 1], const int* rowmap)
{
    const int lane = threadIdx.x & 63;
    const int l16 = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int rt = 0; rt < JRT; ++rt) {
#pragma unroll
        for (int k = 0; k < JR / 4; ++k) rl.pa[rt][k] = Ps[rt * 16 + l16][4 * k + lq];
#pragma unroll
        for (int r = 0; r < 4; ++r) rl.grow[rt][r] = rowmap[rt * 16 + lq + 4 * r];
    }
}

// One chunk held in x (as loaded, with its in-range mask ok) at columns c0..
// of M.
__device__ __forceinline__ void rotate_chunk(const RotLane& rl, const double (&x)[JPF], uint32_t ok, GLB double* M,
                                             int64_t ldm, int ncols, int c0)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gc = c0 + 16 * wave + (lane & 15);
    if (c0 + 16 * wave >= ncols) return;  // wave-uniform: the column tile is outside
    dbl4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < JR / 4; ++k) {
        // padding rows read as zeros (an out-of-range value is any in-range
        // element, and 0 * inf would not vanish)
        const double b = ((ok >> k) & 1u) ? x[k] : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(rl.pa[0][k], b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(rl.pa[1][k], b, acc1, 0, 0, 0);
    }
    if (gc < ncols) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int g0 = rl.grow[0][r], g1 = rl.grow[1][r];
            if (g0 >= 0) st_through(&M[(int64_t)g0 * ldm + gc], acc0[r]);
            if (g1 >= 0) st_through(&M[(int64_t)g1 * ldm + gc], acc1[r]);
        }
    }
}

// Streaming: chunk 0 of the sequence is already in pre; each next chunk is
// loaded into the other register set while the current one is multiplied.
__device__ void apply_rotation(const ChunkSeq& cs, double (&pre)[JPF], uint32_t ok, const RotLane& rl,
                               const int* rowmap)
{
    double nxt[JPF];
    for (int ci = 0; ci < cs.nct; ci += 2) {
        uint32_t okn = 0;
        if (ci + 1 < cs.nct) okn = cs.load(nxt, ci + 1, rowmap);
        GLB double* M;
        int64_t ldm;
        int ncols, c0;
        cs.select(ci, M, ldm, ncols, c0);
        rotate_chunk(rl, pre, ok, M, ldm, ncols, c0);
        if (ci + 1 >= cs.nct) break;
        if (ci + 2 < cs.nct) ok = cs.load(pre, ci + 2, rowmap);
        cs.select(ci + 1, M, ldm, ncols, c0);
        rotate_chunk(rl, nxt, okn, M, ldm, ncols, c0);
    }
}

constexpr int JAC_INNER_SWEEPS = 1;

// Resident: res[ch] is chunk ch0 + ch of the sequence; no load on the way.
template <int NS>
__device__ void apply_rotation_resident(const ChunkSeq& cs, const double (&res)[NS][JPF], const uint32_t (&ok)[NS],
                                        int ch0, int ch_end, const RotLane& rl)
{
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
        const int ci = ch0 + sl;
        if (ci >= ch_end) break;  // uniform
        GLB double* M;
        int64_t ldm;
        int ncols, c0;
        cs.select(ci, M, ldm, ncols, c0);
        rotate_chunk(rl, res[sl], ok[sl], M, ldm, ncols, c0);
    }
}

// One round of the block Jacobi schedule.  RX > 0: the pair's rows of X
// (at most RX column chunks) are loaded into registers at once at the start
// and reused for the rotation, and the rows of P (at most RP chunks) are
// loaded during the inner solve, so that the global-memory latency is paid
// about twice per round instead of once per chunk.  RX = 0: chunks are
// streamed through a one-deep register prefetch (any C and R).
// Outcome of one block-pair task: the problem had already converged (the
// previous sweep rotated nothing), or the task ran (rotating or not).
enum JacOutcome { JAC_CONVERGED = 0, JAC_RAN = 1 };

template <int RX, int RP>
__device__ __forceinline__ int jacobi_pair_task(const JacDesc& d, int slot, int sweep, int round)
{
    __shared__ double Xs[JR][JCH + 1];
    __shared__ double Hbuf[2][JR][JR + 1];
    __shared__ double Ps[JR][JR + 1];
    __shared__ int rowmap[JR];
    __shared__ int any_rot;

    const int nb = d.nb;
    GLB int* __restrict__ rot = to_glb(d.rot);
    // (an atomic load: in the persistent kernel another workgroup set the flag
    // during this launch, and a scalar-cache load could be stale)
    if (sweep > 0 && __hip_atomic_load((int*)&rot[sweep - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return JAC_CONVERGED;
    // With an odd number of row blocks, the padding block (nb - 1) takes the
    // fixed position 0 of the round-robin schedule, so that its pair is always
    // slot 0: that slot is not launched (the other blocks sit out once per sweep).
    const int pi = slot + d.skip0;
    int I = rr_block(pi, round, nb);
    int J = rr_block(nb - 1 - pi, round, nb);
    if (d.skip0) {
        I = I == 0 ? nb - 1 : I - 1;
        J = J == 0 ? nb - 1 : J - 1;
    }
    const int R = d.R, C = d.C;
    const double tol = d.tol;
    GLB double* __restrict__ X = to_glb(d.X);
    const int64_t ldx = d.ldx;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    if (tid < JR) {
        const int gr = (tid < JAC_B) ? I * JAC_B + tid : J * JAC_B + (tid - JAC_B);
        rowmap[tid] = (gr < R) ? gr : -1;
    }
    if (tid == 0) any_rot = 0;
    ChunkSeq seq;
    seq.X = X;
    seq.P = to_glb(d.P);
    seq.ldx = ldx;
    seq.ldp = d.ldp;
    seq.C = C;
    seq.R = R;
    seq.ncx = (C + JCH - 1) / JCH;
    seq.nct = seq.ncx + (d.P ? (R + JCH - 1) / JCH : 0);
    __syncthreads();

    // ---- Gram matrix of the JR rows (FP64 MFMA): wave w forms the 16 x 16
    // tile (w % JTILES) over its share (w / JTILES of JKS) of every column
    // chunk; with JKS = 2 the two halves are added through LDS
    constexpr int NRX = RX > 0 ? RX : 1;
    double resx[NRX][JPF];
    uint32_t okx[NRX] = {};
    {
        const int tile = wave % JTILES;
        const int wi = tile / (JR / 16), wj = tile % (JR / 16), half = wave / JTILES;
        dbl4 acc = {0, 0, 0, 0};
        auto gram_chunk = [&]() {
#pragma unroll 8
            for (int kk = half * (JCH / JKS); kk < (half + 1) * (JCH / JKS); kk += 4) {
                const double av = Xs[wi * 16 + l16][kk + lq];
                const double bv = Xs[wj * 16 + l16][kk + lq];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
        };
        if constexpr (RX > 0) {
            // every X chunk in flight at once (slots past the row length
            // re-read chunk 0 and are not used)
#pragma unroll
            for (int ch = 0; ch < RX; ++ch) okx[ch] = load_chunk(resx[ch], X, ldx, C, (ch < seq.ncx ? ch : 0) * JCH, rowmap);
#pragma unroll
            for (int ch = 0; ch < RX; ++ch) {
                if (ch > 0 && ch >= seq.ncx) break;  // uniform; no load below
                store_chunk(resx[ch], okx[ch], Xs);
                __syncthreads();
                gram_chunk();
                __syncthreads();
            }
        } else {
            double pre[JPF];
            uint32_t okc = load_chunk(pre, X, ldx, C, 0, rowmap);
            for (int c0 = 0; c0 < C; c0 += JCH) {
                store_chunk(pre, okc, Xs);
                __syncthreads();
                if (c0 + JCH < C) okc = load_chunk(pre, X, ldx, C, c0 + JCH, rowmap);
                gram_chunk();
                __syncthreads();
            }
        }
        static_assert(JKS <= 2, "Gram halves");
        if (JKS == 2 && half == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) Hbuf[1][wi * 16 + lq + 4 * r][wj * 16 + l16] = acc[r];
        }
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Hbuf[0][wi * 16 + lq + 4 * r][wj * 16 + l16] =
                    acc[r] + (JKS == 2 ? Hbuf[1][wi * 16 + lq + 4 * r][wj * 16 + l16] : 0.0);
        }
    }
    // streaming: prefetch the first chunk of the rotation phase; it lands during the inner solve
    double pre[JPF];
    uint32_t okpre = 0;
    if constexpr (RX == 0) okpre = seq.load(pre, 0, rowmap);
    __syncthreads();
    // symmetrise from the upper triangle, identity for P
    for (int e = tid; e < JR * JR; e += JT) {
        const int i = e / JR, j = e % JR;
        if (i > j) Hbuf[0][i][j] = Hbuf[0][j][i];
        Ps[i][j] = (i == j) ? 1.0 : 0.0;
    }
    // cross round: only the row pairs across the two blocks are rotated (the
    // pairs inside a block are visited in the full rounds 0 and 1)
    const bool cross = d.cross_rounds && round >= 2;
    __syncthreads();
    // any_rot bit 0: some off-diagonal entry above the threshold (the sweep
    // has not converged); bit 1: some entry that this round rotates.  The
    // lanes' findings are combined by ballot and each wave sets the flag with
    // one LDS atomic (lane atomics on one word serialise across the CU).
    {
        int need = 0;
        for (int e = tid; e < JR * JR; e += JT) {
            const int i = e / JR, j = e % JR;
            if (i < j) {
                const double a = Hbuf[0][i][i], c = Hbuf[0][j][j], g = Hbuf[0][i][j];
                if (jac_needs(a, c, g, tol)) need |= (!cross || (i < JAC_B && j >= JAC_B)) ? 3 : 1;
            }
        }
        const unsigned long long any1 = __ballot(need & 1), any2 = __ballot(need & 2);
        if (lane == 0 && any1) atomicOr(&any_rot, any2 ? 3 : 1);
    }
    __syncthreads();
    if (tid == 0) {
        GLB int* st = to_glb(d.stats);
        atomicAdd((int*)&st[0], 1);
        if (any_rot & 2) atomicAdd((int*)&st[1], 1);
        if (any_rot) rot[sweep] = 1;
    }
    if (!(any_rot & 2)) return JAC_RAN;
    // resident: the rows of P, in flight during the inner solve
    constexpr int NRP = RP > 0 ? RP : 1;
    double resp[NRP][JPF];
    uint32_t okp[NRP] = {};
    if constexpr (RX > 0) {
#pragma unroll
        for (int sl = 0; sl < RP; ++sl) {
            const int ci = seq.ncx + sl;
            okp[sl] = seq.load(resp[sl], ci < seq.nct ? ci : 0, rowmap);
        }
    }

    // ---- inner cyclic Jacobi on the JR x JR Gram matrix, parallel order.
    // Thread t (mod JHB), (pi_, pj_) = (t / JNP, t % JNP), owns the 2 x 2 block
    // (pair pi_ rows) x (pair pj_ cols) of H and/or the 2 x 2 block (pair pi_
    // rows) x (columns 2 pj_, 2 pj_ + 1) of P: with 2 JHB <= 1024 threads the
    // two updates run side by side on separate threads.  H is double-buffered
    // so one barrier per step suffices.  With separate P threads, only the H
    // threads compute the rotations: they leave the step's JNP rotations in an
    // LDS table (double-buffered by step parity), and the P threads apply step
    // s - 1's during step s (nothing in H depends on P), and the last one after
    // the loop; the same products as when every thread computes them.
    const bool on_h = !JSPLIT || tid < JHB;
    const bool on_p = !JSPLIT || tid >= JHB;
    const int pr_i = (tid % JHB) / JNP, pr_j = tid % JNP;
    static_assert(JNP <= 64 && 64 % JNP == 0, "every wave computes all plane-pair rotations");
    __shared__ double rot_tab[2][JNP][2];
    const int nsteps = cross ? JAC_B : JR - 1;
    const int gsteps = JAC_INNER_SWEEPS * nsteps;
    // The plane pair indices at step 0 and their advance by one step, instead
    // of the schedule's modulo arithmetic at every step: in a full round
    // (round robin over all JR rows) a position other than 0 moves to the next
    // one, JR wrapping to 1; in a cross round row p of block I stays and row
    // JAC_B + (p + step) mod JAC_B of block J moves on, JR wrapping to JAC_B.
    // Both cycles have nsteps steps, so the indices are back at their step-0
    // values after every inner sweep.  The advance is plain arithmetic (JR is
    // a power of two and a position at most JR after the increment), so no
    // lane branches on it.
    static_assert((JR & (JR - 1)) == 0, "power-of-two pair rows");
    const unsigned q_back = cross ? JR - JAC_B : JR - 1;  // JR -> restart row
    auto first = [&](int pr, unsigned& p, unsigned& q, unsigned& p_inc) {
        p = cross ? pr : rr_block(pr, 0, JR);
        q = cross ? JAC_B + pr : rr_block(JR - 1 - pr, 0, JR);
        p_inc = (cross || pr == 0) ? 0u : 1u;
    };
    auto advance = [&](unsigned& p, unsigned& q, unsigned p_inc) {
        p += p_inc;
        p -= __umul24(p / JR, JR - 1);
        q += 1;
        q -= __umul24(q / JR, q_back);
        __builtin_assume(p < JR);
        __builtin_assume(q < JR);
    };
    // element (r, c) of a JR x (JR + 1) LDS array, the row offset by a 24-bit
    // multiply (indices below JR)
    auto at = [](double (*M)[JR + 1], unsigned r, unsigned c) -> double& {
        return (&M[0][0])[__umul24(r, JR + 1) + c];
    };
    auto update_p = [&](unsigned p_i, unsigned q_i, double ci, double si) {
        if (si != 0.0) {
            const unsigned c0 = 2 * pr_j, c1 = 2 * pr_j + 1;
            const double x0 = at(Ps, p_i, c0), x1 = at(Ps, p_i, c1), y0 = at(Ps, q_i, c0), y1 = at(Ps, q_i, c1);
            at(Ps, p_i, c0) = ci * x0 - si * y0;
            at(Ps, p_i, c1) = ci * x1 - si * y1;
            at(Ps, q_i, c0) = si * x0 + ci * y0;
            at(Ps, q_i, c1) = si * x1 + ci * y1;
        }
    };
    unsigned p_i, q_i, p_j, q_j;  // this step's rows of pair pr_i and pair pr_j (P threads: the previous step's)
    unsigned inc_i, inc_j;
    first(pr_i, p_i, q_i, inc_i);
    first(pr_j, p_j, q_j, inc_j);
    for (int gs = 0; gs < gsteps; ++gs) {
        if (on_h) {
            double (*H)[JR + 1] = Hbuf[gs & 1];
            double (*Hn)[JR + 1] = Hbuf[(gs & 1) ^ 1];
            // each lane computes the rotation of plane pair pr_j (= lane % JNP,
            // so every wave holds all JNP of them) and takes pair pr_i's from
            // the lane that computed it: one rotation per thread, not two
            double cj, sj;
            jac_rotation(at(H, p_j, p_j), at(H, q_j, q_j), at(H, p_j, q_j), tol, cj, sj);
            const double ci = __shfl(cj, pr_i, 64), si = __shfl(sj, pr_i, 64);
            const double b00 = at(H, p_i, p_j), b01 = at(H, p_i, q_j), b10 = at(H, q_i, p_j), b11 = at(H, q_i, q_j);
            const double t00 = ci * b00 - si * b10, t01 = ci * b01 - si * b11;
            const double t10 = si * b00 + ci * b10, t11 = si * b01 + ci * b11;
            at(Hn, p_i, p_j) = t00 * cj - t01 * sj;
            at(Hn, p_i, q_j) = t00 * sj + t01 * cj;
            at(Hn, q_i, p_j) = t10 * cj - t11 * sj;
            at(Hn, q_i, q_j) = t10 * sj + t11 * cj;
            if constexpr (JSPLIT) {
                if (tid < JNP) {
                    rot_tab[gs & 1][tid][0] = cj;
                    rot_tab[gs & 1][tid][1] = sj;
                }
            } else {
                update_p(p_i, q_i, ci, si);
            }
            advance(p_i, q_i, inc_i);
            advance(p_j, q_j, inc_j);
        } else if (gs > 0) {
            update_p(p_i, q_i, rot_tab[(gs - 1) & 1][pr_i][0], rot_tab[(gs - 1) & 1][pr_i][1]);
            advance(p_i, q_i, inc_i);
        }
        __syncthreads();
    }
    if (JSPLIT && on_p && gsteps > 0)
        update_p(p_i, q_i, rot_tab[(gsteps - 1) & 1][pr_i][0], rot_tab[(gsteps - 1) & 1][pr_i][1]);

    // ---- apply the accumulated rotation to the rows of X and of P
    __syncthreads();  // Ps complete
    RotLane rl;
    rot_lane_init(rl, Ps, rowmap);
    if constexpr (RX > 0) {
        apply_rotation_resident<RX>(seq, resx, okx, 0, seq.ncx, rl);
        apply_rotation_resident<RP>(seq, resp, okp, seq.ncx, seq.nct, rl);
    } else {
        apply_rotation(seq, pre, okpre, rl, rowmap);
    }
    return JAC_RAN;
}

template <int RX, int RP>
__global__ __launch_bounds__(JT) void jacobi_round_kernel(const JacDesc* __restrict__ descs,
                                                           const int* __restrict__ pair_begin, int nprob,
                                                           int sweep, int round)
{
    const int2 wi_ = wg_item(pair_begin, blockIdx.x);
    const JacDesc& d = descs[wi_.x];
    if (round >= d.nb - 1) return;
    (void)jacobi_pair_task<RX, RP>(d, wi_.y, sweep, round);
}

// All rounds of all sweeps in one launch.  The tasks are the (sweep, round,
// block pair) items of the round launches above, in the same order: task t
// is round g = t / total_pairs of the schedule and entry t % total_pairs of
// the launch's pair map.  Workgroups take tasks from a global counter and
// wait only for their own problem: a task of local round r (r counts the
// rounds that problem takes part in) starts once the problem's first r
// rounds have all finished, which the problem's task counter (stats[2])
// shows as r * pairs-per-round.  Problems therefore advance independently
// (no grid-wide step), so one problem's row traffic overlaps another's inner
// sweeps, and no launch boundary separates the rounds.
//   - Deadlock freedom: tasks are taken in order and a task depends only on
//     earlier tasks, which were taken by running workgroups; the earliest
//     unfinished task always has its dependencies met.  Residency of the
//     grid is not assumed.
//   - Memory: a finished task's stores reach every XCD by an agent-scope
//     release before its counter increment; a waiting task acquires at agent
//     scope after seeing the count (the L2 of each XCD is written back and
//     invalidated).  Flags are read with atomic loads, never from the scalar
//     cache.
//   - Convergence: the first task of a converged problem sets stats[3]; later
//     tasks of that problem skip without waiting.
//   - Every wait is bounded: after spin_limit polls the workgroup sets the
//     error flag sched[1] and every workgroup leaves at its next poll or
//     task, so the grid always drains; the finishing step reports the error.
template <int RX, int RP>
__global__ __launch_bounds__(JT) void jacobi_persistent_kernel(const JacDesc* __restrict__ descs,
                                                                const int* __restrict__ pair_map, int total_pairs,
                                                                int rounds_per_sweep, int max_sweeps,
                                                                int* __restrict__ sched, int spin_limit)
{
    __shared__ int ctl[4];  // task state, problem, slot, schedule round
    const int tid = threadIdx.x;
    const int64_t ntasks = (int64_t)max_sweeps * rounds_per_sweep * total_pairs;
    int* next = sched;
    int* err = sched + 1;
    for (;;) {
        __syncthreads();  // the previous task is done with the shared arrays and ctl
        if (tid == 0) {
            // state: 0 no work in this task, 1 run, 2 leave
            int state = 2, b = 0, slot = 0, g = 0;
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                const int t = __hip_atomic_fetch_add(next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((int64_t)t < ntasks) {
                    g = t / total_pairs;
                    const int2 wi = wg_item(pair_map, t % total_pairs);
                    b = wi.x;
                    slot = wi.y;
                    const JacDesc& d = descs[b];
                    const int sweep = g / rounds_per_sweep, round = g % rounds_per_sweep;
                    state = 0;
                    if (round < d.nb - 1) {
                        int* cnt = d.stats + 2;
                        int* done = d.stats + 3;
                        const int np = d.nb / 2 - d.skip0;
                        const int need = (sweep * (d.nb - 1) + round) * np;
                        for (int it = 0;; ++it) {
                            if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                            if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) {
                                state = 1;
                                break;
                            }
                            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                state = 2;
                                break;
                            }
                            if (it >= spin_limit) {
                                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                state = 2;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(2);
                        }
                        // the rows written by the tasks just counted are visible below
                        if (state == 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                }
            }
            ctl[0] = state;
            ctl[1] = b;
            ctl[2] = slot;
            ctl[3] = g;
        }
        __syncthreads();
        const int state = ctl[0];
        if (state == 2) break;
        if (state == 0) continue;
        const JacDesc& d = descs[ctl[1]];
        const int g = ctl[3];
        const int res = jacobi_pair_task<RX, RP>(d, ctl[2], g / rounds_per_sweep, g % rounds_per_sweep);
        __syncthreads();  // every wave's stores of this task are issued before the release below
        if (tid == 0) {
            if (res == JAC_CONVERGED) {
                __hip_atomic_store(d.stats + 3, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(d.stats + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

int jacobi_resident_variant(int max_x_chunks, int max_p_chunks)
{
    if (max_x_chunks <= 4 && max_p_chunks <= 3) return 1;
    if (max_x_chunks <= 4 && max_p_chunks <= 4) return 2;
    if (max_x_chunks <= 8 && max_p_chunks <= 2) return 3;
    return 0;
}

template <int RX, int RP>
static hipError_t persistent_t(const JacDesc* d, const int* pair_map, int total_pairs, int rounds_per_sweep,
                               int max_sweeps, int* sched, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((jacobi_persistent_kernel<RX, RP>), dim3(grid), dim3(JT), 0, s, d, pair_map, total_pairs,
                       rounds_per_sweep, max_sweeps, sched, JAC_SPIN_LIMIT);
    return hipGetLastError();
}

hipError_t launch_jacobi_persistent(const JacDesc* d, const int* pair_map, int total_pairs, int rounds_per_sweep,
                                    int max_sweeps, int* sched, int grid, int variant, hipStream_t s)
{
    if (total_pairs <= 0 || grid <= 0) return hipSuccess;
    switch (variant) {
    case 1: return persistent_t<4, 3>(d, pair_map, total_pairs, rounds_per_sweep, max_sweeps, sched, grid, s);
    case 2: return persistent_t<4, 4>(d, pair_map, total_pairs, rounds_per_sweep, max_sweeps, sched, grid, s);
    case 3: return persistent_t<8, 2>(d, pair_map, total_pairs, rounds_per_sweep, max_sweeps, sched, grid, s);
    default: return persistent_t<0, 0>(d, pair_map, total_pairs, rounds_per_sweep, max_sweeps, sched, grid, s);
    }
}

int jacobi_persistent_blocks_per_cu(int variant)
{
    int nb = 0;
    hipError_t e;
    switch (variant) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, jacobi_persistent_kernel<4, 3>, JT, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, jacobi_persistent_kernel<4, 4>, JT, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, jacobi_persistent_kernel<8, 2>, JT, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, jacobi_persistent_kernel<0, 0>, JT, 0); break;
    }
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_jacobi_round(const JacDesc* d, const int* pair_begin, int nprob, int total_pairs,
                               int sweep, int round, int variant, hipStream_t s)
{
    if (total_pairs <= 0) return hipSuccess;
    switch (variant) {
    case 1:
        hipLaunchKernelGGL((jacobi_round_kernel<4, 3>), dim3(total_pairs), dim3(JT), 0, s, d, pair_begin, nprob, sweep,
                           round);
        break;
    case 2:
        hipLaunchKernelGGL((jacobi_round_kernel<4, 4>), dim3(total_pairs), dim3(JT), 0, s, d, pair_begin, nprob, sweep,
                           round);
        break;
    case 3:
        hipLaunchKernelGGL((jacobi_round_kernel<8, 2>), dim3(total_pairs), dim3(JT), 0, s, d, pair_begin, nprob, sweep,
                           round);
        break;
    default:
        hipLaunchKernelGGL((jacobi_round_kernel<0, 0>), dim3(total_pairs), dim3(JT), 0, s, d, pair_begin, nprob, sweep,
                           round);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- finishing
// The finishing step is split so that only the O(R^2) rank sort and the
// serial discarded-weight scan run in one workgroup per problem; the row norms
// before it and the gathers of the singular vectors after it are wide,
// coalesced launches over (problem, row group) work items.
constexpr int FIN_MAXR = 2048;

// sig[i] = ||X row i|| for the R rows of every problem (unsorted); one wave per row.
__global__ __launch_bounds__(256) void rownorm_kernel(const FinDesc* __restrict__ descs,
                                                      const int* __restrict__ map, int nprob)
{
    const int2 wi_ = wg_item(map, blockIdx.x);
    const FinDesc& d = descs[wi_.x];
    const int lane = threadIdx.x & 63, i = 4 * wi_.y + (threadIdx.x >> 6);
    if (i >= d.R) return;
    const int C = d.C;
    const GLB double* __restrict__ X = to_glb(d.X) + (int64_t)i * d.ldx;
    double s = 0.0;
    for (int t0 = lane; t0 < C; t0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 64 * u;
            v[u] = ld_or0(X, t, t < C);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fma(v[u], v[u], s);
    }
    s = wave_sum(s);
    if (lane == 0) to_glb(d.sig)[i] = sqrt(s);
}

// Rank sort of the row norms, truncation rule, discarded weight, status and S.
template <typename TO>
__global__ __launch_bounds__(256) void finish_kernel(const FinDesc* __restrict__ descs)
{
    __shared__ double sig[FIN_MAXR];
    __shared__ double tail[FIN_MAXR + 1];
    __shared__ int perm_s[FIN_MAXR];
    const FinDesc& d = descs[blockIdx.x];
    const int R = d.R;
    const int tid = threadIdx.x;
    for (int i = tid; i < R; i += 256) sig[i] = to_glb(d.sig)[i];
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
        to_glb(d.sig)[j] = sig[perm_s[j]];
        to_glb(d.perm)[j] = perm_s[j];
    }
    __shared__ int kk_s;
    if (tid == 0) {
        const double normA2 = *to_glb(d.normA2);
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
                    // single view: keeping triplet i removes 2 sigma_i u_i^T A v_i - sigma_i^2
                    const double x = d.cross ? sj * sj - to_glb(d.cross)[perm_s[j - 1]] : -sj * sj;
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
        if (info == 0 && d.rot && to_glb(d.rot)[d.max_sweeps - 1] != 0) info = -5;  // sweep cap reached
        if (d.jac_err && *to_glb(d.jac_err) != 0) info = -3;  // the persistent Jacobi gave up waiting
        if (info != -4 && d.sv_flag && *to_glb(d.sv_flag) != 0) info = -6;  // singular co-range system
        kk_s = kk;
        *to_glb(d.w_out) = w;
        *to_glb(d.kkept_out) = kk;
        *to_glb(d.info_out) = info;
    }
    __syncthreads();
    const int kk = kk_s;
    GLB TO* __restrict__ S = (GLB TO*)d.S;
    for (int j = tid; j < d.k; j += 256) S[j] = (j < kk) ? (TO)sig[perm_s[j]] : (TO)0;
}

// Source of output vector j: row perm[j] of X scaled by 1/sigma_j (a column of
// X^T divided by its norm), or row perm[j] of the accumulated rotation P.
struct VecSrc {
    const GLB double* base;
    int64_t ld;
    bool scaled;
};
__device__ __forceinline__ VecSrc vec_src(const FinDesc& d, bool from_p)
{
    return from_p ? VecSrc{to_glb(d.P), d.ldp, false} : VecSrc{to_glb(d.X), d.ldx, true};
}

// Rows j of VT (zero for j >= k_kept): one wave per row, coalesced over the row.
template <typename TO>
__global__ __launch_bounds__(256) void gather_vt_kernel(const FinDesc* __restrict__ descs,
                                                        const int* __restrict__ map, int nprob)
{
    const int2 wi_ = wg_item(map, blockIdx.x);
    const FinDesc& d = descs[wi_.x];
    const int lane = threadIdx.x & 63, j = 4 * wi_.y + (threadIdx.x >> 6);
    if (j >= d.k) return;
    const int n = d.n;
    const bool keep = j < *to_glb(d.kkept_out);
    const VecSrc vs = vec_src(d, d.mode == 2);
    const int src = to_glb(d.perm)[keep ? j : 0];
    const double sj = to_glb(d.sig)[keep ? j : 0];
    const double scale = !keep ? 0.0 : (!vs.scaled ? 1.0 : (sj > 0.0 ? 1.0 / sj : 0.0));
    const GLB double* __restrict__ row = vs.base + (int64_t)src * vs.ld;
    GLB TO* __restrict__ out = (GLB TO*)d.VT + (int64_t)j * d.ldvt;
    for (int t0 = lane; t0 < n; t0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 64 * u;
            v[u] = ld_or0(row, t, keep && t < n);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 64 * u;
            if (t < n) out[t] = (TO)(v[u] * scale);
        }
    }
}

// Columns j of U for the full SVD, through a 64 x 64 LDS transpose so that
// both the reads (rows of the source) and the writes (rows of U) are coalesced.
template <typename TO>
__global__ __launch_bounds__(256) void gather_u_kernel(const FinDesc* __restrict__ descs,
                                                       const int* __restrict__ map, int nprob)
{
    __shared__ double tile[64][65];
    const int2 wi_ = wg_item(map, blockIdx.x);
    const FinDesc& d = descs[wi_.x];
    const int m = d.m, k = d.k;
    const int tiles_j = (k + 63) / 64;
    const int j0 = 64 * (wi_.y % tiles_j), i0 = 64 * (wi_.y / tiles_j);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kk = (int)*to_glb(d.kkept_out);
    const VecSrc vs = vec_src(d, d.mode == 1);
    const int i = i0 + lane;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        const int jj = wave + 4 * r, j = j0 + jj;
        const bool keep = j < kk;
        const int src = to_glb(d.perm)[keep ? j : 0];
        const double sj = to_glb(d.sig)[keep ? j : 0];
        const double scale = !keep ? 0.0 : (!vs.scaled ? 1.0 : (sj > 0.0 ? 1.0 / sj : 0.0));
        tile[jj][lane] = ld_or0(vs.base, (int64_t)src * vs.ld + i, keep && i < m) * scale;
    }
    __syncthreads();
    const int j = j0 + lane;
    GLB TO* __restrict__ U = (GLB TO*)d.U;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        const int ii = wave + 4 * r;
        if (i0 + ii < m && j < k) U[(int64_t)(i0 + ii) * d.ldu + j] = (TO)tile[lane][ii];
    }
}

hipError_t launch_finish(const FinDesc* d, int nprob, const int* norm_map, int norm_total, const int* vt_map,
                         int vt_total, const int* u_map, int u_total, int out_f64, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    if (norm_total > 0) hipLaunchKernelGGL(rownorm_kernel, dim3(norm_total), dim3(256), 0, s, d, norm_map, nprob);
    if (out_f64) {
        hipLaunchKernelGGL(finish_kernel<double>, dim3(nprob), dim3(256), 0, s, d);
        if (vt_total > 0)
            hipLaunchKernelGGL(gather_vt_kernel<double>, dim3(vt_total), dim3(256), 0, s, d, vt_map, nprob);
        if (u_total > 0)
            hipLaunchKernelGGL(gather_u_kernel<double>, dim3(u_total), dim3(256), 0, s, d, u_map, nprob);
    } else {
        hipLaunchKernelGGL(finish_kernel<float>, dim3(nprob), dim3(256), 0, s, d);
        if (vt_total > 0)
            hipLaunchKernelGGL(gather_vt_kernel<float>, dim3(vt_total), dim3(256), 0, s, d, vt_map, nprob);
        if (u_total > 0)
            hipLaunchKernelGGL(gather_u_kernel<float>, dim3(u_total), dim3(256), 0, s, d, u_map, nprob);
    }
    return hipGetLastError();
}

// Canonical signs: for 64 columns of U per workgroup (lane = column, so every
// access is a coalesced row segment), find the entry of largest magnitude
// (lowest row on ties, NaN never chosen), make it positive by flipping the
// column of U and the matching row of VT, and zero the columns >= k_kept.
constexpr int SF_WAVES = 16;
template <typename TO>
__global__ __launch_bounds__(64 * SF_WAVES) void signfix_kernel(const FinDesc* __restrict__ descs,
                                                                const int* __restrict__ map, int nprob)
{
    __shared__ double best_s[SF_WAVES][64];
    __shared__ int idx_s[SF_WAVES][64];
    __shared__ int flip_s[64];
    const int2 wi_ = wg_item(map, blockIdx.x);
    const FinDesc& d = descs[wi_.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = d.m, n = d.n, k = d.k;
    const int j0 = 64 * wi_.y, j = j0 + lane;
    const int kk = (int)*to_glb(d.kkept_out);
    const bool col = j < k, kept = j < kk;
    GLB TO* __restrict__ U = (GLB TO*)d.U;
    GLB TO* __restrict__ VT = (GLB TO*)d.VT;
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i0 = wave; i0 < m; i0 += SF_WAVES * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + SF_WAVES * u;
            const bool ok = kept && i < m;
            v[u] = ok ? fabs((double)ld_or0((const GLB TO*)U, (int64_t)i * d.ldu + j, ok)) : -1.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (v[u] > best) {
                best = v[u];
                bi = i0 + SF_WAVES * u;
            }
        }
    }
    best_s[wave][lane] = best;
    idx_s[wave][lane] = bi;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < SF_WAVES; ++w) {
            const double ob = best_s[w][lane];
            const int oi = idx_s[w][lane];
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        // no finite entry: the column is left as it is
        const bool flip = kept && bi < m && (double)U[(int64_t)(bi < m ? bi : 0) * d.ldu + j] < 0.0;
        flip_s[lane] = flip;
        GLB double* __restrict__ sgn = to_glb(d.sgn);
        if (sgn && col) sgn[j] = !kept ? 0.0 : (flip ? -1.0 : 1.0);
    }
    __syncthreads();
    const bool flip = flip_s[lane];
    if (col && (flip || !kept)) {
        for (int i0 = wave; i0 < m; i0 += SF_WAVES * 8) {
            TO v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + SF_WAVES * u;
                v[u] = ld_or0((const GLB TO*)U, (int64_t)i * d.ldu + j, kept && i < m);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + SF_WAVES * u;
                if (i < m) U[(int64_t)i * d.ldu + j] = kept ? -v[u] : (TO)0;
            }
        }
    }
    // rows of VT: wave w takes rows j0 + w, j0 + w + SF_WAVES, ...; rows past
    // k_kept are zeroed (they are zero already unless V^T came from a product
    // with non-finite factors)
    for (int r = wave; r < 64; r += SF_WAVES) {
        if (j0 + r >= kk && j0 + r < k) {
            GLB TO* __restrict__ zrow = VT + (int64_t)(j0 + r) * d.ldvt;
            for (int x = lane; x < n; x += 64) zrow[x] = (TO)0;
            continue;
        }
        if (!flip_s[r] || j0 + r >= k) continue;
        GLB TO* __restrict__ vrow = VT + (int64_t)(j0 + r) * d.ldvt;
        for (int x0 = lane; x0 < n; x0 += 64 * 8) {
            TO v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = x0 + 64 * u;
                v[u] = ld_or0((const GLB TO*)vrow, x, x < n);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int x = x0 + 64 * u;
                if (x < n) vrow[x] = -v[u];
            }
        }
    }
}

hipError_t launch_signfix(const FinDesc* d, const int* map, int nprob, int total, int out_f64, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    if (out_f64)
        hipLaunchKernelGGL(signfix_kernel<double>, dim3(total), dim3(64 * SF_WAVES), 0, s, d, map, nprob);
    else
        hipLaunchKernelGGL(signfix_kernel<float>, dim3(total), dim3(64 * SF_WAVES), 0, s, d, map, nprob);
    return hipGetLastError();
}

}  // namespace rsvd
