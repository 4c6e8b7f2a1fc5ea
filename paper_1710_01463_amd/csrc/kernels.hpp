// Host-visible kernel descriptors and launchers of librsvd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

// One GEMM of a batched launch:  C (M x N) [+]= op(A) (M x K) * op(X) (K x N)
//   op(A)(i, t) = transA ? A[t*lda + i] : A[i*lda + t]
//   op(X)(t, j) = transX ? X[g(j)*ldx + t] : X[t*ldx + j],  g(j) = gather ? gather[j] : j
//   C written at C[i*ldc + j] (transC = 0) or C[j*ldc + i] (transC = 1).
// skip: when non-null and *skip != 0 the problem is left untouched.
struct GemmDesc {
    const void* A;
    const void* X;
    void* C;
    const int* gather;
    const int* skip;
    int64_t lda, ldx, ldc;
    int M, N, K;
    int transA, transX, transC;
    int accumulate;
    int tiles_n;
    int lower;         // 1: only the tiles on or below the diagonal of C (M == N, square tiles)
};

// Storage kinds of the operands of a GEMM launch and the MFMA used.
enum GemmKind : int {
    GK_F64 = 0,   // FP64 MFMA 16x16x4, operands converted to double on load
    GK_F32 = 1,   // FP32 MFMA 16x16x4, operands converted to float on load
    GK_BF16 = 2,  // BF16 MFMA 16x16x32 (FP32 accumulate), operands rounded to bf16 on load
};

enum Elem : int { E_F64 = 0, E_F32 = 1, E_BF16 = 2 };

// Workgroup output tile of a GEMM launch (256 threads, 2 x 2 waves).
enum GemmTile : int { GT_64x64 = 0, GT_128x64 = 1, GT_64x128 = 2, GT_128x128 = 3 };
constexpr int gemm_tile_m(GemmTile t) { return (t == GT_128x64 || t == GT_128x128) ? 128 : 64; }
constexpr int gemm_tile_n(GemmTile t) { return (t == GT_64x128 || t == GT_128x128) ? 128 : 64; }

// descs: device array of nprob descriptors; tile_begin: the launch's work-item map,
// total_tiles int pairs (problem, tile index), a problem with ceil(M/BM) * ceil(N/BN)
// tiles contributing that many consecutive entries (BM x BN = the launch's GemmTile;
// tiles_n of every descriptor must be ceil(N/BN)).  Every "*_begin" argument of
// the launchers below is such a map over that launch's items.
// gather: the descriptors carry gather arrays (FP64 operands only; tile forced to 64 x 64).
hipError_t launch_gemm(GemmKind kind, Elem ea, Elem ex, Elem ec, GemmTile tile, bool gather, const GemmDesc* descs,
                       const int* tile_begin, int nprob, int total_tiles, hipStream_t stream);

// ---------------------------------------------------------------- QR (orthonormalisation)
// One orthonormalisation of a (rows x l) matrix M into Qout (rows x l, FP64),
// by Cholesky QR (Gram G = M^T M, G = L L^T, Qout = M L^-T) with a Householder
// fallback.  Buffers are per problem.
struct QrDesc {
    const void* Min;   // rows x l, row-major, ld = l
    double* Qout;      // rows x l, ld = l
    double* G;         // l x l Gram
    double* L;         // l x l Cholesky factor (lower)
    double* D;         // ceil(l/16) inverses of the 16 x 16 diagonal blocks of L
    int* flag;         // breakdown flag: set to 1 when Cholesky QR cannot be used
    int rows, l;
    int min_elem;      // Elem of Min
    int pad_;
};

// Cholesky of G into L and the diagonal-block inverses D; sets *flag on
// breakdown.  max_l: largest l of the batch.  Skips problems with Qout ==
// nullptr or *flag already set.
constexpr int CHOL_MAX_L = 1024;
hipError_t launch_chol(const QrDesc* d, int nprob, int max_l, hipStream_t s);
// Qout = src L^-T, src = Min (from_min = 1) or Qout (from_min = 0, in place);
// row_begin: item map over the ceil(rows / 16) row blocks of every problem.
// src_elem: element type of Min when from_min (E_F64 or E_F32).
hipError_t launch_trsm(const QrDesc* d, const int* row_begin, int nprob, int total_blocks, int from_min,
                       int src_elem, int max_l, hipStream_t s);
// Raises the dynamic-LDS limit of the Cholesky kernel.
hipError_t init_qr_kernels();
// Householder QR of Min into Qout for the problems whose flag is set.
hipError_t launch_householder(const QrDesc* d, int nprob, hipStream_t s);
// The same QR by panels of 16 columns (compact WY): 2 ceil(max_l / 16) launches,
// the trailing updates spread over 64-column tiles.  Uses G (the panels' T
// factors) and D (tau, beta) of each descriptor as scratch.  Every problem's
// rows must be <= householder_blocked_rows_max() (hipErrorInvalidValue).
hipError_t launch_householder_blocked(const QrDesc* d, int nprob, int max_l, int max_rows, hipStream_t s);
int householder_blocked_rows_max();
// Adjoint helpers on QrDesc fields: L holds R (l x l, row-major) = Q^T M of a
// stage; tri_prep zeroes its strictly lower part and writes the diagonal-block
// inverses of L = R^T into D.  trsm_upper replaces Qout (rows x l) by
// Qout R^-T.  Problems with Qout == nullptr are skipped.
hipError_t launch_tri_prep(const QrDesc* d, int nprob, int max_l, hipStream_t s);
hipError_t launch_trsm_upper(const QrDesc* d, const int* row_begin, int nprob, int total_blocks, int max_l,
                             hipStream_t s);

// ---------------------------------------------------------------- block one-sided Jacobi
// Orthogonalises the R rows of X (R x C, row-major, R <= C) by left rotations,
// accumulating them in P (R x R).  Rows are grouped in blocks of 16; the nb
// blocks (nb even) are paired by the round-robin schedule, one round per
// launch.
struct JacDesc {
    double* X;
    double* P;
    int* rot;          // per-sweep "rotated" flags, max_sweeps entries
    int* stats;        // [0] block pairs whose Gram was formed, [1] rotations applied,
                       // [2] tasks finished and [3] converged (persistent launch)
    int64_t ldx, ldp;
    int R, C, nb;
    int skip0;         // 1: block nb - 1 is all padding and its pair is not launched
    int cross_rounds;  // 1: rounds >= 2 of a sweep rotate only the pairs across the two blocks
    int pad_;
    double tol;
};
constexpr int JAC_B = 16;
// variant: 0 streams the column chunks of every pair (any size); k > 0 keeps
// the pair's rows in registers, for problems whose row lengths fit the
// variant (jacobi_resident_variant of the largest chunk counts, JAC_CHUNK
// columns per chunk, X and P counted apart).
constexpr int JAC_CHUNK = 128;
int jacobi_resident_variant(int max_x_chunks, int max_p_chunks);
hipError_t launch_jacobi_round(const JacDesc* d, const int* pair_begin, int nprob, int total_pairs,
                               int sweep, int round, int variant, hipStream_t s);
// Every round of every sweep in one launch of `grid` workgroups that take
// block-pair tasks from a queue (sched[0], zero before the launch) and wait
// only on their own problem's earlier rounds (stats[2], stats[3] zero before
// the launch).  sched[1] (zero before the launch) is set when a wait exceeds
// JAC_SPIN_LIMIT polls; every workgroup then leaves.
constexpr int JAC_SPIN_LIMIT = 1 << 22;
hipError_t launch_jacobi_persistent(const JacDesc* d, const int* pair_map, int total_pairs, int rounds_per_sweep,
                                    int max_sweeps, int* sched, int grid, int variant, hipStream_t s);
// Workgroups of the persistent Jacobi kernel that fit on one compute unit.
int jacobi_persistent_blocks_per_cu(int variant);

// ---------------------------------------------------------------- finishing
// mode 0: RSVD (X = B rows, w from ||A||^2 - sum), mode 1: full SVD with X = A,
// mode 2: full SVD with X = A^T.  Writes sigma, perm, S, VT (mode 0,1) or U
// (mode 2 from X; mode 1 from P), discarded weight, k_kept and info.
struct FinDesc {
    const double* X;
    const double* P;
    double* sig;       // R
    int* perm;         // R
    const double* normA2;
    const int* rot;    // Jacobi flags, to detect the sweep cap
    const int* jac_err; // error flag of the persistent Jacobi launch (may be null)
    const double* cross; // single-view plans: 2 sigma_i u_i^T A v_i per Jacobi row (else null)
    const int* sv_flag; // single-view plans: breakdown flag of the co-range system (else null)
    void* U;
    void* S;
    void* VT;
    double* sgn;       // k: sign applied to triplet j (+-1), 0 beyond k_kept; may be null
    double* w_out;
    int64_t* kkept_out;
    int* info_out;
    int64_t ldx, ldp, ldu, ldvt;
    int R, C, m, n, k;
    int mode;
    int max_sweeps;
    int pad_;
    double delta;
};
// Row norms (item map over groups of 4 rows of X), rank sort and truncation
// (one workgroup per problem), then the gathers of VT (item map over groups of
// 4 rows of VT) and, for the full SVD, of U (item map over 64 x 64 tiles of U).
hipError_t launch_finish(const FinDesc* d, int nprob, const int* norm_map, int norm_total, const int* vt_map,
                         int vt_total, const int* u_map, int u_total, int out_f64, hipStream_t s);
// Zero columns >= k_kept of U and make the largest-magnitude entry of every kept
// left vector positive (flipping the matching row of VT).  map: item map over
// groups of 64 columns.
hipError_t launch_signfix(const FinDesc* d, const int* map, int nprob, int total, int out_f64, hipStream_t s);

// ---------------------------------------------------------------- sector post-selection
// Keep the chi largest singular values over all problems of a plan (the
// outputs its FinDesc table points to): chi_s[b] (device) receives how many
// problem b keeps; the rest are dropped (weight added to w, zero-filled,
// k_kept lowered).  At most SELECT_MAX_SECTORS problems.
constexpr int SELECT_MAX_SECTORS = 8192;
// max_candidates: sum over problems of k (bounds sum k_kept).
hipError_t launch_postselect(const FinDesc* d, int nprob, int64_t max_candidates, int64_t chi, int64_t* chi_s,
                             int out_f64, hipStream_t s);
hipError_t init_select_kernels();

// ---------------------------------------------------------------- staging
// ||A||_F^2 (deterministic two-level FP64 reduction) and optional cast of A.
struct StageDesc {
    const void* A;
    void* Acast;       // may be null
    double* partial;   // one per row chunk
    double* normA2;
    int64_t lda;
    int m, n;
    int a_elem, cast_elem;
    int chunk_begin, nchunks;
};
constexpr int STAGE_ROWS = 8;
hipError_t launch_stage(const StageDesc* d, const int* chunk_begin, int nprob, int total_chunks,
                        hipStream_t s);
hipError_t launch_stage_final(const StageDesc* d, int nprob, hipStream_t s);

// Gaussian test matrix Omega (n x l) of every problem, element type elem.
// complex_embed: Omega is the real 2n x 2l embedding [[Wr, -Wi], [Wi, Wr]] of
// the n x l circular complex Gaussian W of the seed (counter (i, j, 1, 0)),
// n and l being the complex sizes; the item map then covers n l entries.
struct OmegaDesc {
    void* Om;
    uint64_t seed;
    int n, l;
    int elem;
    int complex_embed;
};

// Real embedding At = [[Ar, -Ai], [Ai, Ar]] (2m x 2n, FP64, ld ldt) of a complex
// m x n matrix A stored interleaved (re, im) with leading dimension lda in
// complex elements.  Item map over ceil(m n / 256) blocks per problem.
struct CEmbedDesc {
    const double* A;
    double* At;
    int64_t lda, ldt;
    int m, n;
};
hipError_t launch_embed_complex(const CEmbedDesc* d, const int* blk_begin, int nprob, int total_blocks,
                                hipStream_t s);

// Complex triplets from the real SVD of the embedding (the real singular
// values come in pairs, sigma_j twice, with the vectors of [u_r; u_i] and of
// i u): per problem, the 2k leading real triplets of the embedded problem
// (Ur 2m x 2k, Sr 2k sorted, VTr 2k x 2n) give k complex ones (u = x[:m] +
// i x[m:], v likewise from the right vector), made orthonormal in the complex
// inner product against the kept vectors whose values lie within
// CPLX_MIX_REL sigma_1 (which drops the partner of each kept vector and
// resolves degenerate clusters).  Then the truncation rule on the complex
// values, the discarded weight, the canonical phases (largest-modulus entry
// of u real and positive, the row of V^H taking the conjugate phase) and the
// interleaved complex outputs U (m x k, ldu), S, VT = V^H (k x n, ldvt).
constexpr double CPLX_MIX_REL = 1e-4;
struct CFinDesc {
    const double* Ur;     // 2m x 2k, ld 2k
    const double* Sr;     // 2k
    const double* VTr;    // 2k x 2n, ld 2n
    const double* normA2; // ||At||_F^2 = 2 ||A||_F^2
    const double* wr;     // the embedded problem's discarded weight (full SVD: its tail beyond 2k)
    const int* info_in;   // the embedded problem's status
    double* U;            // complex m x k (ldu)
    double* S;            // k
    double* VT;           // complex k x n (ldvt)
    double* sig;          // k: the complex singular values
    double* w_out;
    int64_t* kkept_out;
    int* info_out;
    int64_t ldu, ldvt;
    int m, n, k;
    int full;             // 1: full-SVD truncation (w is the tail sum), 0: RSVD (||A||^2 - sum)
    double delta;
};
hipError_t launch_complex_finish(const CFinDesc* d, int nprob, const int* col_map, int col_total, hipStream_t s);
hipError_t launch_omega(const OmegaDesc* d, const int* blk_begin, int nprob, int total_blocks,
                        hipStream_t s);

hipError_t launch_philox_words(const uint32_t* in, uint32_t* out, int64_t count, hipStream_t s);

// Copies `bytes` host bytes from src to device memory dst on stream s, in
// chunks of UPLOAD_CHUNK_BYTES passed by value as kernel arguments (no
// staging allocation; src may be reused as soon as the call returns).
constexpr int UPLOAD_CHUNK_BYTES = 2048;
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s);

// Fill helpers (graph-safe replacements for memset).
hipError_t launch_fill_i32(int* p, int value, int64_t count, hipStream_t s);
// Copy A (m x n, lda, any elem) into X as FP64, transposed or not, for the full SVD.
struct CopyDesc {
    const void* A;
    double* X;
    int64_t lda, ldx;
    int m, n;
    int a_elem, transpose;
};
hipError_t launch_copy_f64(const CopyDesc* d, const int* blk_begin, int nprob, int total_blocks,
                           hipStream_t s);
// P = identity (R x R) for every problem.
struct EyeDesc {
    double* P;
    int64_t ldp;
    int R;
    int pad_;
};
hipError_t launch_eye(const EyeDesc* d, const int* blk_begin, int nprob, int total_blocks, hipStream_t s);

// out[i] = alpha * sum_j X[i][j] Y[i][j] for the rows i < rows (row-major,
// leading dimensions ldx, ldy); item map over groups of 4 rows, one wave per row.
struct RowDotDesc {
    const double* X;
    const double* Y;
    double* out;
    int64_t ldx, ldy;
    int rows, cols;
    double alpha;
};
hipError_t launch_rowdot(const RowDotDesc* d, const int* blk_begin, int nprob, int total_blocks, hipStream_t s);

// ---------------------------------------------------------------- adjoint
// Elementwise steps of the reverse pass of one RSVD (cotangent staging, the
// SVD-adjoint core matrix, the symmetrisation of the QR adjoint).  Row-major
// FP64 buffers unless stated.
struct BwDesc {
    const void* dU;     // m x k (ldu), cotangent element type
    const void* dS;     // k
    const void* dVT;    // k x n (ldvt)
    const double* X;    // rotated B, l x n (ld n): row perm[j] = sigma_j v_j^T
    const double* P;    // accumulated rotations, l x l: row perm[j] = u_j^T (of B)
    const double* sig;  // l, sorted descending
    const int* perm;    // l
    const double* sgn;  // k, from the forward's sign fix (0 beyond k_kept)
    double* Ub;         // m x l   cotangent of Q Utilde (signs applied, zero beyond k_kept)
    double* Vbt;        // l x n   cotangent of Vtilde^T; scaled in place to Sigma^-1 Vbar^T
    double* Vts;        // l x n   sorted Vtilde^T
    double* Ut;         // l x l   sorted Utilde
    double* sb;         // l       cotangent of sigma
    const double* EU;   // l x l   Utilde^T Utilde_bar
    const double* EV;   // l x l   Vtilde^T Vbar
    double* Kp;         // l x l   core matrix
    const double* C;    // l x l   Qbar^T Q of a stage
    double* S;          // l x l   -copyltu(C)
    int64_t ldu, ldvt;
    int m, n, l, k;
    int elem;           // Elem of dU, dS, dVT
    int pad_;
    double broad;       // Lorentzian broadening eps = broad * sigma_1^4
};
// blk_begin: item map over ceil(bw_*_elems / BW_ELEMS_PER_BLOCK) blocks per problem.
int64_t bw_prep_elems(int m, int n, int l);
int64_t bw_core_elems(int n, int l);
int64_t bw_sym_elems(int l);
constexpr int BW_ELEMS_PER_BLOCK = 1024;
hipError_t launch_bw_prep(const BwDesc* d, const int* blk_begin, int nprob, int total, int cot_f64,
                          hipStream_t s);
hipError_t launch_bw_core(const BwDesc* d, const int* blk_begin, int nprob, int total, hipStream_t s);
hipError_t launch_bw_sym(const BwDesc* d, const int* blk_begin, int nprob, int total, hipStream_t s);

}  // namespace rsvd
