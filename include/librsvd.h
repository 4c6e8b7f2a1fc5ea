/*
 * librsvd -- randomized truncated SVD on one AMD MI355X (gfx950).
 *
 * The method is the randomized SVD of Kohn et al., "Probabilistic low-rank
 * factorization accelerates tensor network simulations of critical quantum
 * many-body ground states", Sec. II.B, Alg. RSVD: a Gaussian test matrix
 * Omega (n x l), the sample Y = (A A^T)^q A Omega formed as a power iteration
 * with an orthonormalisation after every product, Q = orthonormal basis of Y,
 * the SVD of B = Q^T A, left vectors Q Utilde, right vectors Vtilde.  The
 * deterministic comparison is Alg. TSVD of Sec. II.A (full SVD, then keep the
 * leading triplets).
 *
 * Conventions shared by every entry point
 *  - Matrices are row-major with an explicit leading dimension in elements.
 *  - All matrix, vector and scalar-output pointers are DEVICE pointers owned
 *    by the caller; the library never frees them.  Library-owned device
 *    memory lives only inside an rsvd_plan_t (workspace, descriptors, graph),
 *    in the small plan cache of the one-shot calls, or in the static scratch
 *    array of rsvd_truncate_noalloc.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).
 *  - k is clamped to min(m, n) (small symmetry sectors routinely ask for more
 *    triplets than the block has).  l = min(k + p, m, n).
 *  - Outputs: U is m x k (ldu >= k), S has k entries, VT is k x n (ldvt >= n).
 *    S is sorted in descending order.  Only the first k_kept triplets are
 *    filled; columns k_kept..k-1 of U, rows k_kept..k-1 of VT and entries
 *    k_kept..k-1 of S are zero.
 *  - Sign convention: the entry of largest magnitude of every kept column of
 *    U is positive (lowest row index on ties); VT follows.
 *  - Truncation (paper Sec. II.A measures the truncation error in the
 *    Frobenius norm): w(k') = discarded squared Frobenius weight when k'
 *    triplets are kept.  k_kept = k when delta_trunc == 0, otherwise the
 *    smallest k' >= 1 with w(k') <= delta_trunc * ||A||_F^2, capped at k.
 *    ||A||_F = 0 gives k_kept = 0 and w = 0.  The reported discarded weight
 *    is the absolute w(k_kept), in FP64.  For the RSVD it is
 *    ||A||_F^2 - sum_{j<=k_kept} sigma_j^2, which equals ||A - U S VT||_F^2;
 *    for the full SVD it is the tail sum of the discarded sigma_j^2.
 *  - Gaussian test matrix: entry (i, j) of Omega for seed s is the
 *    Box-Muller normal built from Philox4x32-10 with key (s mod 2^32, s >> 32)
 *    and counter (i/2, j, 0, 0): u1 = 1 - ((w0:w1) >> 11) 2^-53,
 *    u2 = ((w2:w3) >> 11) 2^-53, r = sqrt(-2 ln u1), r cos(2 pi u2) for even
 *    i and r sin(2 pi u2) for odd i.  A problem's Omega depends only on its
 *    seed, never on its position in a batch.
 *
 * Errors: every entry point returns an rsvd_status_t and never throws.
 * RSVD_ERR_INVALID leaves all outputs untouched.  rsvd_last_error() returns a
 * thread-local description of the last failure.
 */
#ifndef LIBRSVD_H
#define LIBRSVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSVD_OK = 0,
    RSVD_ERR_INVALID = -1,   /* bad argument: sizes, leading dimensions, null pointers, delta < 0 or NaN */
    RSVD_ERR_ALLOC = -2,     /* device or pinned-host allocation failed */
    RSVD_ERR_HIP = -3,       /* a HIP runtime call failed */
    RSVD_ERR_NONFINITE = -4, /* ||A||_F^2 is not finite (NaN or Inf in A); outputs zero, k_kept = 0 */
    RSVD_ERR_NOCONV = -5,    /* Jacobi sweep cap reached; outputs are still filled */
    RSVD_ERR_SINGULAR = -6   /* single-view plans: Psi Q numerically rank deficient; outputs filled, unreliable */
} rsvd_status_t;

/* Storage type of A, U, S and VT. */
typedef enum { RSVD_F64 = 0, RSVD_F32 = 1 } rsvd_dtype_t;

/* Arithmetic of the sketch and power-iteration products (Y = A Omega, A^T Q,
 * A Z).  The Gram matrices, Cholesky factors, the projection B = Q^T A (from
 * the stored A, upcast exactly), the small Jacobi SVD and the back-projection
 * always run in FP64.  BF16 rounds A, Omega and Q to bf16 and accumulates in
 * FP32; F32 rounds them to FP32 and accumulates in FP32. */
typedef enum { RSVD_PREC_F64 = 0, RSVD_PREC_F32 = 1, RSVD_PREC_BF16 = 2 } rsvd_prec_t;

/*
 * rsvd_truncate -- one randomized truncated SVD (Alg. RSVD, Sec. II.B).
 *   A        device, m x n, leading dimension lda >= n, dtype dt
 *   k, p, q  target rank (>= 1), oversampling (>= 0), power iterations (>= 0)
 *   seed     Gaussian test-matrix seed (see conventions)
 *   delta_trunc  relative discarded-weight threshold (>= 0; 0 disables)
 *   prec     arithmetic of the sketch / power products
 *   U, S, VT device outputs (dtype dt), see conventions
 *   discarded_weight  device double[1]; k_kept  device int64_t[1]
 * Blocking: returns after the factorisation has completed on the stream, so
 * that RSVD_ERR_NONFINITE / RSVD_ERR_NOCONV can be reported.  Plans are cached
 * per shape, so repeated calls of one shape reuse their workspace and graph.
 */
int rsvd_truncate(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k,
                  int64_t p, int64_t q, uint64_t seed, double delta_trunc, rsvd_prec_t prec, void* U,
                  int64_t ldu, void* S, void* VT, int64_t ldvt, double* discarded_weight,
                  int64_t* k_kept, void* stream);

/*
 * rsvd_truncate_noalloc -- rsvd_truncate for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, arithmetic and results
 * as rsvd_truncate (bit for bit: the same kernels run in the same order),
 * with these differences:
 *  - Nothing is allocated.  The workspace and the descriptor tables of the
 *    call live in one static device array of RSVD_NOALLOC_SCRATCH_BYTES per
 *    GPU, held by the library from load until the process ends.  A problem
 *    whose workspace and descriptors do not fit returns RSVD_ERR_INVALID
 *    before any device work (512 x 512 at k + p = 272 needs about 10 MiB;
 *    2048 x 2048 at k + p = 256 about 33 MiB).
 *  - Asynchronous on stream: no graph, no plan cache, no synchronisation.
 *    info (device int, may be NULL) receives the status of the factorisation
 *    (RSVD_OK, RSVD_ERR_NONFINITE or RSVD_ERR_NOCONV); the return value only
 *    reports argument and launch errors.
 *  - Every call on one GPU shares that GPU's scratch array, which keeps the
 *    last call's contents.  Calls whose executions overlap on one GPU (on
 *    different streams or from different threads) race and must be ordered
 *    by the caller.  The descriptors are passed by value in the call's
 *    launches, so a graph captured around one call replays that call.
 */
#define RSVD_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
int rsvd_truncate_noalloc(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k,
                          int64_t p, int64_t q, uint64_t seed, double delta_trunc, rsvd_prec_t prec, void* U,
                          int64_t ldu, void* S, void* VT, int64_t ldvt, double* discarded_weight,
                          int64_t* k_kept, int* info, void* stream);

/*
 * rsvd_truncate_adaptive -- fixed-error truncation with an adaptive rank (the
 * outlook of Sec. V: let the error target, not a rank guess, drive the
 * RSVD).  Runs rsvd_truncate with k = k0, 2 k0, 4 k0, ... (capped at
 * kcap = min(k_max, m, n)), the same seed throughout (so each sketch extends
 * the previous one by new columns of Omega), until the discarded-weight cut
 * binds inside the sketch (k_kept < k) or k reaches kcap.  Since
 * w = ||A - U S V^T||_F^2 exactly for the computed factorisation, the result
 * meets w <= delta_trunc ||A||_F^2 whenever k_kept < k; at the cap it is the
 * rank-kcap truncation (exact when kcap = min(m, n)).
 *   k0, k_max    1 <= k0 <= k_max
 *   delta_trunc  finite, > 0 (required: it is the stopping rule)
 *   U, S, VT     sized for kcap: U m x kcap (ldu >= kcap), S kcap, VT kcap x n;
 *                triplets from k_kept on are zero
 *   attempts     host int*, receives the number of RSVDs run (may be NULL)
 * Other arguments as rsvd_truncate.  Each new k is a new cached plan shape.
 * Blocking.  Returns RSVD_ERR_INVALID for bad sizes, delta_trunc <= 0 or
 * null outputs, else the status of the last RSVD run. */
int rsvd_truncate_adaptive(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k0,
                           int64_t k_max, int64_t p, int64_t q, uint64_t seed, double delta_trunc,
                           rsvd_prec_t prec, void* U, int64_t ldu, void* S, void* VT, int64_t ldvt,
                           double* discarded_weight, int64_t* k_kept, int* attempts, void* stream);

/*
 * fullsvd_truncate -- deterministic truncation by the full SVD (Alg. TSVD,
 * Sec. II.A), computed by block one-sided Jacobi in FP64 on A (m <= n) or A^T
 * (m > n).  Arguments as for rsvd_truncate.  Blocking, cached like it.
 */
int fullsvd_truncate(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k,
                     double delta_trunc, void* U, int64_t ldu, void* S, void* VT, int64_t ldvt,
                     double* discarded_weight, int64_t* k_kept, void* stream);

/*
 * rsvd_gaussian -- the Gaussian test matrix Omega (n x l, row-major, FP64,
 * device output) that rsvd_truncate draws for this seed (Alg. RSVD step 1,
 * layout in the conventions above).  Blocking.  Lets callers reproduce or
 * differentiate with the exact test matrix of a factorisation.
 */
int rsvd_gaussian(uint64_t seed, int64_t n, int64_t l, double* omega, void* stream);

/*
 * rsvd_philox4x32_10 -- raw Philox4x32-10 words of the device generator:
 * in holds count groups of 6 words (counter c0..c3, key k0, k1), out receives
 * count groups of 4 output words.  Both device pointers.  Asynchronous.
 */
int rsvd_philox4x32_10(const uint32_t* in, uint32_t* out, int64_t count, void* stream);

/* ---------------------------------------------------------------- batches
 * A plan holds many independent problems of arbitrary, uneven sizes (for
 * example the symmetry sectors of one compression, paper Sec. III.A) and runs
 * them all with one batched launch per phase, optionally captured once into a
 * HIP graph so that an execute is one graph launch. */
typedef struct {
    int64_t m, n, lda, k, p, q;
    uint64_t seed;
    double delta_trunc;
    int64_t ldu;  /* 0 means k (after clamping) */
    int64_t ldvt; /* 0 means n */
} rsvd_problem_t;

typedef struct rsvd_plan rsvd_plan_t;

#define RSVD_PLAN_FULLSVD 1u /* the plan runs fullsvd_truncate instead of the RSVD (p, q, seed ignored) */
#define RSVD_PLAN_GRAPH 2u   /* capture the launch sequence into a HIP graph on first execute */
#define RSVD_PLAN_SAVE 4u    /* keep every intermediate basis and the adjoint workspace for rsvd_plan_backward */
#define RSVD_PLAN_NO_REFINE 8u /* form B = Q^T A in the sketch precision instead of FP64 (accuracy study) */
#define RSVD_PLAN_TUNE 16u     /* choose the workgroup tile of every forward product by measurement (below) */
/* Run the Jacobi SVD as one launch per round of its schedule.  Without this
 * flag, plans whose rounds have at most 64 block pairs over all problems (small
 * problems or batches, whose rounds cannot fill the GPU) run the whole Jacobi
 * phase as one persistent launch whose workgroups take the same block-pair
 * tasks from a queue and wait only for their own problem's previous round;
 * both forms compute the same rotations in the same order per problem and
 * give bit-identical results.  A wait of the persistent launch that exceeds
 * its bound (a fault, not an expected case) makes every problem of that
 * execute report RSVD_ERR_HIP in info. */
#define RSVD_PLAN_ROUND_LAUNCHES 32u
/* Block-Krylov variant (the faster-converging power scheme named in the
 * outlook, Sec. V): the small SVD is taken over the whole block Krylov space
 * span{A Omega, (A A^T) A Omega, ..., (A A^T)^q A Omega} instead of its last
 * block.  The range finder is unchanged; the q + 1 orthonormal bases of the
 * stages that multiply by A are placed side by side, the first
 * L = min((k + p)(q + 1), m, n) columns are orthonormalised (Cholesky QR
 * twice, Householder on breakdown), and B = Q^T A (L x n), its SVD, the
 * truncation and U = Q Utilde follow as for the RSVD.  With q = 0 this is the
 * RSVD.  Truncation, outputs and discarded weight as for the RSVD (w equals
 * ||A - U S V^T||_F^2).  Not with RSVD_PLAN_FULLSVD or RSVD_PLAN_SAVE; L must
 * be <= 1024 (RSVD_ERR_INVALID otherwise). */
#define RSVD_PLAN_BLOCK_KRYLOV 64u
/* Complex matrices (the paper's simulations run in complex double, Sec. IV):
 * A, U and VT hold complex double, interleaved (re, im), with leading
 * dimensions lda, ldu, ldvt counted in complex elements; S holds real
 * doubles; dtype must be RSVD_F64.  The method is Alg. RSVD (or Alg. TSVD
 * with RSVD_PLAN_FULLSVD) with Hermitian transposes: Y = A Omega with a
 * circular complex Gaussian Omega (entry (i, j) = (x + i y) / sqrt(2) with x, y
 * the Box-Muller pair of the Philox4x32-10 words of counter (i, j, 1, 0) under
 * the seed's key), W = A^H Q, B = Q^H A, U = Q Utilde, VT = V^H.  Canonical
 * phases: the entry of largest modulus of each kept column of U (lowest row
 * on ties) is real and positive, the matching row of VT taking the conjugate
 * phase.  Truncation and discarded weight as for real problems.  Computed on
 * the real embedding [[Ar, -Ai], [Ai, Ar]] (2m x 2n, whose singular values are
 * those of A, twice): the product, orthonormalisation and Jacobi kernels of
 * the real path at twice the sizes, so the limits are those of the real path
 * at 2m x 2n, rank 2k and oversampling 2p (min(k + p, m, n) <= 512; full SVD
 * min(m, n) <= 1024).  Not with RSVD_PLAN_SAVE, RSVD_PLAN_TUNE (the shape
 * heuristic picks the tiles) or rsvd_plan_postselect. */
#define RSVD_PLAN_COMPLEX 128u
/* Blocked Householder fallback: when a Cholesky QR breaks down (a pivot below
 * 1e-13 of its diagonal entry, i.e. a basis too ill-conditioned for the Gram
 * matrix), the problem's basis is re-orthonormalised by Householder QR.  By
 * default the plan takes the blocked form (panels of 16 columns in compact WY
 * form, the trailing updates as FP64 MFMA products spread over many
 * workgroups; two launches per panel) when max(m, n) (k + p)^2 of some problem
 * is at least 2^27, and the one-workgroup-per-problem form otherwise (one
 * launch; cheaper when no problem breaks down).  This flag asks for the
 * blocked form for every size.  Both give Q with diag(R) >= 0 and agree to
 * rounding.  The blocked form needs max(m, n) <= 2048 for every problem and is
 * not used otherwise. */
#define RSVD_PLAN_BLOCKED_QR 256u
/* Single-view variant (the one-pass scheme named in the outlook, Sec. V, after
 * Tropp, Yurtsever, Udell and Cevher): A is sketched once from both sides and
 * the small matrix is recovered from the sketches alone.  With l = min(k + p,
 * m, n) and s = min(2 l + 1, m):
 *   Omega = the n x l Gaussian of the seed (as for the RSVD), Psi = the
 *   transpose of the m x s Gaussian of the seed with its top bit flipped
 *   (seed ^ 2^63, an independent Philox key);
 *   Y = A Omega (the plan's sketch precision), W = Psi A (FP64);
 *   Q = orth(Y) (Cholesky QR twice, Householder on breakdown);
 *   X = (Psi Q)^+ W (FP64; from the normal equations of Psi Q, whose
 *   condition number is about (sqrt(s) + sqrt(l)) / (sqrt(s) - sqrt(l)) for a
 *   Gaussian Psi);
 *   X = Utilde S V^T by the Jacobi of the RSVD, U = Q Utilde, canonical signs.
 * q is ignored.  Q X is not a projection of A, so the discarded weight is the
 * true error ||A - U S V^T||_F^2 of the kept triplets, evaluated from
 * u_i^T A v_i by one more product with A (the truncation rule needs it): w =
 * ||A||^2 - sum over kept i of (2 sigma_i u_i^T A v_i - sigma_i^2).  k_kept is
 * the smallest k' >= 1 whose w is at most delta ||A||_F^2, at most k.  info
 * RSVD_ERR_SINGULAR when the Cholesky factorisation of (Psi Q)^T (Psi Q)
 * breaks down.  Not with RSVD_PLAN_FULLSVD, RSVD_PLAN_SAVE,
 * RSVD_PLAN_BLOCK_KRYLOV, RSVD_PLAN_COMPLEX or rsvd_plan_postselect. */
#define RSVD_PLAN_SINGLE_VIEW 512u
/* FP64 final power step for mixed-precision plans (RSVD_PREC_F32 or
 * RSVD_PREC_BF16): the last power iteration, W = A^T Q and Y = A Z with their
 * orthonormalisations, runs in FP64 from the stored A, so only the earlier
 * steps use the sketch precision.  The range basis then carries the sketch
 * precision's rounding only through what the last FP64 step does not damp:
 * about a factor (sigma_{l+1} / sigma_k)^2 less on decaying spectra, nothing
 * on nearly flat ones.  The singular values of FP32-output plans sit at
 * their own FP32 rounding either way (the sketch rounding reaches them only
 * through incoherent sums, far below an FP32 ulp), so there the option moves
 * the bases only.  Every problem of the plan must have the same q >= 1.
 * Not with RSVD_PLAN_SAVE, RSVD_PLAN_BLOCK_KRYLOV, RSVD_PLAN_SINGLE_VIEW or
 * RSVD_PLAN_FULLSVD; no effect on FP64 plans. */
#define RSVD_PLAN_FP64_FINAL 1024u

/* Validates the problems, sizes and allocates the plan's device workspace.
 * Returns RSVD_ERR_INVALID for bad problem descriptions. */
int rsvd_plan_create(const rsvd_problem_t* probs, int64_t batch, rsvd_dtype_t dt, rsvd_prec_t prec,
                     unsigned flags, rsvd_plan_t** plan);

/* Runs every problem of the plan, asynchronously on stream.
 *   A, U, S, VT  host arrays of batch device pointers (dtype of the plan)
 *   discarded_weight  device double[batch]; k_kept device int64_t[batch];
 *   info  device int[batch] receiving each problem's status (RSVD_OK,
 *         RSVD_ERR_NONFINITE or RSVD_ERR_NOCONV).
 * The pointer arrays are read during the call; the device buffers must stay
 * valid until the stream reaches the end of the launch.  Returns RSVD_OK or a
 * launch-level error. */
int rsvd_plan_execute(rsvd_plan_t* plan, const void* const* A, void* const* U, void* const* S,
                      void* const* VT, double* discarded_weight, int64_t* k_kept, int* info,
                      void* stream);

/* Phases reported by rsvd_plan_profile. */
enum {
    RSVD_PHASE_STAGE = 0,      /* ||A||_F^2 and the low-precision copy of A */
    RSVD_PHASE_OMEGA = 1,      /* Gaussian test matrices */
    RSVD_PHASE_SKETCH = 2,     /* Y = A Omega, A^T Q, A Z */
    RSVD_PHASE_GRAM = 3,       /* Gram matrices of the Cholesky QR */
    RSVD_PHASE_CHOL = 4,       /* Cholesky factorisations */
    RSVD_PHASE_TRSM = 5,       /* Q = M L^-T */
    RSVD_PHASE_HOUSEHOLDER = 6,
    RSVD_PHASE_PROJECT = 7,    /* B = Q^T A */
    RSVD_PHASE_JACOBI = 8,     /* block one-sided Jacobi rounds */
    RSVD_PHASE_FINISH = 9,     /* norms, sort, truncation */
    RSVD_PHASE_BACKPROJ = 10,  /* U = Q Utilde */
    RSVD_PHASE_SIGNFIX = 11,
    RSVD_PHASE_OTHER = 12,     /* fills, copies */
    RSVD_PHASE_BW_GEMM = 13,   /* products of the reverse pass (rsvd_plan_backward) */
    RSVD_PHASE_BW_SMALL = 14,  /* cotangent staging, adjoint core, triangular solves of the reverse pass */
    RSVD_NUM_PHASES = 15
};

/* rsvd_plan_profile -- one execute run without the graph, with HIP events
 * around every launch on stream.  For each phase c < ncat: ms[c] = summed
 * kernel time, launches[c] = number of launches, flops[c] = algorithmic FLOPs
 * (GEMMs: 2 M N K per problem; Jacobi: 2 b^2 C for every block-pair Gram
 * formed plus 2 b^2 (C + R) for every rotation applied, b = rows per block
 * pair (32); other phases 0).  Arguments otherwise as rsvd_plan_execute.  Blocking. */
int rsvd_plan_profile(rsvd_plan_t* plan, const void* const* A, void* const* U, void* const* S,
                      void* const* VT, double* discarded_weight, int64_t* k_kept, int* info,
                      double* ms, int64_t* launches, double* flops, int ncat, void* stream);

/* rsvd_plan_backward -- reverse-mode derivative of the most recent
 * rsvd_plan_execute of a plan created with RSVD_PLAN_SAVE (RSVD plans only).
 * The paper's method (Sec. II.B, Alg. RSVD) is differentiated with the Gaussian
 * test matrix held fixed (it is a function of the seed only): the standard
 * adjoint of the SVD of B = Q^T A, the thin-QR adjoint of every
 * orthonormalisation, and the product rule through every GEMM.  For each
 * problem it writes
 *     dA = gradient over A of  <dU, U> + <dS, S> + <dVT, VT>
 * for the outputs (U, S, VT) of that execute.
 *   dU, dS, dVT  host arrays of batch device pointers: cotangents shaped like
 *                U (m x k, leading dimension ldu), S (k) and VT (k x n, ldvt),
 *                in the plan's dtype.  Entries of the triplets beyond k_kept
 *                (whose outputs are constant zeros) are ignored.
 *   dA           host array of batch device pointers, m x n with leading
 *                dimension lda, the plan's dtype; overwritten.  Must not
 *                overlap A or the cotangents.
 *   broadening   >= 0.  The factor 1 / (s_j^2 - s_i^2) of the SVD adjoint is
 *                replaced by d / (d^2 + eps), d = s_j^2 - s_i^2,
 *                eps = broadening * s_1^4; 0 gives the exact adjoint, which
 *                diverges as two kept singular values approach each other.
 * The products run in FP64 on the stored A whatever the plan's precision.
 * The forward's A and outputs must be unchanged since that execute, and the
 * call must be stream-ordered after it.  Asynchronous on stream.  Returns
 * RSVD_ERR_INVALID without a saved forward, for a negative or NaN
 * broadening, or for null pointers. */
int rsvd_plan_backward(rsvd_plan_t* plan, const void* const* dU, const void* const* dS,
                       const void* const* dVT, void* const* dA, double broadening, void* stream);

/* rsvd_plan_profile_backward -- rsvd_plan_backward without the graph, with
 * HIP events around every launch; outputs as rsvd_plan_profile (phases
 * RSVD_PHASE_BW_GEMM and RSVD_PHASE_BW_SMALL).  Blocking. */
int rsvd_plan_profile_backward(rsvd_plan_t* plan, const void* const* dU, const void* const* dS,
                               const void* const* dVT, void* const* dA, double broadening, double* ms,
                               int64_t* launches, double* flops, int ncat, void* stream);

/* rsvd_plan_postselect -- sector post-selection (paper Sec. III.A).  When a
 * block-diagonal matrix (one block per symmetry sector) is truncated block by
 * block, each sector's RSVD is run with a guessed rank chi'_s; afterwards the
 * chi largest singular values over all sectors are kept, which sets the
 * sector ranks chi_s.  The sectors are the problems of the plan, and the
 * candidates are the k_kept values each kept in the plan's last
 * rsvd_plan_execute (same output buffers, which must still be valid).
 *   chi    >= 0, the total number of singular values to keep.
 *   chi_s  device int64_t[batch], receives chi_s[b], the number kept in
 *          problem b.  sum chi_s = min(chi, sum k_kept).
 * The kept values are the first chi in the order (value descending, problem
 * ascending, index ascending), so each problem keeps a prefix of its sorted S.
 * For the dropped triplets of each problem the call adds their squared
 * singular values to discarded_weight[b] (which stays the squared Frobenius
 * error of that problem's truncation), zero-fills them in S, U (columns) and
 * VT (rows), and sets k_kept[b] = chi_s[b].  A later rsvd_plan_backward
 * treats the dropped triplets like any beyond k_kept.  At most 8192 problems.
 * Asynchronous on stream, which must order it after the execute.  Returns
 * RSVD_ERR_INVALID for a null plan or chi_s, chi < 0, more than 8192
 * problems, or a plan that has not been executed. */
int rsvd_plan_postselect(rsvd_plan_t* plan, int64_t chi, int64_t* chi_s, void* stream);

/* Tile autotuning (batching of uneven problem lists).  A plan created with
 * RSVD_PLAN_TUNE spends its first rsvd_plan_execute (or rsvd_plan_profile)
 * measuring, before the normal execute: every forward product that is not
 * gathered, accumulating or lower-triangular (the sketch and power-iteration
 * products A Omega, A^T Q, A Z, the projection B = Q^T A and the products of
 * the triangular-factor small SVD) is launched with each workgroup tile
 * (64x64, 128x64, 64x128, 128x128 outputs) on the call's own inputs, one
 * warm-up and three timed launches each (HIP events), and the fastest is kept
 * for the life of the plan and captured in its graph.  All tiles give
 * bit-identical products (each output element is summed in the same K order).
 * Choices are remembered per launch signature (kinds, element types and every
 * problem's M, N, K and transposes) in a process-wide table, so a later plan
 * with the same shapes measures nothing; when the environment variable
 * RSVD_TUNE_CACHE names a file, the table is read from it once and rewritten
 * (a JSON object, signature -> "BMxBN") after each new entry.  The tuning
 * execute synchronizes the stream and is blocking.  Without RSVD_PLAN_TUNE a
 * shape heuristic picks the tile (128x64 for products with M >= 512 and
 * N <= 160 that give at least 512 such tiles, else 64x64).
 *
 * rsvd_plan_tiles -- the tile in use for each of those products, in launch
 * order: tiles[2 i] = rows, tiles[2 i + 1] = columns of product i's output
 * tile, for i < min(cap, *count); *count = number of such products.  Host
 * pointers.  Returns RSVD_ERR_INVALID for a null plan or count, cap < 0, or
 * tiles null with cap > 0. */
int rsvd_plan_tiles(const rsvd_plan_t* plan, int32_t* tiles, int64_t cap, int64_t* count);

/* rsvd_plan_set_tiles -- fixes the tile of each of those products (same
 * order and encoding as rsvd_plan_tiles; count must equal its *count), for
 * example to replay tiles tuned offline.  The plan counts as tuned afterwards
 * (RSVD_PLAN_TUNE then measures nothing) and its graph is re-captured at the
 * next execute.  Waits for the device to be idle; no execute of the plan may
 * be in flight on another thread.  Returns RSVD_ERR_INVALID for a null plan,
 * a wrong count or a tile that is not one of the four. */
int rsvd_plan_set_tiles(rsvd_plan_t* plan, const int32_t* tiles, int64_t count);

/* Device bytes of the plan's workspace. */
int64_t rsvd_plan_workspace_bytes(const rsvd_plan_t* plan);

/* Releases the plan's device memory and graph.  Safe on NULL. */
void rsvd_plan_destroy(rsvd_plan_t* plan);

/* Thread-local description of the most recent failure ("" if none). */
const char* rsvd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBRSVD_H */
