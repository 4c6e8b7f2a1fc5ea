/*
 * FP64 CPU oracle for the randomized truncated SVD (RSVD) and the
 * deterministic "full SVD, then discard" truncation (TSVD).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct reference that the GPU library is checked against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the GPU
 * library, and the GPU library never calls it.
 *
 * Everything is double precision, row-major, naive loops, one problem per
 * call (the caller may run several calls on several threads).
 *
 * Paper sections followed (Kohn et al., "Probabilistic low-rank
 * factorization accelerates tensor network simulations of critical quantum
 * many-body ground states"):
 *   - Sec. II.A, Alg. TSVD: full SVD of A, keep the chi largest triplets.
 *   - Sec. II.A (Eckart-Young-Mirsky remark): the discarded squared
 *     Frobenius weight is the sum of the squared discarded singular values.
 *   - Sec. II.B, Alg. RSVD steps 1-4: Gaussian test matrix Omega (n x l),
 *     Y = (A A^T)^q A Omega carried out as a power iteration with a QR after
 *     every product (the paper defers to Halko-Martinsson-Tropp 2011,
 *     Algorithm 4.4), Q = orthonormal basis of Y, SVD of B = Q^T A,
 *     left vectors Q*Utilde, right vectors Vtilde.
 * Readings where the paper is silent (random-number layout, truncation by a
 * relative discarded-weight threshold, sign convention, m < n handling) are
 * stated next to the code that implements them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_INVALID -1
#define ORC_ERR_ALLOC -2
#define ORC_ERR_NONFINITE -4
#define ORC_ERR_NOCONV -5

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.                           */
/* ------------------------------------------------------------------------ */
static void philox_mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t prod = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(prod >> 32);
    *lo = (uint32_t)prod;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint32_t hi0, lo0, hi1, lo1;
        philox_mulhilo(mult0, x0, &hi0, &lo0);
        philox_mulhilo(mult1, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Gaussian test matrix, Alg. RSVD step 1.  The paper only asks for i.i.d.
 * standard normal entries and notes that the quality of the random numbers
 * is not critical.  Reading used here (a fixed, documented layout so that
 * two independent implementations draw the same matrix):
 *   key     = (seed mod 2^32, seed >> 32)
 *   counter = (floor(i/2), j, 0, 0)           for entry (i, j), 0-based
 *   words x0..x3 = Philox4x32-10(counter, key)
 *   u1 = 1 - ((x0*2^32 + x1) >> 11) * 2^-53   in (0, 1]
 *   u2 =     ((x2*2^32 + x3) >> 11) * 2^-53   in [0, 1)
 *   r  = sqrt(-2 ln u1)
 *   Omega(i, j) = r cos(2 pi u2)  for even i,  r sin(2 pi u2)  for odd i
 * (the Box-Muller transform; both normals of one pair come from one call).
 */
double orc_omega_entry(uint64_t seed, int64_t i, int64_t j)
{
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)(i / 2), (uint32_t)j, 0u, 0u};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    uint64_t a = ((uint64_t)x[0] << 32) | x[1];
    uint64_t b = ((uint64_t)x[2] << 32) | x[3];
    double u1 = 1.0 - (double)(a >> 11) * 0x1.0p-53;
    double u2 = (double)(b >> 11) * 0x1.0p-53;
    double r = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    return (i % 2 == 0) ? r * cos(ang) : r * sin(ang);
}

void orc_gaussian(uint64_t seed, int64_t n, int64_t l, double *omega)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < l; ++j)
            omega[i * l + j] = orc_omega_entry(seed, i, j);
}

/* ------------------------------------------------------------------------ */
/* Small helpers: compensated (Neumaier) summation and naive products.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double s, c;
} orc_sum;

static void orc_sum_add(orc_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double orc_sum_val(const orc_sum *a) { return a->s + a->c; }

/* C (m x l) = A (m x n, lda) * X (n x l) */
static void mat_a_x(int64_t m, int64_t n, int64_t l, const double *A, int64_t lda,
                    const double *X, double *C)
{
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + i * l;
        for (int64_t j = 0; j < l; ++j) c[j] = 0.0;
        for (int64_t t = 0; t < n; ++t) {
            double a = A[i * lda + t];
            const double *x = X + t * l;
            for (int64_t j = 0; j < l; ++j) c[j] += a * x[j];
        }
    }
}

/* C (n x l) = A^T * X, A m x n (lda), X m x l */
static void mat_at_x(int64_t m, int64_t n, int64_t l, const double *A, int64_t lda,
                     const double *X, double *C)
{
    for (int64_t i = 0; i < n * l; ++i) C[i] = 0.0;
    for (int64_t t = 0; t < m; ++t) {
        const double *x = X + t * l;
        for (int64_t i = 0; i < n; ++i) {
            double a = A[t * lda + i];
            double *c = C + i * l;
            for (int64_t j = 0; j < l; ++j) c[j] += a * x[j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Householder thin QR, Y (m x l, m >= l) -> Q (m x l), R (l x l), with the  */
/* sign convention diag(R) >= 0 so that Q is unique for full-rank Y.        */
/* Used for every "orthonormalise" of Alg. RSVD (steps 2 and 3).            */
/* ------------------------------------------------------------------------ */
int orc_hqr(int64_t m, int64_t l, const double *Y, double *Q, double *R)
{
    if (m < l || l < 1) return ORC_ERR_INVALID;
    double *W = (double *)malloc(sizeof(double) * m * l);
    double *V = (double *)calloc((size_t)(m * l), sizeof(double)); /* reflectors */
    double *tau = (double *)calloc((size_t)l, sizeof(double));
    if (!W || !V || !tau) {
        free(W); free(V); free(tau);
        return ORC_ERR_ALLOC;
    }
    memcpy(W, Y, sizeof(double) * m * l);
    for (int64_t j = 0; j < l; ++j) {
        double nrm2 = 0.0;
        for (int64_t i = j; i < m; ++i) nrm2 += W[i * l + j] * W[i * l + j];
        double nrm = sqrt(nrm2);
        if (nrm == 0.0) { /* zero column below the diagonal: H_j = I */
            tau[j] = 0.0;
            continue;
        }
        double x0 = W[j * l + j];
        double alpha = (x0 >= 0.0) ? -nrm : nrm;
        /* v = x - alpha e1 */
        double vv = 0.0;
        for (int64_t i = j; i < m; ++i) {
            double vi = W[i * l + j] - ((i == j) ? alpha : 0.0);
            V[i * l + j] = vi;
            vv += vi * vi;
        }
        tau[j] = (vv > 0.0) ? 2.0 / vv : 0.0;
        /* apply H_j = I - tau v v^T to W[j:, j:] */
        for (int64_t c = j; c < l; ++c) {
            double d = 0.0;
            for (int64_t i = j; i < m; ++i) d += V[i * l + j] * W[i * l + c];
            d *= tau[j];
            for (int64_t i = j; i < m; ++i) W[i * l + c] -= d * V[i * l + j];
        }
    }
    /* R = upper triangle of W */
    for (int64_t i = 0; i < l; ++i)
        for (int64_t c = 0; c < l; ++c) R[i * l + c] = (c >= i) ? W[i * l + c] : 0.0;
    /* Q = H_0 H_1 ... H_{l-1} [I; 0], accumulated from the last reflector */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < l; ++c) Q[i * l + c] = (i == c) ? 1.0 : 0.0;
    for (int64_t j = l - 1; j >= 0; --j) {
        if (tau[j] == 0.0) continue;
        for (int64_t c = 0; c < l; ++c) {
            double d = 0.0;
            for (int64_t i = j; i < m; ++i) d += V[i * l + j] * Q[i * l + c];
            d *= tau[j];
            for (int64_t i = j; i < m; ++i) Q[i * l + c] -= d * V[i * l + j];
        }
    }
    /* sign fix: diag(R) >= 0 */
    for (int64_t j = 0; j < l; ++j) {
        if (R[j * l + j] < 0.0) {
            for (int64_t c = 0; c < l; ++c) R[j * l + c] = -R[j * l + c];
            for (int64_t i = 0; i < m; ++i) Q[i * l + j] = -Q[i * l + j];
        }
    }
    free(W); free(V); free(tau);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One-sided (Hestenes) Jacobi on the columns of G (r x c, row-major).       */
/* On return the columns of G are mutually orthogonal, G_out = G_in * J,    */
/* J (c x c) orthogonal.  Pair order: cyclic by rows (i < j).  A pair is    */
/* rotated when |g_i.g_j| > tol * ||g_i|| ||g_j||; the sweep loop stops     */
/* after a sweep with no rotation (tol = r * 2^-53) or after max_sweeps.    */
/* This is the small SVD of Alg. RSVD step 4 (any backward-stable SVD       */
/* serves there) and the full SVD of Alg. TSVD.                             */
/* ------------------------------------------------------------------------ */
int orc_jacobi_cols(int64_t r, int64_t c, double *G, double *J, int max_sweeps,
                    int *sweeps_out)
{
    const double tol = (double)(r > 1 ? r : 1) * 0x1.0p-53;
    for (int64_t i = 0; i < c; ++i)
        for (int64_t j = 0; j < c; ++j) J[i * c + j] = (i == j) ? 1.0 : 0.0;
    int sweep = 0;
    int converged = 0;
    while (sweep < max_sweeps) {
        ++sweep;
        int64_t rotations = 0;
        for (int64_t p = 0; p + 1 < c; ++p) {
            for (int64_t q = p + 1; q < c; ++q) {
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t t = 0; t < r; ++t) {
                    double gp = G[t * c + p], gq = G[t * c + q];
                    alpha += gp * gp;
                    beta += gq * gq;
                    gamma += gp * gq;
                }
                if (!(fabs(gamma) > tol * sqrt(alpha) * sqrt(beta))) continue;
                ++rotations;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150)
                    t = 0.5 / zeta;
                else
                    t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int64_t s = 0; s < r; ++s) {
                    double gp = G[s * c + p], gq = G[s * c + q];
                    G[s * c + p] = cs * gp - sn * gq;
                    G[s * c + q] = sn * gp + cs * gq;
                }
                for (int64_t s = 0; s < c; ++s) {
                    double jp = J[s * c + p], jq = J[s * c + q];
                    J[s * c + p] = cs * jp - sn * jq;
                    J[s * c + q] = sn * jp + cs * jq;
                }
            }
        }
        if (rotations == 0) {
            converged = 1;
            break;
        }
    }
    if (sweeps_out) *sweeps_out = sweep;
    return converged ? ORC_OK : ORC_ERR_NOCONV;
}

/* Stable sort of indices by value, descending (insertion sort; c is small). */
static void sort_desc(int64_t c, const double *val, int64_t *perm)
{
    for (int64_t i = 0; i < c; ++i) perm[i] = i;
    for (int64_t i = 1; i < c; ++i) {
        int64_t x = perm[i];
        int64_t j = i - 1;
        while (j >= 0 && val[perm[j]] < val[x]) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = x;
    }
}

/*
 * Truncation rule (reading of the paper's discarded-weight truncation; the
 * paper measures the truncation error in the Frobenius norm, Sec. II.A):
 *   w(k') = discarded squared Frobenius weight when keeping k' triplets,
 *   k_kept = k                                    if delta == 0,
 *          = min(k, smallest k' >= 1 with w(k') <= delta * ||A||_F^2)  else,
 *   k_kept = 0 when ||A||_F = 0.
 * wk[j] holds w(j) for j = 0..k.
 */
static int64_t choose_k(int64_t k, double delta, double normA2, const double *wk)
{
    if (normA2 == 0.0) return 0;
    if (delta == 0.0) return k;
    for (int64_t kp = 1; kp <= k; ++kp)
        if (wk[kp] <= delta * normA2) return kp;
    return k;
}

/* Sign convention: the entry of largest magnitude of every kept left vector
 * is positive (first such entry on ties); the right vector follows. */
static void canonical_signs(int64_t m, int64_t n, int64_t kk, double *U, int64_t ldu,
                            double *VT, int64_t ldvt)
{
    for (int64_t j = 0; j < kk; ++j) {
        int64_t best = 0;
        double bv = -1.0;
        for (int64_t i = 0; i < m; ++i) {
            double a = fabs(U[i * ldu + j]);
            if (a > bv) {
                bv = a;
                best = i;
            }
        }
        if (U[best * ldu + j] < 0.0) {
            for (int64_t i = 0; i < m; ++i) U[i * ldu + j] = -U[i * ldu + j];
            for (int64_t t = 0; t < n; ++t) VT[j * ldvt + t] = -VT[j * ldvt + t];
        }
    }
}

static int check_args(const double *A, int64_t m, int64_t n, int64_t lda, int64_t k,
                      double delta, const void *U, int64_t ldu, const void *S,
                      const void *VT, int64_t ldvt)
{
    if (!A || !U || !S || !VT) return ORC_ERR_INVALID;
    if (m < 1 || n < 1 || k < 1 || lda < n) return ORC_ERR_INVALID;
    if (!(delta >= 0.0)) return ORC_ERR_INVALID; /* also rejects NaN */
    int64_t kk = k < (m < n ? m : n) ? k : (m < n ? m : n);
    if (ldu < kk || ldvt < n) return ORC_ERR_INVALID;
    return ORC_OK;
}

static double frob2(const double *A, int64_t m, int64_t n, int64_t lda)
{
    orc_sum s = {0.0, 0.0};
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) orc_sum_add(&s, A[i * lda + j] * A[i * lda + j]);
    return orc_sum_val(&s);
}

/* ------------------------------------------------------------------------ */
/* Alg. RSVD (Sec. II.B), with the power iteration in the Halko et al.       */
/* Algorithm 4.4 form the paper prescribes: QR after every product with A    */
/* and with A^T.                                                             */
/*   kk = min(k, m, n); l = min(kk + p, m, n)                                */
/*   Omega = Gaussian(seed) (n x l)                                          */
/*   Q0 = qr(A Omega)                                                        */
/*   for j = 1..q:  Z = qr(A^T Q);  Q = qr(A Z)                              */
/*   B^T = A^T Q  (n x l)                                                    */
/*   one-sided Jacobi on the columns of B^T: B^T J = Vt Sigma  ->            */
/*       B = J Sigma Vt^T, so Utilde = J, Vtilde = columns of B^T J / sigma  */
/*   sort, truncate (choose_k), U = Q Utilde[:, :k_kept], signs, zero-fill.  */
/* Optional outputs: sig_all (l values, sorted), Q_out (m x l final basis),  */
/* l_out, sweeps_out.  Returns ORC_OK, ORC_ERR_* as documented.             */
/* ------------------------------------------------------------------------ */
int orc_rsvd(const double *A, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
             int64_t q, uint64_t seed, double delta, double *U, int64_t ldu, double *S,
             double *VT, int64_t ldvt, double *w_out, int64_t *k_kept_out,
             double *sig_all, double *Q_out, int64_t *l_out, int *sweeps_out)
{
    int st = check_args(A, m, n, lda, k, delta, U, ldu, S, VT, ldvt);
    if (st != ORC_OK) return st;
    if (p < 0 || q < 0) return ORC_ERR_INVALID;
    int64_t mn = m < n ? m : n;
    int64_t kk = k < mn ? k : mn;
    int64_t l = kk + p < mn ? kk + p : mn;
    if (l_out) *l_out = l;

    double normA2 = frob2(A, m, n, lda);
    if (!isfinite(normA2)) return ORC_ERR_NONFINITE;

    double *Om = (double *)malloc(sizeof(double) * n * l);
    double *Y = (double *)malloc(sizeof(double) * m * l);
    double *Q = (double *)malloc(sizeof(double) * m * l);
    double *Wt = (double *)malloc(sizeof(double) * n * l);
    double *Z = (double *)malloc(sizeof(double) * n * l);
    double *R = (double *)malloc(sizeof(double) * l * l);
    double *J = (double *)malloc(sizeof(double) * l * l);
    double *sig = (double *)malloc(sizeof(double) * l);
    double *wk = (double *)malloc(sizeof(double) * (kk + 1));
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * l);
    if (!Om || !Y || !Q || !Wt || !Z || !R || !J || !sig || !wk || !perm) {
        st = ORC_ERR_ALLOC;
        goto done;
    }

    /* step 1: Gaussian test matrix */
    orc_gaussian(seed, n, l, Om);
    /* step 2 (power iteration) and step 3 (orthonormal basis) */
    mat_a_x(m, n, l, A, lda, Om, Y);
    st = orc_hqr(m, l, Y, Q, R);
    if (st != ORC_OK) goto done;
    for (int64_t it = 0; it < q; ++it) {
        mat_at_x(m, n, l, A, lda, Q, Wt);
        st = orc_hqr(n, l, Wt, Z, R);
        if (st != ORC_OK) goto done;
        mat_a_x(m, n, l, A, lda, Z, Y);
        st = orc_hqr(m, l, Y, Q, R);
        if (st != ORC_OK) goto done;
    }
    if (Q_out) memcpy(Q_out, Q, sizeof(double) * m * l);
    /* step 4: B^T = A^T Q, then its SVD by one-sided Jacobi */
    mat_at_x(m, n, l, A, lda, Q, Wt);
    int sweeps = 0;
    int jst = orc_jacobi_cols(n, l, Wt, J, 60, &sweeps);
    if (sweeps_out) *sweeps_out = sweeps;
    for (int64_t j = 0; j < l; ++j) {
        double s2 = 0.0;
        for (int64_t t = 0; t < n; ++t) s2 += Wt[t * l + j] * Wt[t * l + j];
        sig[j] = sqrt(s2);
    }
    sort_desc(l, sig, perm);
    if (sig_all)
        for (int64_t j = 0; j < l; ++j) sig_all[j] = sig[perm[j]];

    /* discarded weight w(k') = ||A||^2 - sum_{j<=k'} sigma_j^2 (>= 0) */
    {
        orc_sum acc = {0.0, 0.0};
        orc_sum_add(&acc, normA2);
        wk[0] = normA2;
        for (int64_t j = 1; j <= kk; ++j) {
            double sj = sig[perm[j - 1]];
            orc_sum_add(&acc, -sj * sj);
            double v = orc_sum_val(&acc);
            wk[j] = v > 0.0 ? v : 0.0;
        }
    }
    int64_t kkeep = choose_k(kk, delta, normA2, wk);
    if (k_kept_out) *k_kept_out = kkeep;
    if (w_out) *w_out = (normA2 == 0.0) ? 0.0 : wk[kkeep];

    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < kk; ++j) U[i * ldu + j] = 0.0;
    for (int64_t j = 0; j < kk; ++j) {
        S[j] = 0.0;
        for (int64_t t = 0; t < n; ++t) VT[j * ldvt + t] = 0.0;
    }
    for (int64_t j = 0; j < kkeep; ++j) {
        int64_t c = perm[j];
        S[j] = sig[c];
        /* U(:, j) = Q * J(:, c) */
        for (int64_t i = 0; i < m; ++i) {
            double a = 0.0;
            for (int64_t t = 0; t < l; ++t) a += Q[i * l + t] * J[t * l + c];
            U[i * ldu + j] = a;
        }
        /* VT(j, :) = column c of B^T J, normalised */
        double inv = sig[c] > 0.0 ? 1.0 / sig[c] : 0.0;
        for (int64_t t = 0; t < n; ++t) VT[j * ldvt + t] = Wt[t * l + c] * inv;
    }
    canonical_signs(m, n, kkeep, U, ldu, VT, ldvt);
    st = (jst == ORC_OK) ? ORC_OK : ORC_ERR_NOCONV;
done:
    free(Om); free(Y); free(Q); free(Wt); free(Z); free(R); free(J);
    free(sig); free(wk); free(perm);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Alg. TSVD (Sec. II.A): full SVD by one-sided Jacobi (on A when m >= n,   */
/* on A^T otherwise), then keep the leading triplets.  Discarded weight is */
/* the direct tail sum of squared singular values (Eckart-Young-Mirsky).   */
/* Optional sig_all receives all min(m, n) singular values, sorted.        */
/* ------------------------------------------------------------------------ */
int orc_fullsvd(const double *A, int64_t m, int64_t n, int64_t lda, int64_t k,
                double delta, double *U, int64_t ldu, double *S, double *VT,
                int64_t ldvt, double *w_out, int64_t *k_kept_out, double *sig_all,
                int *sweeps_out)
{
    int st = check_args(A, m, n, lda, k, delta, U, ldu, S, VT, ldvt);
    if (st != ORC_OK) return st;
    int64_t mn = m < n ? m : n;
    int64_t kk = k < mn ? k : mn;
    double normA2 = frob2(A, m, n, lda);
    if (!isfinite(normA2)) return ORC_ERR_NONFINITE;

    int tall = (m >= n);
    int64_t r = tall ? m : n;   /* column length */
    int64_t c = mn;             /* number of columns */
    double *G = (double *)malloc(sizeof(double) * r * c);
    double *J = (double *)malloc(sizeof(double) * c * c);
    double *sig = (double *)malloc(sizeof(double) * c);
    double *wk = (double *)malloc(sizeof(double) * (kk + 1));
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * c);
    if (!G || !J || !sig || !wk || !perm) {
        st = ORC_ERR_ALLOC;
        goto done;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (tall)
                G[i * c + j] = A[i * lda + j];
            else
                G[j * c + i] = A[i * lda + j];
        }
    int sweeps = 0;
    int jst = orc_jacobi_cols(r, c, G, J, 60, &sweeps);
    if (sweeps_out) *sweeps_out = sweeps;
    for (int64_t j = 0; j < c; ++j) {
        double s2 = 0.0;
        for (int64_t t = 0; t < r; ++t) s2 += G[t * c + j] * G[t * c + j];
        sig[j] = sqrt(s2);
    }
    sort_desc(c, sig, perm);
    if (sig_all)
        for (int64_t j = 0; j < c; ++j) sig_all[j] = sig[perm[j]];
    /* w(k') = sum_{j > k'} sigma_j^2, summed from the smallest upward */
    {
        orc_sum acc = {0.0, 0.0};
        double *tail = (double *)malloc(sizeof(double) * (c + 1));
        if (!tail) {
            st = ORC_ERR_ALLOC;
            goto done;
        }
        tail[c] = 0.0;
        for (int64_t j = c - 1; j >= 0; --j) {
            double sj = sig[perm[j]];
            orc_sum_add(&acc, sj * sj);
            tail[j] = orc_sum_val(&acc);
        }
        for (int64_t j = 0; j <= kk; ++j) wk[j] = tail[j];
        free(tail);
    }
    int64_t kkeep = choose_k(kk, delta, normA2, wk);
    if (k_kept_out) *k_kept_out = kkeep;
    if (w_out) *w_out = (normA2 == 0.0) ? 0.0 : wk[kkeep];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < kk; ++j) U[i * ldu + j] = 0.0;
    for (int64_t j = 0; j < kk; ++j) {
        S[j] = 0.0;
        for (int64_t t = 0; t < n; ++t) VT[j * ldvt + t] = 0.0;
    }
    for (int64_t j = 0; j < kkeep; ++j) {
        int64_t cidx = perm[j];
        S[j] = sig[cidx];
        double inv = sig[cidx] > 0.0 ? 1.0 / sig[cidx] : 0.0;
        if (tall) {
            /* A J = G  ->  U = G / sigma, V = J */
            for (int64_t i = 0; i < m; ++i) U[i * ldu + j] = G[i * c + cidx] * inv;
            for (int64_t t = 0; t < n; ++t) VT[j * ldvt + t] = J[t * c + cidx];
        } else {
            /* A^T J = G  ->  V = G / sigma, U = J */
            for (int64_t i = 0; i < m; ++i) U[i * ldu + j] = J[i * c + cidx];
            for (int64_t t = 0; t < n; ++t) VT[j * ldvt + t] = G[t * c + cidx] * inv;
        }
    }
    canonical_signs(m, n, kkeep, U, ldu, VT, ldvt);
    st = (jst == ORC_OK) ? ORC_OK : ORC_ERR_NOCONV;
done:
    free(G); free(J); free(sig); free(wk); free(perm);
    return st;
}

/* ======================================================================== */
/* Reverse-mode derivatives (adjoints), FP64, Gaussian test matrix fixed.   */
/* The paper has no derivative; these follow the standard matrix-calculus  */
/* results: the SVD adjoint (Townsend 2016, "Differentiating the singular  */
/* value decomposition"; Seeger et al. 2017) with optional Lorentzian      */
/* broadening of 1/(s_j^2 - s_i^2), the thin-QR adjoint (Walter & Lehmann  */
/* 2018; Liao et al. 2019), and the product rule through every GEMM of     */
/* Alg. RSVD.                                                              */
/* ======================================================================== */

/* C (M x N) = beta C + op(X) op(Y), op(X) M x K; tx/ty: 0 plain, 1 transposed */
static void mm(int tx, int ty, int64_t M, int64_t N, int64_t K, const double *X, int64_t ldx,
               const double *Y, int64_t ldy, double beta, double *C, int64_t ldc)
{
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            for (int64_t t = 0; t < K; ++t) {
                double a = tx ? X[t * ldx + i] : X[i * ldx + t];
                double b = ty ? Y[j * ldy + t] : Y[t * ldy + j];
                s += a * b;
            }
            C[i * ldc + j] = (beta == 0.0) ? s : beta * C[i * ldc + j] + s;  /* beta = 0 overwrites */
        }
}

/* F_ij = 1/(s_j^2 - s_i^2) (i != j), broadened to d/(d^2 + eps); F_ii = 0 */
static double fmat(double si, double sj, double eps)
{
    double d = sj * sj - si * si;
    if (eps > 0.0) return d / (d * d + eps);
    return d != 0.0 ? 1.0 / d : 0.0;
}

/*
 * SVD adjoint for X (r x c, r <= c) = Ut diag(s) Vt^T with Ut (r x r)
 * orthogonal, Vt (c x r) orthonormal columns, given cotangents Ub (r x r),
 * sb (r), Vb (c x r).  Result Xb (r x c):
 *   Xb = Ut [diag(sb) + J_U S + S J_V] Vt^T + Ut S^-1 Vb^T (I - Vt Vt^T),
 *   J_U = F o (Ut^T Ub - Ub^T Ut),  J_V = F o (Vt^T Vb - Vb^T Vt).
 * Rows with s_i = 0 take no S^-1 term.
 */
static void svd_adjoint_wide(int64_t r, int64_t c, const double *Ut, const double *s, const double *Vt,
                             const double *Ub, const double *sb, const double *Vb, double eps,
                             double *Xb)
{
    double *EU = (double *)malloc(sizeof(double) * r * r);
    double *EV = (double *)malloc(sizeof(double) * r * r);
    double *K = (double *)malloc(sizeof(double) * r * r);
    double *N = (double *)malloc(sizeof(double) * r * c);
    mm(1, 0, r, r, r, Ut, r, Ub, r, 0.0, EU, r);   /* Ut^T Ub */
    mm(1, 0, r, r, c, Vt, r, Vb, r, 0.0, EV, r);   /* Vt^T Vb */
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < r; ++j) {
            double f = (i == j) ? 0.0 : fmat(s[i], s[j], eps);
            double ju = f * (EU[i * r + j] - EU[j * r + i]);
            double jv = f * (EV[i * r + j] - EV[j * r + i]);
            K[i * r + j] = ((i == j) ? sb[i] : 0.0) + ju * s[j] + s[i] * jv;
        }
    /* N = K Vt^T + S^-1 (Vb^T - EV^T Vt^T) */
    mm(0, 1, r, c, r, K, r, Vt, r, 0.0, N, c);
    for (int64_t i = 0; i < r; ++i) {
        if (!(s[i] > 0.0)) continue;
        double inv = 1.0 / s[i];
        for (int64_t t = 0; t < c; ++t) {
            double v = Vb[t * r + i];
            for (int64_t j = 0; j < r; ++j) v -= EV[j * r + i] * Vt[t * r + j];
            N[i * c + t] += inv * v;
        }
    }
    mm(0, 0, r, c, r, Ut, r, N, c, 0.0, Xb, c);
    free(EU); free(EV); free(K); free(N);
}

/* Thin-QR adjoint: M = Q R (rows x l, R upper with positive diagonal), given
 * Qb: Mb = (Qb + Q copyltu(-Qb^T Q)) R^-T, copyltu(X) = tril(X) + tril(X,-1)^T. */
static void qr_adjoint(int64_t rows, int64_t l, const double *Q, const double *R, const double *Qb,
                       double *Mb)
{
    double *C = (double *)malloc(sizeof(double) * l * l);
    double *S = (double *)malloc(sizeof(double) * l * l);
    mm(1, 0, l, l, rows, Qb, l, Q, l, 0.0, C, l); /* Qb^T Q */
    for (int64_t i = 0; i < l; ++i)
        for (int64_t j = 0; j < l; ++j) S[i * l + j] = -((i >= j) ? C[i * l + j] : C[j * l + i]);
    double *X = (double *)malloc(sizeof(double) * rows * l);
    memcpy(X, Qb, sizeof(double) * rows * l);
    mm(0, 0, rows, l, l, Q, l, S, l, 1.0, X, l);
    /* Mb R^T = X: back substitution per row */
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t rr = l - 1; rr >= 0; --rr) {
            double v = X[i * l + rr];
            for (int64_t c = rr + 1; c < l; ++c) v -= Mb[i * l + c] * R[rr * l + c];
            Mb[i * l + rr] = (R[rr * l + rr] != 0.0) ? v / R[rr * l + rr] : 0.0;
        }
    free(C); free(S); free(X);
}

/* Sorted thin factors of B^T's Jacobi result and the truncation/sign state
 * of the forward, recomputed exactly as orc_rsvd does. */
typedef struct {
    int64_t m, n, kk, l, kkeep, nst;
    double *Om, **M, **Q, **R, *Ut, *s, *Vt, *sgn;
} rsvd_state;

static void state_free(rsvd_state *st)
{
    if (st->M)
        for (int64_t i = 0; i < st->nst; ++i) {
            free(st->M[i]); free(st->Q[i]); free(st->R[i]);
        }
    free(st->M); free(st->Q); free(st->R);
    free(st->Om); free(st->Ut); free(st->s); free(st->Vt); free(st->sgn);
}

static int rsvd_forward_state(const double *A, int64_t m, int64_t n, int64_t lda, int64_t k,
                              int64_t p, int64_t q, uint64_t seed, double delta, rsvd_state *st)
{
    memset(st, 0, sizeof(*st));
    int64_t mn = m < n ? m : n;
    int64_t kk = k < mn ? k : mn;
    int64_t l = kk + p < mn ? kk + p : mn;
    int64_t nst = 2 * q + 1;
    st->m = m; st->n = n; st->kk = kk; st->l = l; st->nst = nst;
    double normA2 = frob2(A, m, n, lda);
    if (!isfinite(normA2)) return ORC_ERR_NONFINITE;
    st->Om = (double *)malloc(sizeof(double) * n * l);
    st->M = (double **)calloc((size_t)nst, sizeof(double *));
    st->Q = (double **)calloc((size_t)nst, sizeof(double *));
    st->R = (double **)calloc((size_t)nst, sizeof(double *));
    orc_gaussian(seed, n, l, st->Om);
    for (int64_t s = 0; s < nst; ++s) {
        int64_t rows = (s % 2 == 0) ? m : n;
        st->M[s] = (double *)malloc(sizeof(double) * rows * l);
        st->Q[s] = (double *)malloc(sizeof(double) * rows * l);
        st->R[s] = (double *)malloc(sizeof(double) * l * l);
        if (s == 0)
            mat_a_x(m, n, l, A, lda, st->Om, st->M[s]);
        else if (s % 2 == 1)
            mat_at_x(m, n, l, A, lda, st->Q[s - 1], st->M[s]);
        else
            mat_a_x(m, n, l, A, lda, st->Q[s - 1], st->M[s]);
        int rc = orc_hqr(rows, l, st->M[s], st->Q[s], st->R[s]);
        if (rc != ORC_OK) return rc;
    }
    double *G = (double *)malloc(sizeof(double) * n * l);
    double *J = (double *)malloc(sizeof(double) * l * l);
    double *sig = (double *)malloc(sizeof(double) * l);
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * l);
    double *wk = (double *)malloc(sizeof(double) * (kk + 1));
    mat_at_x(m, n, l, A, lda, st->Q[nst - 1], G);
    orc_jacobi_cols(n, l, G, J, 60, NULL);
    for (int64_t j = 0; j < l; ++j) {
        double s2 = 0.0;
        for (int64_t t = 0; t < n; ++t) s2 += G[t * l + j] * G[t * l + j];
        sig[j] = sqrt(s2);
    }
    sort_desc(l, sig, perm);
    st->Ut = (double *)malloc(sizeof(double) * l * l);
    st->Vt = (double *)malloc(sizeof(double) * n * l);
    st->s = (double *)malloc(sizeof(double) * l);
    st->sgn = (double *)malloc(sizeof(double) * l);
    for (int64_t j = 0; j < l; ++j) {
        int64_t c = perm[j];
        st->s[j] = sig[c];
        double inv = sig[c] > 0.0 ? 1.0 / sig[c] : 0.0;
        for (int64_t r = 0; r < l; ++r) st->Ut[r * l + j] = J[r * l + c];
        for (int64_t t = 0; t < n; ++t) st->Vt[t * l + j] = G[t * l + c] * inv;
    }
    {
        orc_sum acc = {0.0, 0.0};
        orc_sum_add(&acc, normA2);
        wk[0] = normA2;
        for (int64_t j = 1; j <= kk; ++j) {
            orc_sum_add(&acc, -st->s[j - 1] * st->s[j - 1]);
            double v = orc_sum_val(&acc);
            wk[j] = v > 0.0 ? v : 0.0;
        }
    }
    st->kkeep = choose_k(kk, delta, normA2, wk);
    /* signs of the kept left vectors Q Ut[:, j] (largest magnitude positive) */
    const double *Qf = st->Q[nst - 1];
    for (int64_t j = 0; j < l; ++j) {
        double best = -1.0, val = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double a = 0.0;
            for (int64_t t = 0; t < l; ++t) a += Qf[i * l + t] * st->Ut[t * l + j];
            if (fabs(a) > best) {
                best = fabs(a);
                val = a;
            }
        }
        st->sgn[j] = (val < 0.0) ? -1.0 : 1.0;
    }
    free(G); free(J); free(sig); free(perm); free(wk);
    return ORC_OK;
}

/*
 * dA of L = <dU, U> + <dS, S> + <dVT, VT> for the outputs of orc_rsvd
 * (U m x kk, S kk, VT kk x n, kk = min(k, m, n)), with Omega fixed by the seed.
 * Cotangents of the zero-filled triplets beyond k_kept are ignored.
 * broad: Lorentzian broadening eps = broad * sigma_1^4 (0 = exact).
 */
int orc_rsvd_backward(const double *A, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
                      int64_t q, uint64_t seed, double delta, const double *dU, const double *dS,
                      const double *dVT, double broad, double *dA)
{
    if (!A || !dU || !dS || !dVT || !dA || m < 1 || n < 1 || k < 1 || p < 0 || q < 0 || lda < n)
        return ORC_ERR_INVALID;
    rsvd_state st;
    int rc = rsvd_forward_state(A, m, n, lda, k, p, q, seed, delta, &st);
    if (rc != ORC_OK) {
        state_free(&st);
        return rc;
    }
    const int64_t l = st.l, kk = st.kk, kp = st.kkeep, nst = st.nst;
    const double eps = broad * pow(st.s[0], 4);
    double *Ub = (double *)calloc((size_t)(m * l), sizeof(double));  /* cotangent of Q Ut */
    double *Vb = (double *)calloc((size_t)(n * l), sizeof(double));  /* cotangent of Vt */
    double *sb = (double *)calloc((size_t)l, sizeof(double));
    for (int64_t j = 0; j < kp; ++j) {
        for (int64_t i = 0; i < m; ++i) Ub[i * l + j] = dU[i * kk + j] * st.sgn[j];
        for (int64_t t = 0; t < n; ++t) Vb[t * l + j] = dVT[j * n + t] * st.sgn[j];
        sb[j] = dS[j];
    }
    const double *Qf = st.Q[nst - 1];
    double *Utb = (double *)malloc(sizeof(double) * l * l);
    double *Bb = (double *)malloc(sizeof(double) * l * n);
    double *Qb = (double *)malloc(sizeof(double) * (m > n ? m : n) * l);
    double *Mb = (double *)malloc(sizeof(double) * (m > n ? m : n) * l);
    /* U = Q Ut: Utb = Q^T Ub, Qb = Ub Ut^T */
    mm(1, 0, l, l, m, Qf, l, Ub, l, 0.0, Utb, l);
    mm(0, 1, m, l, l, Ub, l, st.Ut, l, 0.0, Qb, l);
    /* SVD of B = Q^T A (l x n) */
    svd_adjoint_wide(l, n, st.Ut, st.s, st.Vt, Utb, sb, Vb, eps, Bb);
    /* B = Q^T A: Qb += A Bb^T, dA = Q Bb */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < l; ++j) {
            double v = 0.0;
            for (int64_t t = 0; t < n; ++t) v += A[i * lda + t] * Bb[j * n + t];
            Qb[i * l + j] += v;
        }
    mm(0, 0, m, n, l, Qf, l, Bb, n, 0.0, dA, n);
    /* stages in reverse: M_s = Q_s R_s, M_s = A Q_{s-1} (even s > 0), A^T Q_{s-1} (odd), A Omega (s = 0) */
    for (int64_t s = nst - 1; s >= 0; --s) {
        int64_t rows = (s % 2 == 0) ? m : n;
        qr_adjoint(rows, l, st.Q[s], st.R[s], Qb, Mb);
        if (s % 2 == 0) {
            const double *X = (s == 0) ? st.Om : st.Q[s - 1];  /* n x l */
            mm(0, 1, m, n, l, Mb, l, X, l, 1.0, dA, n);         /* dA += Mb X^T */
            if (s > 0) {                                        /* Qb_{s-1} = A^T Mb */
                for (int64_t i = 0; i < n; ++i)
                    for (int64_t j = 0; j < l; ++j) {
                        double v = 0.0;
                        for (int64_t t = 0; t < m; ++t) v += A[t * lda + i] * Mb[t * l + j];
                        Qb[i * l + j] = v;
                    }
            }
        } else {
            const double *X = st.Q[s - 1];                      /* m x l */
            mm(0, 1, m, n, l, X, l, Mb, l, 1.0, dA, n);         /* dA += Q_{s-1} Mb^T */
            for (int64_t i = 0; i < m; ++i)                     /* Qb_{s-1} = A Mb */
                for (int64_t j = 0; j < l; ++j) {
                    double v = 0.0;
                    for (int64_t t = 0; t < n; ++t) v += A[i * lda + t] * Mb[t * l + j];
                    Qb[i * l + j] = v;
                }
        }
    }
    free(Ub); free(Vb); free(sb); free(Utb); free(Bb); free(Qb); free(Mb);
    state_free(&st);
    return ORC_OK;
}

/*
 * Reference gradient of the exact truncated SVD (Alg. TSVD) for the same
 * loss, by the SVD adjoint applied to A's full SVD (cotangents zero beyond
 * k_kept).  Works on A (m <= n) or on A^T (m > n).
 */
int orc_fullsvd_backward(const double *A, int64_t m, int64_t n, int64_t lda, int64_t k, double delta,
                         const double *dU, const double *dS, const double *dVT, double broad,
                         double *dA)
{
    if (!A || !dU || !dS || !dVT || !dA || m < 1 || n < 1 || k < 1 || lda < n) return ORC_ERR_INVALID;
    int64_t mn = m < n ? m : n, kk = k < mn ? k : mn;
    double *U = (double *)malloc(sizeof(double) * m * kk);
    double *S = (double *)malloc(sizeof(double) * kk);
    double *VT = (double *)malloc(sizeof(double) * kk * n);
    double *sall = (double *)malloc(sizeof(double) * mn);
    double w;
    int64_t kp;
    /* full factors: U_f (m x mn), V_f (n x mn) from a full-rank truncation */
    double *Uf = (double *)malloc(sizeof(double) * m * mn);
    double *Sf = (double *)malloc(sizeof(double) * mn);
    double *VTf = (double *)malloc(sizeof(double) * mn * n);
    int rc = orc_fullsvd(A, m, n, lda, mn, 0.0, Uf, mn, Sf, VTf, n, &w, &kp, sall, NULL);
    int rc2 = orc_fullsvd(A, m, n, lda, k, delta, U, kk, S, VT, n, &w, &kp, NULL, NULL);
    if ((rc != ORC_OK && rc != ORC_ERR_NOCONV) || (rc2 != ORC_OK && rc2 != ORC_ERR_NOCONV)) {
        free(U); free(S); free(VT); free(sall); free(Uf); free(Sf); free(VTf);
        return rc != ORC_OK ? rc : rc2;
    }
    const double eps = broad * pow(Sf[0], 4);
    /* the kept triplets of the truncated call equal the leading ones of the full call */
    int tall = m > n;
    int64_t r = mn, c = tall ? m : n;
    double *Ut = (double *)malloc(sizeof(double) * r * r);
    double *Vt = (double *)malloc(sizeof(double) * c * r);
    double *Ub = (double *)calloc((size_t)(r * r), sizeof(double));
    double *Vb = (double *)calloc((size_t)(c * r), sizeof(double));
    double *sb = (double *)calloc((size_t)r, sizeof(double));
    double *Xb = (double *)malloc(sizeof(double) * r * c);
    /* wide form X = A (m <= n): Ut = U_f (m x m), Vt = V_f; tall form X = A^T: Ut = V_f, Vt = U_f */
    for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < r; ++j) Ut[i * r + j] = tall ? VTf[j * n + i] : Uf[i * mn + j];
    for (int64_t t = 0; t < c; ++t)
        for (int64_t j = 0; j < r; ++j) Vt[t * r + j] = tall ? Uf[t * mn + j] : VTf[j * n + t];
    for (int64_t j = 0; j < kp; ++j) {
        sb[j] = dS[j];
        if (!tall) {
            for (int64_t i = 0; i < m; ++i) Ub[i * r + j] = dU[i * kk + j];
            for (int64_t t = 0; t < n; ++t) Vb[t * r + j] = dVT[j * n + t];
        } else {
            for (int64_t i = 0; i < n; ++i) Ub[i * r + j] = dVT[j * n + i];
            for (int64_t t = 0; t < m; ++t) Vb[t * r + j] = dU[t * kk + j];
        }
    }
    svd_adjoint_wide(r, c, Ut, Sf, Vt, Ub, sb, Vb, eps, Xb);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) dA[i * n + j] = tall ? Xb[j * c + i] : Xb[i * c + j];
    free(U); free(S); free(VT); free(sall); free(Uf); free(Sf); free(VTf);
    free(Ut); free(Vt); free(Ub); free(Vb); free(sb); free(Xb);
    return ORC_OK;
}
