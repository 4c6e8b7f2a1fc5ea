// Host side of librsvd: problem validation, workspace layout, descriptor
// tables, the launch sequence of the RSVD (paper Sec. II.B, Alg. RSVD) and of
// the full-SVD truncation (Sec. II.A, Alg. TSVD), HIP-graph capture, the
// one-shot plan cache and the C ABI declared in include/librsvd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/librsvd.h"
#include "kernels.hpp"

using namespace rsvd;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return fail(RSVD_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Sweep caps of the block Jacobi.  The small SVD of B converges in 6-9 sweeps
// for l <= 272 on every workload measured (the last sweep only confirms
// convergence); wider sketches of steep spectra (l >= 288 with tails far below
// the working precision) need more.  Every sweep past convergence still costs
// one graph node per round (a few microseconds each), so the cap follows the
// widest sketch of the plan; a problem that reaches it reports
// RSVD_ERR_NOCONV with its results filled in.
constexpr int JAC_MAX_SWEEPS_RSVD = 14;
constexpr int JAC_MAX_SWEEPS_RSVD_WIDE = 30;
constexpr int JAC_WIDE_L = 272;
constexpr int JAC_MAX_SWEEPS_FULL = 30;
// The small SVD runs on the l x l triangular factor of B (B^T = Q_B R, Jacobi
// on R^T, V^T = W Q_B^T) instead of on B itself when n >= ratio * l: the Gram
// of the rows is the same (B B^T = R^T R), so the sweeps are the same, but
// every Jacobi round moves l + l instead of n + l columns per row, at the
// price of a Cholesky QR of the n x l matrix B^T and two small products.
// Measured per batch: 64 x 1024^2 FP32 at l = 144 (n = 7.1 l) 8.4 -> 7.7 ms;
// 32 x 500^2 at l = 110 (n = 4.5 l) 3.1 -> 2.9 ms; 32 x 512^2 at l = 272
// (n = 1.9 l) 8.33 -> 8.35 ms, even (the Jacobi saves what the extra QR
// costs), and even again with the faster Jacobi rounds (6.80 -> 6.85 ms:
// Jacobi 5.18 -> 4.59 ms, the QR of B^T and the products +0.63 ms); the
// 512-problem uneven batch with the cut at 1.5 l instead of 4 l 308 -> 270
// ms.  Plans without a saved forward only (the adjoint is that of the plain
// path).
constexpr double JAC_LQ_MIN_RATIO = 2.0;
// From this many row blocks on, rounds 2.. of every sweep rotate only the
// row pairs across the two blocks of a pair (half the inner steps): every
// block still gets a full inner sweep in round 0 or 1, so every pair of rows
// is visited at least once per sweep.  With fewer blocks this costs more extra
// sweeps than it saves.
constexpr int JAC_CROSS_MIN_NB = 16;
// The Jacobi phase runs as one persistent launch when a round has at most
// JAC_PERSISTENT_MAX_PAIRS block pairs over the whole plan (and the plan at
// most JAC_PERSISTENT_MAX_TASKS tasks), else round by round.  Measured inside
// HIP graphs: 1 x 128^2 (3 pairs per round) 1.29 -> 1.24 ms per step and
// 16 x 1024^2 at l = 80 (48 pairs) 3.27 -> 3.23 ms, where each round is far too
// small to fill the GPU and the launches dominate; 32 x 500^2 at l = 110 (128
// pairs) 2.90 -> 2.98 ms and 32 x 512^2 at l = 272 (256 pairs, one per
// compute unit) 8.93 -> 9.66 ms, where a round fills the GPU and the
// per-task release/acquire (an L2 write-back and invalidate on the XCD)
// costs more than the launch boundaries it replaces.
constexpr int JAC_PERSISTENT_MAX_PAIRS = 64;
// Plans with max(m, n) l^2 at least this large take the blocked Householder
// fallback: the one-workgroup form moves about 8 max(m, n) l^2 bytes per
// factorisation through one CU, while the blocked form costs two launches per
// 16-column panel even when no problem breaks down.
constexpr double HH_BLOCKED_MIN_COST = (double)(1 << 27);
constexpr int64_t JAC_PERSISTENT_MAX_TASKS = 1 << 18;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int elem_bytes(Elem e) { return e == E_F64 ? 8 : (e == E_F32 ? 4 : 2); }

// Byte blob holding every descriptor table and prefix array of a plan; the
// same layout is rebuilt for every execute, only pointers and scalars change.
struct Blob {
    std::vector<char> bytes;
    template <typename T> size_t add(const std::vector<T>& v)
    {
        size_t off = align_up(bytes.size(), 64);
        bytes.resize(off + v.size() * sizeof(T));
        if (!v.empty()) memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

struct ProbHost {
    int64_t m, n, lda, k, p, q, ldu, ldvt;
    uint64_t seed;
    double delta;
    int l;       // sketch width
    int R, C;    // Jacobi rows / columns
    int nb;      // Jacobi blocks (even)
    int mode;    // finish mode
    bool lq;     // small SVD of the triangular factor of B (see JAC_LQ_MIN_RATIO)
    // workspace offsets (bytes)
    size_t o_acast, o_om, o_m[2], o_q[2], o_g, o_l1, o_l2, o_b, o_p, o_sig, o_perm, o_norm, o_part,
        o_flags, o_rot, o_stats, o_info_local;
    std::vector<size_t> o_mstage, o_qstage, o_l1stage, o_l2stage;  // l1/l2: inverse Cholesky factors
    size_t o_lwork, o_dwork;
    size_t o_bt, o_qb;  // B^T = A^T Q and its orthonormal factor Q_B (n x R, FP64), lq problems only
    size_t o_kraw, o_kq;  // block-Krylov plans: the power bases side by side (m x R) and their orthonormal basis
    size_t o_sgn;  // k canonical signs written by the sign fix (0 beyond k_kept)
    // single-view plans: s = min(2 l + 1, m) rows of the co-range sketch; Psi^T (m x s),
    // W = Psi A (s x n), Z = Psi Q (s x l, then its orthonormal factor in place), L^-T (l x l),
    // Z^T W / its solve (l x n), F = A X^T (m x l), F^T Q (l x l), 2 sigma_i u_i^T A v_i (l)
    int sv_s = 0;
    size_t o_psi = 0, o_w = 0, o_z = 0, o_linv = 0, o_msv = 0, o_f = 0, o_ht = 0, o_cross = 0;
    // reverse pass (RSVD_PLAN_SAVE only)
    size_t o_bw_w[2], o_bw_vbt, o_bw_vts, o_bw_bb, o_bw_ut, o_bw_utb, o_bw_eu, o_bw_ev, o_bw_kp, o_bw_sb;
    // dA = Lcat Rcat^T: the 2q + 2 terms L_t R_t^T of the reverse pass side by side (m x (2q + 2) l, n x (2q + 2) l)
    size_t o_bw_lcat, o_bw_rcat;
    int nchunks;
};

struct GemmLaunch {
    GemmKind kind;
    GemmTile tile;
    bool gather;
    Elem ea, ex, ec;
    size_t off_desc, off_begin;
    int total;
    double flops;  // algorithmic 2 M N K summed over the problems
    int slot = -1;     // index among the plan's tunable forward launches, -1 if not tunable
    int cap = 0;       // workgroups reserved in the item map (the 64 x 64 count, the largest)
    uint64_t sig = 0;  // shape signature: kinds, element types and every problem's M, N, K, transposes
};

// Events around every launch of an eager execute (rsvd_plan_profile).
struct Profiler {
    std::vector<hipEvent_t> ev;
    std::vector<int> cat;
    std::vector<double> flops;
    size_t used = 0;
    hipStream_t s = nullptr;
    hipError_t begin(int c, double f)
    {
        if (ev.size() < 2 * (used + 1)) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreate(&a);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&b);
            if (e != hipSuccess) return e;
            ev.push_back(a);
            ev.push_back(b);
        }
        if (cat.size() < used + 1) {
            cat.push_back(c);
            flops.push_back(f);
        } else {
            cat[used] = c;
            flops[used] = f;
        }
        return hipEventRecord(ev[2 * used], s);
    }
    hipError_t end() { return hipEventRecord(ev[2 * used + 1], s), ++used, hipSuccess; }
    ~Profiler()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};
struct IdxLaunch {
    size_t off_desc, off_begin;
    int total;
};

// Private plan flag: the Gaussian test matrix is the real embedding of the
// complex circular Gaussian (the embedded problems of a complex plan).
constexpr unsigned PLAN_CPLX_OMEGA = 1u << 30;

}  // namespace

struct ComplexExt;

struct rsvd_plan {
    int nprob = 0;
    rsvd_dtype_t dt = RSVD_F64;
    rsvd_prec_t prec = RSVD_PREC_F64;
    unsigned flags = 0;
    bool fullsvd = false;
    bool complex_omega = false;  // embedded complex Gaussian (set on the inner plan of a complex plan)
    ComplexExt* cx = nullptr;    // RSVD_PLAN_COMPLEX: the embedded real plan and the complex finishing step
    std::vector<ProbHost> probs;
    int max_l = 0, max_nb = 2, max_q = 0;
    int jac_variant = 0;
    bool krylov = false;          // block-Krylov variant (RSVD_PLAN_BLOCK_KRYLOV)
    std::vector<IdxLaunch> kcopy; // per stage: copy of the stage's basis into the Krylov block (even stages)
    GemmLaunch g_kgram1, g_kgram2;
    IdxLaunch k_qr[2], k_trsm[2];
    bool single_view = false;     // single-view variant (RSVD_PLAN_SINGLE_VIEW)
    int fp64_from = 1 << 30;      // RSVD_PLAN_FP64_FINAL: the first stage whose products are FP64
    IdxLaunch omega_psi, sv_qr, sv_trsm_z, sv_trsm_i, sv_eye, sv_cross;
    GemmLaunch g_sv_w, g_sv_z, g_sv_gram, g_sv_m, g_sv_x, g_sv_f, g_sv_ht;
    bool hh_blocked = false;      // the Householder fallback runs in blocked form
    int hh_rows = 0;              // largest number of rows of any orthonormalised basis
    bool jac_persistent = false;  // the Jacobi phase is one persistent launch
    int jac_grid = 0;             // its workgroups
    size_t off_sched = 0;         // its task counter and error flag (2 ints, cleared every execute)
    int max_sweeps = 20;
    Elem e_store = E_F64, e_sketch = E_F64, e_y = E_F64;
    bool need_cast = false;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    size_t off_one = 0;  // an int that is always 1 (static skip)
    // descriptor blob
    Blob hb;
    char* dblob = nullptr;
    char* hblob_pinned = nullptr;
    size_t blob_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    // recorded launch layout (offsets into the blob)
    IdxLaunch stage, omega, copy, eye, finish, fin_norm, fin_vt, fin_u, signfix;
    std::vector<GemmLaunch> g_sketch, g_gram1, g_gram2;
    std::vector<IdxLaunch> qr, trsm;
    GemmLaunch g_b, g_u;
    // triangular-factor small SVD (lq problems): B^T = A^T Q, its Cholesky QR, V^T = W Q_B^T
    bool any_lq = false;
    GemmLaunch g_lqbt, g_lqgram1, g_lqgram2, g_lqx, g_lqvt;
    IdxLaunch lq_qr[2], lq_trsm[2];
    IdxLaunch jac;
    int total_flags = 0;
    size_t off_flags_base = 0;
    // last pointers used to build the blob
    std::vector<const void*> lastA;
    std::vector<void*> lastU, lastS, lastVT;
    double* lastW = nullptr;
    int64_t* lastK = nullptr;
    int* lastInfo = nullptr;
    bool blob_valid = false;
    // graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    Profiler* prof = nullptr;  // set only during rsvd_plan_profile
    uint64_t fwd_gen = 0;      // bumped whenever the forward descriptors are rebuilt
    bool fwd_saved = false;    // a forward execute of a RSVD_PLAN_SAVE plan was enqueued
    // tile autotuning (RSVD_PLAN_TUNE): per tunable forward launch, the tile in use
    // and the tuned override (-1: the shape heuristic)
    std::vector<int> slot_tile, tile_ovr;
    bool tuner = false;  // the eager execute under way times the candidate tiles
    bool tuned = false;
    struct BwStage {
        GemmLaunch c, qs, r, qprev;
        IdxLaunch sym, tri, trsm;
        IdxLaunch cat_l, cat_r;  // the stage's dA term L R^T copied into its slices of Lcat, Rcat
    };
    struct Backward {
        Blob hb;
        char* dblob = nullptr;
        char* hpinned = nullptr;
        size_t bytes = 0;
        hipEvent_t upload_done = nullptr;
        bool upload_pending = false;
        bool valid = false;
        uint64_t gen = 0;
        std::vector<const void*> ldU, ldS, ldVT;
        std::vector<void*> ldA;
        double broad = 0.0;
        IdxLaunch prep, core;
        GemmLaunch utb, qb0, eu, ev, nn, bb, qba;
        IdxLaunch cat_l0, cat_r0;  // the head's dA term Q Bbar into slice 0
        GemmLaunch da;             // dA = Lcat Rcat^T, every term in one product
        std::vector<BwStage> st;  // indexed by stage
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
    } bw;
};

namespace {

int validate_problem(const rsvd_problem_t& p, bool fullsvd)
{
    if (p.m < 1 || p.n < 1 || p.k < 1) return fail(RSVD_ERR_INVALID, "m, n and k must be >= 1");
    if (p.m > (1 << 24) || p.n > (1 << 24)) return fail(RSVD_ERR_INVALID, "m or n too large");
    if (p.lda < p.n) return fail(RSVD_ERR_INVALID, "lda < n");
    if (!fullsvd && (p.p < 0 || p.q < 0)) return fail(RSVD_ERR_INVALID, "p and q must be >= 0");
    if (!fullsvd && p.q > 64) return fail(RSVD_ERR_INVALID, "q > 64");
    if (!(p.delta_trunc >= 0.0)) return fail(RSVD_ERR_INVALID, "delta_trunc must be >= 0 and not NaN");
    int64_t mn = std::min(p.m, p.n);
    int64_t kk = std::min(p.k, mn);
    if (p.ldu != 0 && p.ldu < kk) return fail(RSVD_ERR_INVALID, "ldu < k");
    if (p.ldvt != 0 && p.ldvt < p.n) return fail(RSVD_ERR_INVALID, "ldvt < n");
    if (fullsvd && mn > 2048) return fail(RSVD_ERR_INVALID, "full SVD supports min(m, n) <= 2048");
    if (!fullsvd) {
        int64_t l = std::min(kk + p.p, mn);
        if (l > 1024) return fail(RSVD_ERR_INVALID, "k + p must be <= 1024");
    }
    return RSVD_OK;
}

Elem store_elem(rsvd_dtype_t dt) { return dt == RSVD_F64 ? E_F64 : E_F32; }

// ---------------------------------------------------------------- workspace layout
void layout(rsvd_plan& P)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    P.off_one = take(sizeof(int));
    const bool save = (P.flags & RSVD_PLAN_SAVE) != 0;
    P.total_flags = 0;
    for (auto& h : P.probs) {
        const int64_t m = h.m, n = h.n, l = h.l;
        const int64_t lw = std::max<int64_t>(l, h.R);  // widest basis orthonormalised (the Krylov block)
        h.nchunks = (int)((m + STAGE_ROWS - 1) / STAGE_ROWS);
        h.o_norm = take(sizeof(double));
        h.o_part = take(sizeof(double) * h.nchunks);
        h.o_sig = take(sizeof(double) * h.R);
        h.o_perm = take(sizeof(int) * h.R);
        h.o_p = take(sizeof(double) * (size_t)h.R * h.R);
        h.o_info_local = take(sizeof(int));
        h.o_sgn = take(sizeof(double) * h.k);
        if (P.fullsvd) {
            h.o_b = take(sizeof(double) * (size_t)h.R * h.C);
            continue;
        }
        h.o_acast = P.need_cast ? take((size_t)elem_bytes(P.e_sketch) * m * n) : 0;
        h.o_om = take((size_t)elem_bytes(P.e_sketch) * n * l);
        const int nst = (int)(2 * h.q + 1);
        h.o_mstage.assign(nst, 0);
        h.o_qstage.assign(nst, 0);
        h.o_l1stage.assign(nst, 0);
        h.o_l2stage.assign(nst, 0);
        size_t shared_m[2], shared_q[2], sl1 = 0, sl2 = 0;
        h.o_lwork = take(sizeof(double) * lw * lw);
        h.o_dwork = take(sizeof(double) * ((lw + 15) / 16) * 256);
        if (!save) {
            // FP64 final power step: the shared buffers also hold FP64 products
            const size_t ey = P.fp64_from <= 2 * P.max_q ? sizeof(double) : (size_t)elem_bytes(P.e_y);
            shared_m[0] = take(ey * m * l);
            shared_m[1] = take(ey * n * l);
            shared_q[0] = take(sizeof(double) * m * l);
            shared_q[1] = take(sizeof(double) * n * l);
            sl1 = take(sizeof(double) * l * l);
            sl2 = take(sizeof(double) * l * l);
        }
        for (int s = 0; s < nst; ++s) {
            const int64_t rows = (s % 2 == 0) ? m : n;
            if (save) {
                h.o_mstage[s] = take((size_t)elem_bytes(P.e_y) * rows * l);
                h.o_qstage[s] = take(sizeof(double) * rows * l);
                h.o_l1stage[s] = take(sizeof(double) * l * l);
                h.o_l2stage[s] = take(sizeof(double) * l * l);
            } else {
                h.o_mstage[s] = shared_m[s % 2];
                h.o_qstage[s] = shared_q[s % 2];
                h.o_l1stage[s] = sl1;
                h.o_l2stage[s] = sl2;
            }
        }
        h.o_g = take(sizeof(double) * lw * lw);
        h.o_b = take(sizeof(double) * (size_t)h.R * h.C);
        h.o_bt = h.lq ? take(sizeof(double) * n * h.R) : 0;
        h.o_qb = h.lq ? take(sizeof(double) * n * h.R) : 0;
        h.o_kraw = P.krylov ? take(sizeof(double) * m * h.R) : 0;
        h.o_kq = P.krylov ? take(sizeof(double) * m * h.R) : 0;
        if (P.single_view) {
            const int64_t sv = h.sv_s, R = h.R;
            h.o_psi = take(sizeof(double) * m * sv);
            h.o_w = take(sizeof(double) * sv * n);
            h.o_z = take(sizeof(double) * sv * R);
            h.o_linv = take(sizeof(double) * R * R);
            h.o_msv = take(sizeof(double) * R * n);
            h.o_f = take(sizeof(double) * m * R);
            h.o_ht = take(sizeof(double) * R * R);
            h.o_cross = take(sizeof(double) * R);
        }
        if (save) {
            const int64_t mx = std::max(m, n);
            h.o_bw_w[0] = take(sizeof(double) * mx * l);
            h.o_bw_w[1] = take(sizeof(double) * mx * l);
            h.o_bw_vbt = take(sizeof(double) * l * n);
            h.o_bw_vts = take(sizeof(double) * l * n);
            h.o_bw_bb = take(sizeof(double) * l * n);
            h.o_bw_ut = take(sizeof(double) * l * l);
            h.o_bw_utb = take(sizeof(double) * l * l);
            h.o_bw_eu = take(sizeof(double) * l * l);
            h.o_bw_ev = take(sizeof(double) * l * l);
            h.o_bw_kp = take(sizeof(double) * l * l);
            h.o_bw_sb = take(sizeof(double) * l);
            const int64_t tl = (2 * h.q + 2) * l;
            h.o_bw_lcat = take(sizeof(double) * m * tl);
            h.o_bw_rcat = take(sizeof(double) * n * tl);
        }
    }
    // flags: per problem (2 q_max + 1) QR flags followed by max_sweeps rot flags
    P.off_flags_base = take(0);
    // per problem: 2 q_max + 1 stage QR flags, the lq factorisation's, the
    // Krylov block's, then the sweeps' rotation flags and four Jacobi counters
    const int per = (int)(2 * P.max_q + 3) + P.max_sweeps + 4;
    for (size_t b = 0; b < P.probs.size(); ++b) {
        P.probs[b].o_flags = P.off_flags_base + sizeof(int) * (size_t)per * b;
        P.probs[b].o_rot = P.probs[b].o_flags + sizeof(int) * (size_t)(2 * P.max_q + 3);
        P.probs[b].o_stats = P.probs[b].o_rot + sizeof(int) * (size_t)P.max_sweeps;
    }
    P.off_sched = P.off_flags_base + sizeof(int) * (size_t)per * P.probs.size();
    P.total_flags = per * (int)P.probs.size() + 2;
    off = align_up(P.off_flags_base + sizeof(int) * (size_t)P.total_flags, 256);
    P.ws_bytes = off;
}

template <typename T> T* wsp(const rsvd_plan& P, size_t off) { return (T*)(P.ws + off); }

// Element of a stage's product M (the sketch precision's, or FP64 for the
// stages of an FP64 final power step).
Elem stage_y(const rsvd_plan& P, int s) { return s >= P.fp64_from ? E_F64 : P.e_y; }

int tiles_of(int M, int N, GemmTile t)
{
    const int bm = gemm_tile_m(t), bn = gemm_tile_n(t);
    return ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
}

// Workgroup tile of a GEMM launch: 128 x 64 for tall, narrow products with
// enough tiles to fill the GPU twice over, else 64 x 64.
GemmTile choose_tile(const std::vector<GemmDesc>& descs)
{
    int64_t tiles128 = 0;
    bool tall = true;
    for (const GemmDesc& d : descs) {
        if (d.A == nullptr || d.M <= 0 || d.N <= 0) continue;
        tiles128 += tiles_of(d.M, d.N, GT_128x64);
        if (!(d.M >= 512 && d.N <= 160)) tall = false;
    }
    return (tall && tiles128 >= 512) ? GT_128x64 : GT_64x64;
}

// Work-item map of a batched launch: entry t = (problem, local item) for
// workgroup t, problems in order, count[b] items each.
std::vector<int> item_map(const std::vector<int>& counts)
{
    std::vector<int> map;
    for (size_t b = 0; b < counts.size(); ++b)
        for (int i = 0; i < counts[b]; ++i) {
            map.push_back((int)b);
            map.push_back(i);
        }
    if (map.empty()) map.assign(2, 0);
    return map;
}

// Tile-dependent fields of a launch's descriptors (tiles_n, lower) and each
// problem's workgroup count.
std::vector<int> finalize_descs(std::vector<GemmDesc>& descs, GemmTile tile, int* total)
{
    std::vector<int> counts(descs.size(), 0);
    *total = 0;
    for (size_t b = 0; b < descs.size(); ++b) {
        GemmDesc& d = descs[b];
        int t = 0;
        if (d.lower && (tile != GT_64x64 || d.M != d.N)) d.lower = 0;  // lower-only needs square tiles
        if (d.M > 0 && d.N > 0 && d.K >= 0 && d.A != nullptr) t = tiles_of(d.M, d.N, tile);
        d.tiles_n = (d.N + gemm_tile_n(tile) - 1) / gemm_tile_n(tile);
        if (d.lower && t > 0) t = d.tiles_n * (d.tiles_n + 1) / 2;
        counts[b] = t;
        *total += t;
    }
    return counts;
}

// FNV-1a over the fields that decide a launch's cost: kinds, element types
// and every problem's shape and transposes (not its pointers).
uint64_t gemm_signature(GemmKind kind, Elem ea, Elem ex, Elem ec, const std::vector<GemmDesc>& descs)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](int64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (uint64_t)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(kind), mix(ea), mix(ex), mix(ec), mix((int64_t)descs.size());
    for (const GemmDesc& d : descs) {
        const bool live = d.A != nullptr && d.M > 0 && d.N > 0;
        mix(live ? d.M : 0), mix(live ? d.N : 0), mix(live ? d.K : 0);
        mix(live ? d.transA * 4 + d.transX * 2 + d.transC : 0);
    }
    return h;
}

// forced >= 0 fixes the tile of a tunable launch (slot >= 0: no gathered,
// accumulating or lower-only product); the item map of a tunable launch is
// sized for the 64 x 64 tiling so that any tile fits the same blob layout.
GemmLaunch add_gemm(Blob& B, GemmKind kind, Elem ea, Elem ex, Elem ec, std::vector<GemmDesc>& descs,
                    int slot = -1, int forced = -1)
{
    bool gather = false, special = false;
    for (const GemmDesc& d : descs) {
        gather = gather || (d.A != nullptr && d.gather != nullptr);
        special = special || (d.A != nullptr && (d.lower || d.accumulate));
    }
    const bool tunable = slot >= 0 && !gather && !special;
    GemmTile tile = gather ? GT_64x64 : choose_tile(descs);
    if (tunable && forced >= 0) tile = (GemmTile)forced;
    GemmLaunch g;
    if (tunable) {
        g.sig = gemm_signature(kind, ea, ex, ec, descs);
        for (const GemmDesc& d : descs)
            if (d.M > 0 && d.N > 0 && d.K >= 0 && d.A != nullptr) g.cap += tiles_of(d.M, d.N, GT_64x64);
    }
    int total = 0;
    const std::vector<int> counts = finalize_descs(descs, tile, &total);
    std::vector<int> map = item_map(counts);
    if (tunable && map.size() < 2 * (size_t)g.cap) map.resize(2 * (size_t)g.cap, 0);
    g.kind = kind;
    g.tile = tile;
    g.gather = gather;
    g.ea = ea;
    g.ex = ex;
    g.ec = ec;
    g.off_desc = B.add(descs);
    g.off_begin = B.add(map);
    g.total = total;
    g.slot = tunable ? slot : -1;
    g.flops = 0.0;
    for (const GemmDesc& d : descs)
        if (d.A != nullptr) g.flops += d.lower ? (double)d.M * (d.M + 1) * d.K : 2.0 * d.M * d.N * d.K;
    return g;
}

template <typename D> IdxLaunch add_idx(Blob& B, const std::vector<D>& descs, const std::vector<int>& counts)
{
    IdxLaunch L;
    L.off_desc = B.add(descs);
    L.off_begin = B.add(item_map(counts));
    L.total = 0;
    for (int c : counts) L.total += c;
    return L;
}

GemmDesc gd(const void* A, int64_t lda, int transA, const void* X, int64_t ldx, int transX, void* C,
            int64_t ldc, int M, int N, int K, const int* skip = nullptr, const int* gather = nullptr)
{
    GemmDesc d;
    memset(&d, 0, sizeof(d));
    d.A = A;
    d.lda = lda;
    d.transA = transA;
    d.X = X;
    d.ldx = ldx;
    d.transX = transX;
    d.C = C;
    d.ldc = ldc;
    d.M = M;
    d.N = N;
    d.K = K;
    d.skip = skip;
    d.gather = gather;
    return d;
}

// Compute units of the current device (queried once per device).
int compute_units()
{
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cus.find(dev);
    if (it == cus.end()) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        it = cus.emplace(dev, n).first;
    }
    return it->second;
}

// Resident workgroups per compute unit of the persistent Jacobi kernel variant.
int persistent_blocks_per_cu(int variant)
{
    static std::mutex mu;
    static std::map<int, int> per;
    std::lock_guard<std::mutex> lk(mu);
    auto it = per.find(variant);
    if (it == per.end()) it = per.emplace(variant, jacobi_persistent_blocks_per_cu(variant)).first;
    return it->second;
}

// The basis the small SVD is projected on (m x R, FP64): the last stage's
// basis, or the orthonormalised block-Krylov block.
const double* final_q(const rsvd_plan& P, const ProbHost& h)
{
    return P.krylov ? wsp<double>(P, h.o_kq) : wsp<double>(P, h.o_qstage[2 * h.q]);
}

// Builds every descriptor table for the given user pointers.
void build_blob(rsvd_plan& P, const void* const* A, void* const* U, void* const* S, void* const* VT,
                double* w, int64_t* kk, int* info)
{
    Blob B;
    const int np = P.nprob;
    const int* one = wsp<int>(P, P.off_one);
    const Elem es = P.e_store;
    const int out_f64 = (P.dt == RSVD_F64);
    (void)out_f64;
    // forward products whose tile the autotuner may choose, numbered in build order
    int nslot = 0;
    P.slot_tile.clear();
    auto tgemm = [&](GemmKind kind, Elem ea, Elem ex, Elem ec, std::vector<GemmDesc>& d) {
        const int slot = nslot++;
        const int forced = slot < (int)P.tile_ovr.size() ? P.tile_ovr[slot] : -1;
        GemmLaunch g = add_gemm(B, kind, ea, ex, ec, d, slot, forced);
        P.slot_tile.push_back(g.slot >= 0 ? (int)g.tile : -1);
        return g;
    };

    // staging: ||A||^2 and the optional cast
    {
        std::vector<StageDesc> d(np);
        std::vector<int> cnt(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            StageDesc& s = d[b];
            memset(&s, 0, sizeof(s));
            s.A = A[b];
            s.Acast = (!P.fullsvd && P.need_cast) ? (void*)wsp<char>(P, h.o_acast) : nullptr;
            s.partial = wsp<double>(P, h.o_part);
            s.normA2 = wsp<double>(P, h.o_norm);
            s.lda = h.lda;
            s.m = (int)h.m;
            s.n = (int)h.n;
            s.a_elem = es;
            s.cast_elem = P.e_sketch;
            s.nchunks = h.nchunks;
            cnt[b] = h.nchunks;
        }
        P.stage = add_idx(B, d, cnt);
    }
    if (!P.fullsvd) {
        // Gaussian test matrices
        {
            std::vector<OmegaDesc> d(np);
            std::vector<int> cnt(np);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                OmegaDesc& o = d[b];
                memset(&o, 0, sizeof(o));
                o.Om = wsp<char>(P, h.o_om);
                o.seed = h.seed;
                o.n = (int)h.n;
                o.l = h.l;
                o.elem = P.e_sketch;
                const int64_t pairs = ((h.n + 1) / 2) * (int64_t)h.l;
                cnt[b] = (int)((pairs + 255) / 256);
                if (P.complex_omega) {  // the embedded problem of an m x n complex one: n and l are doubled
                    o.n = (int)(h.n / 2);
                    o.l = h.l / 2;
                    o.complex_embed = 1;
                    cnt[b] = (int)(((int64_t)o.n * o.l + 255) / 256);
                }
            }
            P.omega = add_idx(B, d, cnt);
        }
        // single-view plans: the co-range test matrix, stored as Psi^T = the m x s
        // Gaussian of the seed with its top bit flipped (FP64)
        if (P.single_view) {
            std::vector<OmegaDesc> d(np);
            std::vector<int> cnt(np);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                OmegaDesc& o = d[b];
                memset(&o, 0, sizeof(o));
                o.Om = wsp<char>(P, h.o_psi);
                o.seed = h.seed ^ (1ull << 63);
                o.n = (int)h.m;
                o.l = h.sv_s;
                o.elem = E_F64;
                const int64_t pairs = ((h.m + 1) / 2) * (int64_t)h.sv_s;
                cnt[b] = (int)((pairs + 255) / 256);
            }
            P.omega_psi = add_idx(B, d, cnt);
        }
        const GemmKind gk = P.prec == RSVD_PREC_F64 ? GK_F64 : (P.prec == RSVD_PREC_F32 ? GK_F32 : GK_BF16);
        const Elem ea_sk = P.need_cast ? P.e_sketch : es;
        const int nst = 2 * P.max_q + 1;
        P.g_sketch.clear();
        P.g_gram1.clear();
        P.g_gram2.clear();
        P.qr.clear();
        P.trsm.clear();
        P.kcopy.clear();
        for (int s = 0; s < nst; ++s) {
            std::vector<GemmDesc> dsk(np), dg1(np), dg2(np);
            std::vector<QrDesc> dq(np), dq2(np);
            std::vector<int> rowblk(np, 0), rowblk2(np, 0);
            const GemmDesc none = gd(nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 0, 0, one);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                const int l = h.l;
                const bool active = s <= 2 * h.q;
                const bool final_stage = s == 2 * h.q;
                const int64_t rows = (s % 2 == 0) ? h.m : h.n;
                memset(&dq[b], 0, sizeof(QrDesc));
                dq[b].flag = const_cast<int*>(one);
                dq[b].l = l;
                dq2[b] = dq[b];
                dsk[b] = dg1[b] = dg2[b] = none;
                if (!active) continue;
                // the FP64 stages read the stored A, the others the sketch precision's copy
                const bool cast = P.need_cast && s < P.fp64_from;
                const void* Aop = cast ? (const void*)wsp<char>(P, h.o_acast) : A[b];
                const int64_t lda_op = cast ? h.n : h.lda;
                void* M = wsp<char>(P, h.o_mstage[s]);
                double* Qs = wsp<double>(P, h.o_qstage[s]);
                int* flag = wsp<int>(P, h.o_flags) + s;
                double* G = wsp<double>(P, h.o_g);
                if (s == 0) {
                    dsk[b] = gd(Aop, lda_op, 0, wsp<char>(P, h.o_om), l, 0, M, l, (int)h.m, l, (int)h.n);
                } else if (s % 2 == 1) {
                    dsk[b] = gd(Aop, lda_op, 1, wsp<double>(P, h.o_qstage[s - 1]), l, 0, M, l, (int)h.n, l,
                                (int)h.m);
                } else {
                    dsk[b] = gd(Aop, lda_op, 0, wsp<double>(P, h.o_qstage[s - 1]), l, 0, M, l, (int)h.m, l,
                                (int)h.n);
                }
                // pass 1: G = M^T M, L L^T = G, Q = M L^-T
                // only the lower triangle of a Gram matrix is read (by the Cholesky)
                dg1[b] = gd(M, l, 1, M, l, 0, G, l, l, l, (int)rows, flag);
                dg1[b].lower = 1;
                QrDesc& q = dq[b];
                q.Min = M;
                q.Qout = Qs;
                q.G = G;
                q.L = wsp<double>(P, h.o_lwork);
                q.D = wsp<double>(P, h.o_dwork);
                q.flag = flag;
                q.rows = (int)rows;
                q.min_elem = stage_y(P, s);
                rowblk[b] = (int)((rows + 15) / 16);
                // pass 2 (final basis only), in place: G = Q^T Q, Q = Q L2^-T
                if (final_stage) {
                    dg2[b] = gd(Qs, l, 1, Qs, l, 0, G, l, l, l, (int)rows, flag);
                    dg2[b].lower = 1;
                    dq2[b] = q;
                    rowblk2[b] = rowblk[b];
                }
            }
            // X operand element of the sketch GEMMs: Omega at s = 0, FP64 bases afterwards
            if (s >= P.fp64_from)
                P.g_sketch.push_back(tgemm(GK_F64, es, E_F64, E_F64, dsk));
            else
                P.g_sketch.push_back(tgemm(gk, ea_sk, s == 0 ? P.e_sketch : E_F64, P.e_y, dsk));
            P.g_gram1.push_back(add_gemm(B, GK_F64, stage_y(P, s), stage_y(P, s), E_F64, dg1));
            P.g_gram2.push_back(add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dg2));
            std::vector<int> ones(np, 1);
            P.qr.push_back(add_idx(B, dq, ones));
            P.qr.push_back(add_idx(B, dq2, ones));
            P.trsm.push_back(add_idx(B, dq, rowblk));
            P.trsm.push_back(add_idx(B, dq2, rowblk2));
            // block-Krylov plans: basis j = s / 2 of an even stage goes to columns
            // j l .. of the Krylov block (its first R = min(l (q + 1), m, n) columns)
            std::vector<CopyDesc> dc(np);
            std::vector<int> cc(np, 0);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                CopyDesc& c = dc[b];
                memset(&c, 0, sizeof(c));
                const int c0 = (s / 2) * h.l, ncols = std::min(h.l, h.R - c0);
                if (!P.krylov || s % 2 == 1 || s > 2 * h.q || ncols <= 0) continue;
                c.A = wsp<double>(P, h.o_qstage[s]);
                c.X = wsp<double>(P, h.o_kraw) + c0;
                c.lda = h.l;
                c.ldx = h.R;
                c.m = (int)h.m;
                c.n = ncols;
                c.a_elem = E_F64;
                c.transpose = 0;
                cc[b] = (int)(((h.m + 63) / 64) * ((ncols + 63) / 64));
            }
            P.kcopy.push_back(add_idx(B, dc, cc));
        }
        // block-Krylov plans: the Krylov block K = Q_K R_K by Cholesky QR twice
        // (Householder on breakdown); Q_K is the basis of the projection
        if (P.krylov) {
            std::vector<GemmDesc> dg1(np), dg2(np);
            std::vector<QrDesc> dq(np), dq2(np);
            std::vector<int> rowblk(np), ones(np, 1);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                const int L = h.R;
                double* K = wsp<double>(P, h.o_kraw);
                double* Qk = wsp<double>(P, h.o_kq);
                double* G = wsp<double>(P, h.o_g);
                int* flag = wsp<int>(P, h.o_flags) + 2 * P.max_q + 2;
                dg1[b] = gd(K, L, 1, K, L, 0, G, L, L, L, (int)h.m, flag);
                dg1[b].lower = 1;
                dg2[b] = gd(Qk, L, 1, Qk, L, 0, G, L, L, L, (int)h.m, flag);
                dg2[b].lower = 1;
                QrDesc& q = dq[b];
                memset(&q, 0, sizeof(q));
                q.Min = K;
                q.Qout = Qk;
                q.G = G;
                q.L = wsp<double>(P, h.o_lwork);
                q.D = wsp<double>(P, h.o_dwork);
                q.flag = flag;
                q.rows = (int)h.m;
                q.l = L;
                q.min_elem = E_F64;
                dq2[b] = q;
                rowblk[b] = (int)((h.m + 15) / 16);
            }
            P.g_kgram1 = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dg1);
            P.g_kgram2 = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dg2);
            P.k_qr[0] = add_idx(B, dq, ones);
            P.k_qr[1] = add_idx(B, dq2, ones);
            P.k_trsm[0] = add_idx(B, dq, rowblk);
            P.k_trsm[1] = add_idx(B, dq2, rowblk);
        }
        // lq problems: B^T = A^T Q (FP64 from the stored A) and its Cholesky QR
        // (two passes, Householder on breakdown), B^T = Q_B R
        P.any_lq = false;
        for (const ProbHost& h : P.probs) P.any_lq = P.any_lq || h.lq;
        if (P.any_lq) {
            std::vector<GemmDesc> dbt(np), dg1(np), dg2(np);
            std::vector<QrDesc> dq(np), dq2(np);
            std::vector<int> rowblk(np, 0), rowblk2(np, 0), ones(np, 1);
            const GemmDesc none = gd(nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 0, 0, one);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                const int l = h.R;  // width of the final basis
                memset(&dq[b], 0, sizeof(QrDesc));
                dq[b].flag = const_cast<int*>(one);
                dq[b].l = l;
                dq2[b] = dq[b];
                dbt[b] = dg1[b] = dg2[b] = none;
                if (!h.lq) continue;
                double* Bt = wsp<double>(P, h.o_bt);
                double* Qb = wsp<double>(P, h.o_qb);
                double* G = wsp<double>(P, h.o_g);
                int* flag = wsp<int>(P, h.o_flags) + 2 * P.max_q + 1;
                dbt[b] = gd(A[b], h.lda, 1, final_q(P, h), l, 0, Bt, l, (int)h.n, l, (int)h.m);
                dg1[b] = gd(Bt, l, 1, Bt, l, 0, G, l, l, l, (int)h.n, flag);
                dg1[b].lower = 1;
                QrDesc& q = dq[b];
                q.Min = Bt;
                q.Qout = Qb;
                q.G = G;
                q.L = wsp<double>(P, h.o_lwork);
                q.D = wsp<double>(P, h.o_dwork);
                q.flag = flag;
                q.rows = (int)h.n;
                q.min_elem = E_F64;
                rowblk[b] = (int)((h.n + 15) / 16);
                dg2[b] = gd(Qb, l, 1, Qb, l, 0, G, l, l, l, (int)h.n, flag);
                dg2[b].lower = 1;
                dq2[b] = q;
                rowblk2[b] = rowblk[b];
            }
            P.g_lqbt = tgemm(GK_F64, es, E_F64, E_F64, dbt);
            P.g_lqgram1 = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dg1);
            P.g_lqgram2 = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dg2);
            P.lq_qr[0] = add_idx(B, dq, ones);
            P.lq_qr[1] = add_idx(B, dq2, ones);
            P.lq_trsm[0] = add_idx(B, dq, rowblk);
            P.lq_trsm[1] = add_idx(B, dq2, rowblk2);
        }
        // lq problems: the Jacobi input is R^T = B Q_B = (B^T)^T Q_B (l x l, FP64 operands)
        if (P.any_lq) {
            const GemmDesc none = gd(nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 0, 0, one);
            std::vector<GemmDesc> dx(np, none);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                if (h.lq)
                    dx[b] = gd(wsp<double>(P, h.o_bt), h.R, 1, wsp<double>(P, h.o_qb), h.R, 0, wsp<double>(P, h.o_b),
                               h.R, h.R, h.R, (int)h.n);
            }
            P.g_lqx = tgemm(GK_F64, E_F64, E_F64, E_F64, dx);
        }
        // single-view plans: W = Psi A and Z = Psi Q (FP64), the Cholesky factor L of
        // Z^T Z, Z <- Z L^-T and L^-T (in place on the identity), M = Z^T W, and the
        // Jacobi input X = L^-T M = (Z^T Z)^-1 Z^T W = (Psi Q)^+ W
        if (P.single_view) {
            std::vector<GemmDesc> dw(np), dz(np), dg(np), dm(np), dx(np);
            std::vector<QrDesc> dq(np), dqi(np);
            std::vector<EyeDesc> de(np);
            std::vector<int> ones(np, 1), rowblk(np), rowblki(np), ce(np);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                const int R = h.R, sv = h.sv_s;
                const double* G = wsp<double>(P, h.o_psi);
                double* W = wsp<double>(P, h.o_w);
                double* Z = wsp<double>(P, h.o_z);
                double* Li = wsp<double>(P, h.o_linv);
                double* M = wsp<double>(P, h.o_msv);
                int* flag = wsp<int>(P, h.o_flags) + 2 * P.max_q + 1;  // the lq slot (single-view plans have no lq)
                dw[b] = gd(G, sv, 1, A[b], h.lda, 0, W, h.n, sv, (int)h.n, (int)h.m);
                dz[b] = gd(G, sv, 1, final_q(P, h), R, 0, Z, R, sv, R, (int)h.m);
                dg[b] = gd(Z, R, 1, Z, R, 0, wsp<double>(P, h.o_g), R, R, R, sv, flag);
                dg[b].lower = 1;
                QrDesc& q = dq[b];
                memset(&q, 0, sizeof(q));
                q.Min = Z;
                q.Qout = Z;
                q.G = wsp<double>(P, h.o_g);
                q.L = wsp<double>(P, h.o_lwork);
                q.D = wsp<double>(P, h.o_dwork);
                q.flag = flag;
                q.rows = sv;
                q.l = R;
                q.min_elem = E_F64;
                dqi[b] = q;
                dqi[b].Min = Li;
                dqi[b].Qout = Li;
                dqi[b].rows = R;
                rowblk[b] = (sv + 15) / 16;
                rowblki[b] = (R + 15) / 16;
                EyeDesc& e = de[b];
                memset(&e, 0, sizeof(e));
                e.P = Li;
                e.ldp = R;
                e.R = R;
                ce[b] = (int)(((int64_t)R * R + 255) / 256);
                dm[b] = gd(Z, R, 1, W, h.n, 0, M, h.n, R, (int)h.n, sv, flag);
                dx[b] = gd(Li, R, 0, M, h.n, 0, wsp<double>(P, h.o_b), h.C, R, (int)h.n, R, flag);
            }
            P.g_sv_w = add_gemm(B, GK_F64, E_F64, es, E_F64, dw);
            P.g_sv_z = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dz);
            P.g_sv_gram = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dg);
            P.sv_qr = add_idx(B, dq, ones);
            P.sv_eye = add_idx(B, de, ce);
            P.sv_trsm_z = add_idx(B, dq, rowblk);
            P.sv_trsm_i = add_idx(B, dqi, rowblki);
            P.g_sv_m = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dm);
            P.g_sv_x = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dx);
        }
        // B = Q^T A in FP64 from the stored A (the other problems)
        {
            std::vector<GemmDesc> d(np);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                const double* Qf = final_q(P, h);
                if (h.lq)
                    d[b] = gd(nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 0, 0, one);
                else
                    d[b] = gd(Qf, h.R, 1, A[b], h.lda, 0, wsp<double>(P, h.o_b), h.n, h.R, (int)h.n, (int)h.m);
            }
            if ((P.flags & RSVD_PLAN_NO_REFINE) && P.prec != RSVD_PREC_F64) {
                // B = Q^T A with the sketch arithmetic (operands rounded on load)
                for (int b = 0; b < np; ++b) {
                    const ProbHost& h = P.probs[b];
                    if (P.need_cast) {
                        d[b].X = wsp<char>(P, h.o_acast);
                        d[b].ldx = h.n;
                    }
                }
                const GemmKind gk2 = P.prec == RSVD_PREC_F32 ? GK_F32 : GK_BF16;
                P.g_b = tgemm(gk2, E_F64, P.need_cast ? P.e_sketch : es, E_F64, d);
            } else {
                P.g_b = tgemm(GK_F64, E_F64, es, E_F64, d);
            }
        }
    } else {
        std::vector<CopyDesc> d(np);
        std::vector<int> cnt(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            CopyDesc& c = d[b];
            memset(&c, 0, sizeof(c));
            c.A = A[b];
            c.X = wsp<double>(P, h.o_b);
            c.lda = h.lda;
            c.ldx = h.C;
            c.m = (int)h.m;
            c.n = (int)h.n;
            c.a_elem = es;
            c.transpose = (h.m > h.n) ? 1 : 0;
            cnt[b] = (int)(((h.m + 63) / 64) * ((h.n + 63) / 64));
        }
        P.copy = add_idx(B, d, cnt);
    }
    // Jacobi
    {
        std::vector<EyeDesc> de(np);
        std::vector<int> ce(np);
        std::vector<JacDesc> dj(np);
        std::vector<int> cj(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            EyeDesc& e = de[b];
            memset(&e, 0, sizeof(e));
            e.P = wsp<double>(P, h.o_p);
            e.ldp = h.R;
            e.R = h.R;
            ce[b] = (int)(((int64_t)h.R * h.R + 255) / 256);
            JacDesc& j = dj[b];
            memset(&j, 0, sizeof(j));
            j.X = wsp<double>(P, h.o_b);
            j.P = wsp<double>(P, h.o_p);
            j.rot = wsp<int>(P, h.o_rot);
            j.stats = wsp<int>(P, h.o_stats);
            j.ldx = h.C;
            j.ldp = h.R;
            j.R = h.R;
            j.C = h.C;
            j.nb = h.nb;
            // odd block count (last block all padding) with at least 3 real blocks
            j.skip0 = (h.nb >= 4 && (h.nb - 1) * JAC_B >= h.R) ? 1 : 0;
            j.cross_rounds = h.nb >= JAC_CROSS_MIN_NB ? 1 : 0;
            // the threshold of the row length of B (n for the RSVD, whether the
            // rows are those of B or of its triangular factor)
            j.tol = (double)(h.mode == 0 ? h.n : h.C) * std::ldexp(1.0, -53);
            cj[b] = h.nb / 2 - j.skip0;
        }
        P.eye = add_idx(B, de, ce);
        P.jac = add_idx(B, dj, cj);
        int mx = 0, mp = 0;
        for (int b = 0; b < np; ++b) {
            mx = std::max(mx, (P.probs[b].C + JAC_CHUNK - 1) / JAC_CHUNK);
            mp = std::max(mp, (P.probs[b].R + JAC_CHUNK - 1) / JAC_CHUNK);
        }
        P.jac_variant = jacobi_resident_variant(mx, mp);
        const int64_t ntasks = (int64_t)P.max_sweeps * (P.max_nb - 1) * P.jac.total;
        P.jac_persistent = !(P.flags & RSVD_PLAN_ROUND_LAUNCHES) && P.jac.total <= JAC_PERSISTENT_MAX_PAIRS &&
                           ntasks <= JAC_PERSISTENT_MAX_TASKS;
        if (P.jac_persistent) {
            const int64_t res = (int64_t)persistent_blocks_per_cu(P.jac_variant) * compute_units();
            P.jac_grid = (int)std::max<int64_t>(1, std::min(ntasks, res));
        }
    }
    // single-view plans: 2 sigma_i u_i^T A v_i for every Jacobi row i, from
    // F = A X^T (X the rotated rows, FP64 from the stored A), H^T = F^T Q and
    // u_i = Q P(i, :)^T: 2 sum_j P(i, j) H^T(i, j)
    if (P.single_view) {
        std::vector<GemmDesc> df(np), dh(np);
        std::vector<RowDotDesc> dr(np);
        std::vector<int> rows4(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            const int R = h.R;
            double* F = wsp<double>(P, h.o_f);
            double* Ht = wsp<double>(P, h.o_ht);
            df[b] = gd(A[b], h.lda, 0, wsp<double>(P, h.o_b), h.C, 1, F, R, (int)h.m, R, (int)h.n);
            dh[b] = gd(F, R, 1, final_q(P, h), R, 0, Ht, R, R, R, (int)h.m);
            RowDotDesc& r = dr[b];
            memset(&r, 0, sizeof(r));
            r.X = wsp<double>(P, h.o_p);
            r.Y = Ht;
            r.out = wsp<double>(P, h.o_cross);
            r.ldx = R;
            r.ldy = R;
            r.rows = R;
            r.cols = R;
            r.alpha = 2.0;
            rows4[b] = (R + 3) / 4;
        }
        P.g_sv_f = add_gemm(B, GK_F64, es, E_F64, E_F64, df);
        P.g_sv_ht = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, dh);
        P.sv_cross = add_idx(B, dr, rows4);
    }
    // finish + sign fix
    {
        std::vector<FinDesc> d(np);
        std::vector<int> ones(np, 1), cols(np), rows4(np), vt4(np), utiles(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            FinDesc& f = d[b];
            memset(&f, 0, sizeof(f));
            f.X = wsp<double>(P, h.o_b);
            f.P = wsp<double>(P, h.o_p);
            f.sig = wsp<double>(P, h.o_sig);
            f.perm = wsp<int>(P, h.o_perm);
            f.normA2 = wsp<double>(P, h.o_norm);
            f.rot = wsp<int>(P, h.o_rot);
            f.U = U[b];
            f.S = S[b];
            f.VT = VT[b];
            f.sgn = wsp<double>(P, h.o_sgn);
            f.w_out = w + b;
            f.kkept_out = kk + b;
            f.info_out = info ? info + b : wsp<int>(P, h.o_info_local);
            f.ldx = h.C;
            f.ldp = h.R;
            f.ldu = h.ldu;
            f.ldvt = h.ldvt;
            f.R = h.R;
            f.C = h.C;
            f.m = (int)h.m;
            f.n = (int)h.n;
            f.k = (int)h.k;
            f.mode = h.mode;
            f.max_sweeps = P.max_sweeps;
            f.delta = h.delta;
            f.jac_err = P.jac_persistent ? wsp<int>(P, P.off_sched) + 1 : nullptr;
            f.cross = P.single_view ? wsp<double>(P, h.o_cross) : nullptr;
            f.sv_flag = P.single_view ? wsp<int>(P, h.o_flags) + 2 * P.max_q + 1 : nullptr;
            rows4[b] = (h.R + 3) / 4;
            vt4[b] = (int)((h.k + 3) / 4);
            utiles[b] = h.mode == 0 ? 0 : (int)(((h.k + 63) / 64) * ((h.m + 63) / 64));
            cols[b] = (int)((h.k + 63) / 64);
        }
        // lq problems: the finishing step gathers W (rows of V^T in the basis
        // Q_B, k x l) into the Gram buffer; V^T = W Q_B^T follows as a GEMM
        std::vector<FinDesc> dfin = d;
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            if (!h.lq) continue;
            dfin[b].VT = wsp<double>(P, h.o_g);
            dfin[b].ldvt = h.R;
            dfin[b].n = h.R;
        }
        P.finish = add_idx(B, dfin, ones);
        P.fin_norm = add_idx(B, dfin, rows4);
        P.fin_vt = add_idx(B, dfin, vt4);
        P.fin_u = add_idx(B, dfin, utiles);
        P.signfix = add_idx(B, d, cols);
    }
    if (!P.fullsvd) {
        // U = Q Utilde[:, perm[:k]],  Utilde = P^T  ->  U(:, j) = Q P(perm[j], :)^T
        std::vector<GemmDesc> d(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            d[b] = gd(final_q(P, h), h.R, 0, wsp<double>(P, h.o_p), h.R, 1, U[b], h.ldu, (int)h.m, (int)h.k, h.R,
                      nullptr, wsp<int>(P, h.o_perm));
        }
        P.g_u = add_gemm(B, GK_F64, E_F64, E_F64, P.dt == RSVD_F64 ? E_F64 : E_F32, d);
        if (P.any_lq) {
            const GemmDesc none = gd(nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 0, 0, wsp<int>(P, P.off_one));
            std::vector<GemmDesc> dv(np, none);
            for (int b = 0; b < np; ++b) {
                const ProbHost& h = P.probs[b];
                if (h.lq)
                    dv[b] = gd(wsp<double>(P, h.o_g), h.R, 0, wsp<double>(P, h.o_qb), h.R, 1, VT[b], h.ldvt, (int)h.k,
                               (int)h.n, h.R);
            }
            // W holds the finishing step's output type (it is written like V^T)
            const Elem eo = P.dt == RSVD_F64 ? E_F64 : E_F32;
            P.g_lqvt = tgemm(GK_F64, eo, E_F64, eo, dv);
        }
    }
    P.hb = std::move(B);
}

#define LCHK(x)                                                                                   \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return fail(RSVD_ERR_HIP, std::string("launch: ") + hipGetErrorString(e_)); \
    } while (0)

// A launch of phase cat (RSVD_PHASE_*), timed when the plan is being profiled.
#define PLAUNCH(cat, flops, x)                                                                   \
    do {                                                                                          \
        if (P.prof) LCHK(P.prof->begin((cat), (flops)));                                          \
        LCHK(x);                                                                                  \
        if (P.prof) LCHK(P.prof->end());                                                          \
    } while (0)

template <typename T> const T* dp(const rsvd_plan& P, size_t off) { return (const T*)(P.dblob + off); }

// ---------------------------------------------------------------- tile autotuner
// Process-wide table: launch signature -> the fastest tile measured for it.
// With RSVD_TUNE_CACHE naming a file, the table is read from it once and
// written back (a flat JSON object, signature -> "BMxBN") after every new entry.
std::mutex g_tune_mu;
std::map<uint64_t, int> g_tune;
bool g_tune_loaded = false;

const char* tile_name(int t)
{
    switch (t) {
    case GT_64x64: return "64x64";
    case GT_128x64: return "128x64";
    case GT_64x128: return "64x128";
    case GT_128x128: return "128x128";
    }
    return "?";
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("RSVD_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    // pairs of quoted strings: "<16 hex digits>": "<tile>"
    std::vector<std::string> q;
    for (size_t i = 0; i < text.size(); ++i) {
        if (text[i] != '"') continue;
        const size_t j = text.find('"', i + 1);
        if (j == std::string::npos) break;
        q.push_back(text.substr(i + 1, j - i - 1));
        i = j;
    }
    for (size_t i = 0; i + 1 < q.size(); i += 2) {
        char* end = nullptr;
        const uint64_t key = strtoull(q[i].c_str(), &end, 16);
        if (!end || *end != 0 || q[i].empty()) continue;
        for (int t = GT_64x64; t <= GT_128x128; ++t)
            if (q[i + 1] == tile_name(t)) g_tune[key] = t;
    }
}

void tune_save_locked()
{
    const char* path = getenv("RSVD_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : g_tune)
        fprintf(f, "  \"%016llx\": \"%s\"%s\n", (unsigned long long)kv.first, tile_name(kv.second),
                ++i < g_tune.size() ? "," : "");
    fprintf(f, "}\n");
    if (fclose(f) == 0) (void)rename(tmp.c_str(), path);
}

// One tunable launch of the tuning execute: unless the table knows its
// signature, time every tile (one warm-up, then the mean of three launches,
// HIP events on the plan's stream) and keep the fastest.  Every tile computes
// each output element with the same K order, so the products are identical
// and repeating a launch (none of these accumulates) leaves the same result.
int tune_gemm(rsvd_plan& P, const GemmLaunch& g, hipStream_t s)
{
    const int np = P.nprob;
    std::vector<GemmDesc> d0(np);
    memcpy(d0.data(), P.hb.bytes.data() + g.off_desc, sizeof(GemmDesc) * np);
    int best = g.tile;
    bool known;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(g.sig);
        known = it != g_tune.end();
        if (known) best = it->second;
    }
    auto install = [&](int tile, int* total) -> int {
        std::vector<GemmDesc> d = d0;
        std::vector<int> map = item_map(finalize_descs(d, (GemmTile)tile, total));
        if (map.size() > 2 * (size_t)std::max(g.cap, 1)) return fail(RSVD_ERR_HIP, "tuner: item map exceeds its reservation");
        map.resize(2 * (size_t)std::max(g.cap, 1), 0);
        HIPCHK(hipStreamSynchronize(s));  // earlier copies out of the pinned blob are done
        memcpy(P.hblob_pinned + g.off_desc, d.data(), sizeof(GemmDesc) * np);
        memcpy(P.hblob_pinned + g.off_begin, map.data(), sizeof(int) * map.size());
        HIPCHK(hipMemcpyAsync(P.dblob + g.off_desc, P.hblob_pinned + g.off_desc, sizeof(GemmDesc) * np,
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(P.dblob + g.off_begin, P.hblob_pinned + g.off_begin, sizeof(int) * map.size(),
                              hipMemcpyHostToDevice, s));
        return RSVD_OK;
    };
    auto run = [&](int tile, int total) -> int {
        if (total <= 0) return RSVD_OK;
        hipError_t e = launch_gemm(g.kind, g.ea, g.ex, g.ec, (GemmTile)tile, false, dp<GemmDesc>(P, g.off_desc),
                                   dp<int>(P, g.off_begin), np, total, s);
        return e == hipSuccess ? RSVD_OK : fail(RSVD_ERR_HIP, std::string("tuner launch: ") + hipGetErrorString(e));
    };
    int rc, total = 0;
    if (!known) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(hipEventCreate(&e0));
        hipError_t he = hipEventCreate(&e1);
        if (he != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(RSVD_ERR_HIP, std::string("tuner event: ") + hipGetErrorString(he));
        }
        float best_ms = 0.f;
        rc = RSVD_OK;
        for (int t = GT_64x64; t <= GT_128x128 && rc == RSVD_OK; ++t) {
            if ((rc = install(t, &total)) != RSVD_OK) break;
            if ((rc = run(t, total)) != RSVD_OK) break;
            if ((he = hipEventRecord(e0, s)) != hipSuccess) break;
            for (int r = 0; r < 3 && rc == RSVD_OK; ++r) rc = run(t, total);
            if (rc != RSVD_OK) break;
            if ((he = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.f;
            if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (t == GT_64x64 || ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != RSVD_OK) return rc;
        if (he != hipSuccess) return fail(RSVD_ERR_HIP, std::string("tuner timing: ") + hipGetErrorString(he));
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[g.sig] = best;
        tune_save_locked();
    }
    if ((rc = install(best, &total)) != RSVD_OK) return rc;
    if ((rc = run(best, total)) != RSVD_OK) return rc;
    if ((int)P.tile_ovr.size() <= g.slot) P.tile_ovr.resize(g.slot + 1, -1);
    P.tile_ovr[g.slot] = best;
    return RSVD_OK;
}

int gemm(rsvd_plan& P, const GemmLaunch& g, hipStream_t s, int cat)
{
    if (g.total <= 0) return RSVD_OK;
    if (P.tuner && g.slot >= 0) return tune_gemm(P, g, s);
    PLAUNCH(cat, g.flops,
            launch_gemm(g.kind, g.ea, g.ex, g.ec, g.tile, g.gather, dp<GemmDesc>(P, g.off_desc), dp<int>(P, g.off_begin), P.nprob,
                        g.total, s));
    return RSVD_OK;
}

// Householder fallback of one orthonormalisation site, blocked or not.
hipError_t householder(const rsvd_plan& P, const QrDesc* d, hipStream_t s)
{
    if (P.hh_blocked) return launch_householder_blocked(d, P.nprob, P.max_l, P.hh_rows, s);
    return launch_householder(d, P.nprob, s);
}

// The full launch sequence of one execute (captured into a graph when asked).
int enqueue(rsvd_plan& P, hipStream_t s)
{
    const int np = P.nprob;
    const int out_f64 = P.dt == RSVD_F64;
    int rc;
    PLAUNCH(RSVD_PHASE_OTHER, 0.0, launch_fill_i32(wsp<int>(P, P.off_one), 1, 1, s));
    PLAUNCH(RSVD_PHASE_OTHER, 0.0, launch_fill_i32(wsp<int>(P, P.off_flags_base), 0, P.total_flags, s));
    PLAUNCH(RSVD_PHASE_STAGE, 0.0,
            launch_stage(dp<StageDesc>(P, P.stage.off_desc), dp<int>(P, P.stage.off_begin), np, P.stage.total, s));
    PLAUNCH(RSVD_PHASE_STAGE, 0.0, launch_stage_final(dp<StageDesc>(P, P.stage.off_desc), np, s));
    if (!P.fullsvd) {
        PLAUNCH(RSVD_PHASE_OMEGA, 0.0,
                launch_omega(dp<OmegaDesc>(P, P.omega.off_desc), dp<int>(P, P.omega.off_begin), np, P.omega.total, s));
        if (P.single_view)
            PLAUNCH(RSVD_PHASE_OMEGA, 0.0,
                    launch_omega(dp<OmegaDesc>(P, P.omega_psi.off_desc), dp<int>(P, P.omega_psi.off_begin), np,
                                 P.omega_psi.total, s));
        const int nst = 2 * P.max_q + 1;
        for (int st = 0; st < nst; ++st) {
            if ((rc = gemm(P, P.g_sketch[st], s, RSVD_PHASE_SKETCH)) != RSVD_OK) return rc;
            const IdxLaunch& q1 = P.qr[2 * st];
            const IdxLaunch& q2 = P.qr[2 * st + 1];
            const IdxLaunch& t1 = P.trsm[2 * st];
            const IdxLaunch& t2 = P.trsm[2 * st + 1];
            // Cholesky QR pass 1
            if ((rc = gemm(P, P.g_gram1[st], s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
            PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, q1.off_desc), np, P.max_l, s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, t1.off_desc), dp<int>(P, t1.off_begin), np, t1.total, 1, stage_y(P, st),
                                P.max_l, s));
            // pass 2 for the problems whose final basis this is
            if (t2.total > 0) {
                if ((rc = gemm(P, P.g_gram2[st], s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
                PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, q2.off_desc), np, P.max_l, s));
                PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                        launch_trsm(dp<QrDesc>(P, t2.off_desc), dp<int>(P, t2.off_begin), np, t2.total, 0, E_F64, P.max_l, s));
            }
            // Householder for the problems whose Cholesky QR broke down
            PLAUNCH(RSVD_PHASE_HOUSEHOLDER, 0.0, householder(P, dp<QrDesc>(P, q1.off_desc), s));
            if (P.krylov && P.kcopy[st].total > 0)
                PLAUNCH(RSVD_PHASE_OTHER, 0.0,
                        launch_copy_f64(dp<CopyDesc>(P, P.kcopy[st].off_desc), dp<int>(P, P.kcopy[st].off_begin), np,
                                        P.kcopy[st].total, s));
        }
        if (P.single_view) {
            // the co-range sketch and the Jacobi input X = (Psi Q)^+ W
            if ((rc = gemm(P, P.g_sv_w, s, RSVD_PHASE_SKETCH)) != RSVD_OK) return rc;
            if ((rc = gemm(P, P.g_sv_z, s, RSVD_PHASE_PROJECT)) != RSVD_OK) return rc;
            if ((rc = gemm(P, P.g_sv_gram, s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
            PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, P.sv_qr.off_desc), np, P.max_l, s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, P.sv_trsm_z.off_desc), dp<int>(P, P.sv_trsm_z.off_begin), np,
                                P.sv_trsm_z.total, 0, E_F64, P.max_l, s));
            PLAUNCH(RSVD_PHASE_OTHER, 0.0,
                    launch_eye(dp<EyeDesc>(P, P.sv_eye.off_desc), dp<int>(P, P.sv_eye.off_begin), np, P.sv_eye.total,
                               s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, P.sv_trsm_i.off_desc), dp<int>(P, P.sv_trsm_i.off_begin), np,
                                P.sv_trsm_i.total, 0, E_F64, P.max_l, s));
            if ((rc = gemm(P, P.g_sv_m, s, RSVD_PHASE_PROJECT)) != RSVD_OK) return rc;
            if ((rc = gemm(P, P.g_sv_x, s, RSVD_PHASE_PROJECT)) != RSVD_OK) return rc;
        }
        if (P.krylov) {
            if ((rc = gemm(P, P.g_kgram1, s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
            PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, P.k_qr[0].off_desc), np, P.max_l, s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, P.k_trsm[0].off_desc), dp<int>(P, P.k_trsm[0].off_begin), np,
                                P.k_trsm[0].total, 1, E_F64, P.max_l, s));
            if ((rc = gemm(P, P.g_kgram2, s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
            PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, P.k_qr[1].off_desc), np, P.max_l, s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, P.k_trsm[1].off_desc), dp<int>(P, P.k_trsm[1].off_begin), np,
                                P.k_trsm[1].total, 0, E_F64, P.max_l, s));
            PLAUNCH(RSVD_PHASE_HOUSEHOLDER, 0.0, householder(P, dp<QrDesc>(P, P.k_qr[0].off_desc), s));
        }
        if (P.any_lq) {
            if ((rc = gemm(P, P.g_lqbt, s, RSVD_PHASE_PROJECT)) != RSVD_OK) return rc;
            if ((rc = gemm(P, P.g_lqgram1, s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
            PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, P.lq_qr[0].off_desc), np, P.max_l, s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, P.lq_trsm[0].off_desc), dp<int>(P, P.lq_trsm[0].off_begin), np,
                                P.lq_trsm[0].total, 1, E_F64, P.max_l, s));
            if ((rc = gemm(P, P.g_lqgram2, s, RSVD_PHASE_GRAM)) != RSVD_OK) return rc;
            PLAUNCH(RSVD_PHASE_CHOL, 0.0, launch_chol(dp<QrDesc>(P, P.lq_qr[1].off_desc), np, P.max_l, s));
            PLAUNCH(RSVD_PHASE_TRSM, 0.0,
                    launch_trsm(dp<QrDesc>(P, P.lq_trsm[1].off_desc), dp<int>(P, P.lq_trsm[1].off_begin), np,
                                P.lq_trsm[1].total, 0, E_F64, P.max_l, s));
            PLAUNCH(RSVD_PHASE_HOUSEHOLDER, 0.0, householder(P, dp<QrDesc>(P, P.lq_qr[0].off_desc), s));
            if ((rc = gemm(P, P.g_lqx, s, RSVD_PHASE_PROJECT)) != RSVD_OK) return rc;
        }
        if (!P.single_view && (rc = gemm(P, P.g_b, s, RSVD_PHASE_PROJECT)) != RSVD_OK) return rc;
    } else {
        PLAUNCH(RSVD_PHASE_OTHER, 0.0,
                launch_copy_f64(dp<CopyDesc>(P, P.copy.off_desc), dp<int>(P, P.copy.off_begin), np, P.copy.total, s));
    }
    PLAUNCH(RSVD_PHASE_OTHER, 0.0,
            launch_eye(dp<EyeDesc>(P, P.eye.off_desc), dp<int>(P, P.eye.off_begin), np, P.eye.total, s));
    if (P.jac_persistent) {
        PLAUNCH(RSVD_PHASE_JACOBI, 0.0,
                launch_jacobi_persistent(dp<JacDesc>(P, P.jac.off_desc), dp<int>(P, P.jac.off_begin), P.jac.total,
                                         P.max_nb - 1, P.max_sweeps, wsp<int>(P, P.off_sched), P.jac_grid,
                                         P.jac_variant, s));
    } else {
        for (int sw = 0; sw < P.max_sweeps; ++sw)
            for (int r = 0; r < P.max_nb - 1; ++r)
                PLAUNCH(RSVD_PHASE_JACOBI, 0.0,
                        launch_jacobi_round(dp<JacDesc>(P, P.jac.off_desc), dp<int>(P, P.jac.off_begin), np,
                                            P.jac.total, sw, r, P.jac_variant, s));
    }
    if (P.single_view) {
        // the true error of each triplet needs u_i^T A v_i: one more product with A
        if ((rc = gemm(P, P.g_sv_f, s, RSVD_PHASE_FINISH)) != RSVD_OK) return rc;
        if ((rc = gemm(P, P.g_sv_ht, s, RSVD_PHASE_FINISH)) != RSVD_OK) return rc;
        PLAUNCH(RSVD_PHASE_FINISH, 0.0,
                launch_rowdot(dp<RowDotDesc>(P, P.sv_cross.off_desc), dp<int>(P, P.sv_cross.off_begin), np,
                              P.sv_cross.total, s));
    }
    PLAUNCH(RSVD_PHASE_FINISH, 0.0,
            launch_finish(dp<FinDesc>(P, P.finish.off_desc), np, dp<int>(P, P.fin_norm.off_begin), P.fin_norm.total,
                          dp<int>(P, P.fin_vt.off_begin), P.fin_vt.total, dp<int>(P, P.fin_u.off_begin), P.fin_u.total,
                          out_f64, s));
    if (!P.fullsvd) {
        if ((rc = gemm(P, P.g_u, s, RSVD_PHASE_BACKPROJ)) != RSVD_OK) return rc;
        if (P.any_lq && (rc = gemm(P, P.g_lqvt, s, RSVD_PHASE_BACKPROJ)) != RSVD_OK) return rc;
    }
    PLAUNCH(RSVD_PHASE_SIGNFIX, 0.0,
            launch_signfix(dp<FinDesc>(P, P.signfix.off_desc), dp<int>(P, P.signfix.off_begin), np,
                           P.signfix.total, out_f64, s));
    return RSVD_OK;
}

// ---------------------------------------------------------------- reverse pass
// Descriptor tables of rsvd_plan_backward.  Per problem (l, m, n, final stage
// f = 2q): the head stages the cotangents and forms Bbar, the cotangent of
// B = Q_f^T A, by the SVD adjoint; then Qbar (cotangent of the current basis)
// walks the stages backwards through the thin-QR adjoint and the products of
// the power iteration, and every product that involves A adds its share of
// dA.  The two (max(m, n) x l) work buffers alternate between Qbar and the
// next stage's Qbar; the triangular solve works in place.
// Copy of the rows x cols matrix A (element elem, leading dimension lda) into
// X (leading dimension ldx), transposed when asked; *count receives its
// 64 x 64 tiles.
CopyDesc copy_desc(const void* A, Elem elem, int rows, int cols, int64_t lda, double* X, int64_t ldx, bool transpose,
                   int* count)
{
    CopyDesc c;
    memset(&c, 0, sizeof(c));
    c.A = A;
    c.X = X;
    c.lda = lda;
    c.ldx = ldx;
    c.m = rows;
    c.n = cols;
    c.a_elem = elem;
    c.transpose = transpose ? 1 : 0;
    *count = ((rows + 63) / 64) * ((cols + 63) / 64);
    return c;
}

void build_bw_blob(rsvd_plan& P, const void* const* dU, const void* const* dS, const void* const* dVT,
                   void* const* dA, double broad)
{
    Blob B;
    auto& W = P.bw;
    const int np = P.nprob;
    const int* one = wsp<int>(P, P.off_one);
    const Elem es = P.e_store;
    const GemmDesc none = gd(nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0, 0, 0, one);
    std::vector<BwDesc> bd(np);
    std::vector<int> cprep(np), ccore(np);
    auto blocks = [](int64_t e) { return (int)((e + BW_ELEMS_PER_BLOCK - 1) / BW_ELEMS_PER_BLOCK); };
    for (int b = 0; b < np; ++b) {
        const ProbHost& h = P.probs[b];
        BwDesc& d = bd[b];
        memset(&d, 0, sizeof(d));
        d.dU = dU[b];
        d.dS = dS[b];
        d.dVT = dVT[b];
        d.X = wsp<double>(P, h.o_b);
        d.P = wsp<double>(P, h.o_p);
        d.sig = wsp<double>(P, h.o_sig);
        d.perm = wsp<int>(P, h.o_perm);
        d.sgn = wsp<double>(P, h.o_sgn);
        d.Ub = wsp<double>(P, h.o_bw_w[1]);
        d.Vbt = wsp<double>(P, h.o_bw_vbt);
        d.Vts = wsp<double>(P, h.o_bw_vts);
        d.Ut = wsp<double>(P, h.o_bw_ut);
        d.sb = wsp<double>(P, h.o_bw_sb);
        d.EU = wsp<double>(P, h.o_bw_eu);
        d.EV = wsp<double>(P, h.o_bw_ev);
        d.Kp = wsp<double>(P, h.o_bw_kp);
        d.C = wsp<double>(P, h.o_bw_eu);
        d.S = wsp<double>(P, h.o_bw_ev);
        d.ldu = h.ldu;
        d.ldvt = h.ldvt;
        d.m = (int)h.m;
        d.n = (int)h.n;
        d.l = h.l;
        d.k = (int)h.k;
        d.elem = es;
        d.broad = broad;
        cprep[b] = blocks(bw_prep_elems(d.m, d.n, d.l));
        ccore[b] = blocks(bw_core_elems(d.n, d.l));
    }
    W.prep = add_idx(B, bd, cprep);
    W.core = add_idx(B, bd, ccore);
    {
        std::vector<GemmDesc> utb(np), qb0(np), eu(np), ev(np), nn(np), bb(np), qba(np), dac(np);
        std::vector<CopyDesc> cl0(np), cr0(np);
        std::vector<int> ccl0(np), ccr0(np);
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            const int l = h.l, m = (int)h.m, n = (int)h.n;
            const double* Qf = wsp<double>(P, h.o_qstage[2 * h.q]);
            double* W0 = wsp<double>(P, h.o_bw_w[0]);
            double* Ub = wsp<double>(P, h.o_bw_w[1]);
            double* Ut = wsp<double>(P, h.o_bw_ut);
            double* Utb = wsp<double>(P, h.o_bw_utb);
            double* Vbt = wsp<double>(P, h.o_bw_vbt);
            double* Vts = wsp<double>(P, h.o_bw_vts);
            double* Bb = wsp<double>(P, h.o_bw_bb);
            // U = Q Utilde:  Utilde_bar = Q^T Ubar,  Qbar = Ubar Utilde^T
            utb[b] = gd(Qf, l, 1, Ub, l, 0, Utb, l, l, l, m);
            qb0[b] = gd(Ub, l, 0, Ut, l, 1, W0, l, m, l, l);
            // SVD of B:  EU = Utilde^T Utilde_bar,  EV = Vtilde^T Vbar
            eu[b] = gd(Ut, l, 1, Utb, l, 0, wsp<double>(P, h.o_bw_eu), l, l, l, l);
            ev[b] = gd(Vts, n, 0, Vbt, n, 1, wsp<double>(P, h.o_bw_ev), l, l, l, n);
            // N = Kp Vtilde^T + Sigma^-1 Vbar^T (the second term staged by the core kernel), Bbar = Utilde N
            nn[b] = gd(wsp<double>(P, h.o_bw_kp), l, 0, Vts, n, 0, Vbt, n, l, n, l);
            nn[b].accumulate = 1;
            bb[b] = gd(Ut, l, 0, Vbt, n, 0, Bb, n, l, n, l);
            // B = Q^T A:  Qbar += A Bbar^T;  dA's term Q Bbar goes into slice 0 (L = Q, R = Bbar^T)
            qba[b] = gd(P.lastA[b], h.lda, 0, Bb, n, 1, W0, l, m, l, n);
            qba[b].accumulate = 1;
            const int64_t tl = (2 * h.q + 2) * l;
            double* Lc = wsp<double>(P, h.o_bw_lcat);
            double* Rc = wsp<double>(P, h.o_bw_rcat);
            cl0[b] = copy_desc(Qf, E_F64, m, l, l, Lc, tl, false, &ccl0[b]);
            cr0[b] = copy_desc(Bb, E_F64, l, n, n, Rc, tl, true, &ccr0[b]);  // Bbar (l x n) transposed
            dac[b] = gd(Lc, tl, 0, Rc, tl, 1, dA[b], h.lda, m, n, (int)tl);
        }
        W.utb = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, utb);
        W.qb0 = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, qb0);
        W.eu = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, eu);
        W.ev = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, ev);
        W.nn = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, nn);
        W.bb = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, bb);
        W.qba = add_gemm(B, GK_F64, es, E_F64, E_F64, qba);
        W.cat_l0 = add_idx(B, cl0, ccl0);
        W.cat_r0 = add_idx(B, cr0, ccr0);
        W.da = add_gemm(B, GK_F64, E_F64, E_F64, es, dac);
    }
    const int nst = 2 * P.max_q + 1;
    W.st.assign(nst, rsvd_plan::BwStage());
    for (int s = nst - 1; s >= 0; --s) {
        std::vector<GemmDesc> c(np, none), qs(np, none), r(np, none), qprev(np, none);
        std::vector<BwDesc> sym(bd);
        std::vector<QrDesc> tri(np);
        std::vector<int> csym(np, 0), ctri(np, 1), ctrsm(np, 0), ccl(np, 0), ccr(np, 0);
        std::vector<CopyDesc> cl(np), cr(np);
        for (int b = 0; b < np; ++b) {
            memset(&cl[b], 0, sizeof(CopyDesc));
            memset(&cr[b], 0, sizeof(CopyDesc));
        }
        for (int b = 0; b < np; ++b) {
            const ProbHost& h = P.probs[b];
            memset(&tri[b], 0, sizeof(QrDesc));
            tri[b].flag = const_cast<int*>(one);
            tri[b].l = h.l;
            if (s > 2 * h.q) continue;
            const int l = h.l, m = (int)h.m, n = (int)h.n;
            const int rows = (s % 2 == 0) ? m : n;
            const int cur = (int)((2 * h.q - s) % 2);
            double* Qb = wsp<double>(P, h.o_bw_w[cur]);
            double* Qn = wsp<double>(P, h.o_bw_w[1 - cur]);
            const double* Qs = wsp<double>(P, h.o_qstage[s]);
            const void* Ms = wsp<char>(P, h.o_mstage[s]);
            double* Cm = wsp<double>(P, h.o_bw_eu);
            double* Sm = wsp<double>(P, h.o_bw_ev);
            double* R = wsp<double>(P, h.o_lwork);
            // thin QR M_s = Q_s R_s:  Mbar = (Qbar + Q_s copyltu(-Qbar^T Q_s)) R_s^-T
            c[b] = gd(Qb, l, 1, Qs, l, 0, Cm, l, l, l, rows);
            csym[b] = blocks(bw_sym_elems(l));
            qs[b] = gd(Qs, l, 0, Sm, l, 0, Qb, l, rows, l, l);
            qs[b].accumulate = 1;
            r[b] = gd(Qs, l, 1, Ms, l, 0, R, l, l, l, rows);
            tri[b].Qout = Qb;
            tri[b].L = R;
            tri[b].D = wsp<double>(P, h.o_dwork);
            tri[b].rows = rows;
            ctrsm[b] = (rows + 15) / 16;
            // the product that formed M_s; its dA term L R^T goes into slice 1 + 2q - s
            const int64_t tl = (2 * h.q + 2) * l, off = (int64_t)(1 + 2 * h.q - s) * l;
            double* Lc = wsp<double>(P, h.o_bw_lcat) + off;
            double* Rc = wsp<double>(P, h.o_bw_rcat) + off;
            if (s % 2 == 0) {
                // M_s = A X_s, X_s = Omega (s = 0) or the previous basis: dA += Mbar X_s^T, Qbar_prev = A^T Mbar
                const void* Xs = (s == 0) ? (const void*)wsp<char>(P, h.o_om) : wsp<double>(P, h.o_qstage[s - 1]);
                cl[b] = copy_desc(Qb, E_F64, m, l, l, Lc, tl, false, &ccl[b]);
                cr[b] = copy_desc(Xs, s == 0 ? P.e_sketch : E_F64, n, l, l, Rc, tl, false, &ccr[b]);
                if (s > 0) qprev[b] = gd(P.lastA[b], h.lda, 1, Qb, l, 0, Qn, l, n, l, m);
            } else {
                // M_s = A^T Q_{s-1}: dA += Q_{s-1} Mbar^T, Qbar_prev = A Mbar
                cl[b] = copy_desc(wsp<double>(P, h.o_qstage[s - 1]), E_F64, m, l, l, Lc, tl, false, &ccl[b]);
                cr[b] = copy_desc(Qb, E_F64, n, l, l, Rc, tl, false, &ccr[b]);
                qprev[b] = gd(P.lastA[b], h.lda, 0, Qb, l, 0, Qn, l, m, l, n);
            }
        }
        rsvd_plan::BwStage& st = W.st[s];
        st.c = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, c);
        st.sym = add_idx(B, sym, csym);
        st.qs = add_gemm(B, GK_F64, E_F64, E_F64, E_F64, qs);
        st.r = add_gemm(B, GK_F64, E_F64, P.e_y, E_F64, r);
        st.tri = add_idx(B, tri, ctri);
        st.trsm = add_idx(B, tri, ctrsm);
        st.cat_l = add_idx(B, cl, ccl);
        st.cat_r = add_idx(B, cr, ccr);
        st.qprev = add_gemm(B, GK_F64, es, E_F64, E_F64, qprev);
    }
    W.hb = std::move(B);
}

int enqueue_backward(rsvd_plan& P, hipStream_t s)
{
    const int np = P.nprob;
    auto& W = P.bw;
    const char* base = W.dblob;
    auto dd = [&](size_t off) { return (const void*)(base + off); };
    auto bgemm = [&](const GemmLaunch& g) -> int {
        if (g.total <= 0) return RSVD_OK;
        PLAUNCH(RSVD_PHASE_BW_GEMM, g.flops,
                launch_gemm(g.kind, g.ea, g.ex, g.ec, g.tile, g.gather, (const GemmDesc*)dd(g.off_desc), (const int*)dd(g.off_begin),
                            np, g.total, s));
        return RSVD_OK;
    };
    int rc;
    const int cot_f64 = P.dt == RSVD_F64;
    PLAUNCH(RSVD_PHASE_BW_SMALL, 0.0,
            launch_bw_prep((const BwDesc*)dd(W.prep.off_desc), (const int*)dd(W.prep.off_begin), np, W.prep.total,
                           cot_f64, s));
    for (const GemmLaunch* g : {&W.utb, &W.qb0, &W.eu, &W.ev})
        if ((rc = bgemm(*g)) != RSVD_OK) return rc;
    PLAUNCH(RSVD_PHASE_BW_SMALL, 0.0,
            launch_bw_core((const BwDesc*)dd(W.core.off_desc), (const int*)dd(W.core.off_begin), np, W.core.total, s));
    auto bcopy = [&](const IdxLaunch& c) -> int {
        if (c.total <= 0) return RSVD_OK;
        PLAUNCH(RSVD_PHASE_BW_SMALL, 0.0,
                launch_copy_f64((const CopyDesc*)dd(c.off_desc), (const int*)dd(c.off_begin), np, c.total, s));
        return RSVD_OK;
    };
    for (const GemmLaunch* g : {&W.nn, &W.bb, &W.qba})
        if ((rc = bgemm(*g)) != RSVD_OK) return rc;
    if ((rc = bcopy(W.cat_l0)) != RSVD_OK || (rc = bcopy(W.cat_r0)) != RSVD_OK) return rc;
    for (int st = (int)W.st.size() - 1; st >= 0; --st) {
        const rsvd_plan::BwStage& S = W.st[st];
        if ((rc = bgemm(S.c)) != RSVD_OK) return rc;
        PLAUNCH(RSVD_PHASE_BW_SMALL, 0.0,
                launch_bw_sym((const BwDesc*)dd(S.sym.off_desc), (const int*)dd(S.sym.off_begin), np, S.sym.total, s));
        if ((rc = bgemm(S.qs)) != RSVD_OK) return rc;
        if ((rc = bgemm(S.r)) != RSVD_OK) return rc;
        PLAUNCH(RSVD_PHASE_BW_SMALL, 0.0, launch_tri_prep((const QrDesc*)dd(S.tri.off_desc), np, P.max_l, s));
        PLAUNCH(RSVD_PHASE_BW_SMALL, 0.0,
                launch_trsm_upper((const QrDesc*)dd(S.trsm.off_desc), (const int*)dd(S.trsm.off_begin), np,
                                  S.trsm.total, P.max_l, s));
        if ((rc = bcopy(S.cat_l)) != RSVD_OK || (rc = bcopy(S.cat_r)) != RSVD_OK) return rc;
        if ((rc = bgemm(S.qprev)) != RSVD_OK) return rc;
    }
    // dA = sum of the 2q + 2 terms L_t R_t^T as one product with inner dimension (2q + 2) l
    return bgemm(W.da);
}

int plan_backward(rsvd_plan* P, const void* const* dU, const void* const* dS, const void* const* dVT,
                  void* const* dA, double broad, hipStream_t stream, bool eager)
{
    if (!P) return fail(RSVD_ERR_INVALID, "plan is null");
    if (P->fullsvd || !(P->flags & RSVD_PLAN_SAVE))
        return fail(RSVD_ERR_INVALID, "backward needs an RSVD plan created with RSVD_PLAN_SAVE");
    if (!P->fwd_saved) return fail(RSVD_ERR_INVALID, "backward needs a preceding rsvd_plan_execute");
    if (!(broad >= 0.0) || !(broad < INFINITY)) return fail(RSVD_ERR_INVALID, "broadening must be finite and >= 0");
    if (!dU || !dS || !dVT || !dA) return fail(RSVD_ERR_INVALID, "null cotangent or gradient array");
    for (int b = 0; b < P->nprob; ++b) {
        if (!dU[b] || !dS[b] || !dVT[b] || !dA[b]) return fail(RSVD_ERR_INVALID, "null matrix pointer in batch");
        if (dA[b] == P->lastA[b]) return fail(RSVD_ERR_INVALID, "dA must not overlap A");
    }
    auto& W = P->bw;
    bool same = W.valid && W.gen == P->fwd_gen && W.broad == broad;
    for (int b = 0; b < P->nprob && same; ++b)
        same = W.ldU[b] == dU[b] && W.ldS[b] == dS[b] && W.ldVT[b] == dVT[b] && W.ldA[b] == dA[b];
    if (!same) {
        if (W.upload_pending) HIPCHK(hipEventSynchronize(W.upload_done));
        build_bw_blob(*P, dU, dS, dVT, dA, broad);
        const size_t bytes = std::max<size_t>(W.hb.bytes.size(), 64);
        if (W.dblob && bytes != W.bytes) return fail(RSVD_ERR_HIP, "descriptor layout changed");
        if (!W.dblob) {
            hipError_t e = hipMalloc(&W.dblob, bytes);
            if (e == hipSuccess) e = hipHostMalloc(&W.hpinned, bytes, 0);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&W.upload_done, hipEventDisableTiming);
            if (e != hipSuccess) return fail(RSVD_ERR_ALLOC, std::string("backward allocation: ") + hipGetErrorString(e));
            W.bytes = bytes;
        }
        memcpy(W.hpinned, W.hb.bytes.data(), W.hb.bytes.size());
        HIPCHK(hipMemcpyAsync(W.dblob, W.hpinned, W.hb.bytes.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipEventRecord(W.upload_done, stream));
        W.upload_pending = true;
        W.ldU.assign(dU, dU + P->nprob);
        W.ldS.assign(dS, dS + P->nprob);
        W.ldVT.assign(dVT, dVT + P->nprob);
        W.ldA.assign(dA, dA + P->nprob);
        W.broad = broad;
        W.gen = P->fwd_gen;
        W.valid = true;
    }
    if ((P->flags & RSVD_PLAN_GRAPH) && !eager) {
        if (!W.gexec) {
            HIPCHK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_backward(*P, P->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
            if (rc != RSVD_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(RSVD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            W.graph = g;
            HIPCHK(hipGraphInstantiate(&W.gexec, W.graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(W.gexec, stream));
        return RSVD_OK;
    }
    return enqueue_backward(*P, stream);
}

void complex_free(ComplexExt* X);

void plan_free(rsvd_plan* P)
{
    if (!P) return;
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->upload_done) (void)hipEventDestroy(P->upload_done);
    if (P->ws) (void)hipFree(P->ws);
    if (P->dblob) (void)hipFree(P->dblob);
    if (P->hblob_pinned) (void)hipHostFree(P->hblob_pinned);
    if (P->bw.gexec) (void)hipGraphExecDestroy(P->bw.gexec);
    if (P->bw.graph) (void)hipGraphDestroy(P->bw.graph);
    if (P->bw.upload_done) (void)hipEventDestroy(P->bw.upload_done);
    if (P->bw.dblob) (void)hipFree(P->bw.dblob);
    if (P->bw.hpinned) (void)hipHostFree(P->bw.hpinned);
    complex_free(P->cx);
    delete P;
}

// Kernel attributes set once per process (dynamic LDS limits).
int kernels_ready()
{
    static std::once_flag once;
    static hipError_t init_err = hipSuccess;
    std::call_once(once, [] {
        init_err = init_qr_kernels();
        if (init_err == hipSuccess) init_err = init_select_kernels();
    });
    if (init_err != hipSuccess) return fail(RSVD_ERR_HIP, std::string("kernel attributes: ") + hipGetErrorString(init_err));
    return RSVD_OK;
}

// Validates the problems and fills the host side of a plan: per-problem
// sizes, Jacobi blocking and the workspace layout (P.ws_bytes).  No device
// memory is touched.
int plan_setup(rsvd_plan* P, const rsvd_problem_t* probs, int64_t batch, rsvd_dtype_t dt, rsvd_prec_t prec,
               unsigned flags)
{
    if (!probs || batch < 1 || batch > (1 << 20)) return fail(RSVD_ERR_INVALID, "batch must be in [1, 2^20]");
    if (dt != RSVD_F64 && dt != RSVD_F32) return fail(RSVD_ERR_INVALID, "unknown dtype");
    if (prec != RSVD_PREC_F64 && prec != RSVD_PREC_F32 && prec != RSVD_PREC_BF16)
        return fail(RSVD_ERR_INVALID, "unknown precision");
    const bool fullsvd = (flags & RSVD_PLAN_FULLSVD) != 0;
    const bool krylov = (flags & RSVD_PLAN_BLOCK_KRYLOV) != 0;
    if (krylov && (fullsvd || (flags & RSVD_PLAN_SAVE)))
        return fail(RSVD_ERR_INVALID, "block-Krylov plans are RSVD plans without a saved forward");
    const bool single_view = (flags & RSVD_PLAN_SINGLE_VIEW) != 0;
    const bool fp64_final = (flags & RSVD_PLAN_FP64_FINAL) != 0 && prec != RSVD_PREC_F64 && !fullsvd;
    if (fp64_final) {
        if (krylov || single_view || (flags & RSVD_PLAN_SAVE))
            return fail(RSVD_ERR_INVALID,
                        "the FP64 final power step is not available with block-Krylov, single-view or saving plans");
        for (int64_t b = 0; b < batch; ++b)
            if (probs[b].q < 1 || probs[b].q != probs[0].q)
                return fail(RSVD_ERR_INVALID, "the FP64 final power step needs the same q >= 1 for every problem");
    }
    if (single_view && (fullsvd || krylov || (flags & RSVD_PLAN_SAVE)))
        return fail(RSVD_ERR_INVALID,
                    "single-view plans are RSVD plans without a saved forward and without block-Krylov");
    for (int64_t b = 0; b < batch; ++b) {
        int rc = validate_problem(probs[b], fullsvd);
        if (rc != RSVD_OK) return fail(rc, "problem " + std::to_string(b) + ": " + g_err);
        if (krylov) {
            const int64_t mn = std::min(probs[b].m, probs[b].n);
            const int64_t l = std::min(std::min(probs[b].k, mn) + probs[b].p, mn);
            if (std::min(l * (probs[b].q + 1), mn) > 1024)
                return fail(RSVD_ERR_INVALID, "problem " + std::to_string(b) +
                                                  ": the block-Krylov width min((k + p)(q + 1), m, n) must be <= 1024");
        }
    }
    P->krylov = krylov;
    P->single_view = single_view;
    if (fp64_final) P->fp64_from = (int)(2 * probs[0].q - 1);
    P->complex_omega = (flags & PLAN_CPLX_OMEGA) != 0;
    P->nprob = (int)batch;
    P->dt = dt;
    P->prec = fullsvd ? RSVD_PREC_F64 : prec;
    P->flags = flags;
    P->fullsvd = fullsvd;
    P->max_sweeps = JAC_MAX_SWEEPS_FULL;
    P->e_store = store_elem(dt);
    P->e_sketch = P->prec == RSVD_PREC_F64 ? E_F64 : (P->prec == RSVD_PREC_F32 ? E_F32 : E_BF16);
    P->e_y = P->prec == RSVD_PREC_F64 ? E_F64 : E_F32;
    P->need_cast = (P->prec == RSVD_PREC_BF16) || (P->prec == RSVD_PREC_F32 && dt == RSVD_F64);
    P->probs.resize(batch);
    for (int64_t b = 0; b < batch; ++b) {
        const rsvd_problem_t& p = probs[b];
        ProbHost& h = P->probs[b];
        h.m = p.m;
        h.n = p.n;
        h.lda = p.lda;
        const int64_t mn = std::min(p.m, p.n);
        h.k = std::min(p.k, mn);
        h.p = fullsvd ? 0 : p.p;
        h.q = (fullsvd || single_view) ? 0 : p.q;  // the single-view scheme has no power steps
        h.ldu = p.ldu ? p.ldu : h.k;
        h.ldvt = p.ldvt ? p.ldvt : p.n;
        h.seed = p.seed;
        h.delta = p.delta_trunc;
        if (fullsvd) {
            h.l = (int)mn;
            h.R = (int)mn;
            h.C = (int)std::max(p.m, p.n);
            h.mode = (p.m > p.n) ? 2 : 1;
            h.lq = false;
        } else {
            h.l = (int)std::min(h.k + p.p, mn);
            // rows of B: the sketch width, or the block-Krylov width min(l (q + 1), m, n)
            h.R = krylov ? (int)std::min<int64_t>((int64_t)h.l * (h.q + 1), mn) : h.l;
            h.lq = !(flags & RSVD_PLAN_SAVE) && !single_view &&
                   !((flags & RSVD_PLAN_NO_REFINE) && prec != RSVD_PREC_F64) && (double)p.n >= JAC_LQ_MIN_RATIO * h.R;
            h.sv_s = single_view ? (int)std::min<int64_t>(2 * (int64_t)h.l + 1, p.m) : 0;
            h.C = h.lq ? h.R : (int)p.n;
            h.mode = 0;
        }
        int nbk = (h.R + JAC_B - 1) / JAC_B;
        if (nbk % 2) ++nbk;
        if (nbk < 2) nbk = 2;
        h.nb = nbk;
        P->max_l = std::max(P->max_l, std::max(h.l, h.R));
        P->max_nb = std::max(P->max_nb, h.nb);
        P->max_q = std::max<int>(P->max_q, (int)h.q);
    }
    if (!fullsvd) P->max_sweeps = P->max_l > JAC_WIDE_L ? JAC_MAX_SWEEPS_RSVD_WIDE : JAC_MAX_SWEEPS_RSVD;
    if (!fullsvd) {
        // blocked Householder fallback for large bases (the one-workgroup form
        // reads the trailing matrix once per column), or when asked for
        double cost = 0.0;
        for (const ProbHost& h : P->probs) {
            const double rows = (double)std::max(h.m, h.n), w = (double)std::max(h.l, h.R);
            P->hh_rows = std::max<int>(P->hh_rows, (int)std::max(h.m, h.n));
            cost = std::max(cost, rows * w * w);
        }
        P->hh_blocked = P->hh_rows <= householder_blocked_rows_max() &&
                        ((flags & RSVD_PLAN_BLOCKED_QR) || cost >= HH_BLOCKED_MIN_COST);
    }
    layout(*P);
    return RSVD_OK;
}

int plan_create(const rsvd_problem_t* probs, int64_t batch, rsvd_dtype_t dt, rsvd_prec_t prec, unsigned flags,
                rsvd_plan** out)
{
    if (!out) return fail(RSVD_ERR_INVALID, "plan output pointer is null");
    *out = nullptr;
    rsvd_plan* P = new rsvd_plan();
    int rc = plan_setup(P, probs, batch, dt, prec, flags);
    if (rc == RSVD_OK) rc = kernels_ready();
    if (rc != RSVD_OK) {
        plan_free(P);
        return rc;
    }
    hipError_t e = hipMalloc(&P->ws, P->ws_bytes);
    if (e != hipSuccess) {
        plan_free(P);
        return fail(RSVD_ERR_ALLOC, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
    }
    // size the descriptor blob with placeholder pointers
    {
        std::vector<const void*> A(batch, (const void*)P->ws);
        std::vector<void*> O(batch, (void*)P->ws);
        build_blob(*P, A.data(), O.data(), O.data(), O.data(), (double*)P->ws, (int64_t*)P->ws, nullptr);
        P->blob_bytes = P->hb.bytes.size();
    }
    e = hipMalloc(&P->dblob, std::max<size_t>(P->blob_bytes, 64));
    if (e == hipSuccess) e = hipHostMalloc(&P->hblob_pinned, std::max<size_t>(P->blob_bytes, 64), 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->upload_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        plan_free(P);
        return fail(RSVD_ERR_ALLOC, std::string("plan allocation: ") + hipGetErrorString(e));
    }
    *out = P;
    return RSVD_OK;
}

// Builds and uploads the descriptor tables for these pointers unless the
// last upload was for the same ones.
int ensure_blob(rsvd_plan* P, const void* const* A, void* const* U, void* const* S, void* const* VT, double* w,
                int64_t* kk, int* info, hipStream_t stream)
{
    bool same = P->blob_valid && P->lastW == w && P->lastK == kk && P->lastInfo == info;
    if (same) {
        for (int b = 0; b < P->nprob && same; ++b)
            same = P->lastA[b] == A[b] && P->lastU[b] == U[b] && P->lastS[b] == S[b] && P->lastVT[b] == VT[b];
    }
    if (same) return RSVD_OK;
    if (P->upload_pending) HIPCHK(hipEventSynchronize(P->upload_done));
    build_blob(*P, A, U, S, VT, w, kk, info);
    if (P->hb.bytes.size() != P->blob_bytes) return fail(RSVD_ERR_HIP, "descriptor layout changed");
    memcpy(P->hblob_pinned, P->hb.bytes.data(), P->blob_bytes);
    HIPCHK(hipMemcpyAsync(P->dblob, P->hblob_pinned, P->blob_bytes, hipMemcpyHostToDevice, stream));
    HIPCHK(hipEventRecord(P->upload_done, stream));
    P->upload_pending = true;
    P->lastA.assign(A, A + P->nprob);
    P->lastU.assign(U, U + P->nprob);
    P->lastS.assign(S, S + P->nprob);
    P->lastVT.assign(VT, VT + P->nprob);
    P->lastW = w;
    P->lastK = kk;
    P->lastInfo = info;
    P->blob_valid = true;
    ++P->fwd_gen;
    return RSVD_OK;
}

int plan_execute(rsvd_plan* P, const void* const* A, void* const* U, void* const* S, void* const* VT, double* w,
                 int64_t* kk, int* info, hipStream_t stream)
{
    if (!P) return fail(RSVD_ERR_INVALID, "plan is null");
    if (!A || !U || !S || !VT || !w || !kk) return fail(RSVD_ERR_INVALID, "null output or input array");
    for (int b = 0; b < P->nprob; ++b)
        if (!A[b] || !U[b] || !S[b] || !VT[b]) return fail(RSVD_ERR_INVALID, "null matrix pointer in batch");
    int rc0 = ensure_blob(P, A, U, S, VT, w, kk, info, stream);
    if (rc0 != RSVD_OK) return rc0;
    P->fwd_saved = false;
    if ((P->flags & RSVD_PLAN_TUNE) && !P->tuned && !P->fullsvd) {
        // one eager execute that times the candidate tiles of every tunable
        // product on these inputs, then the descriptors with the chosen tiles
        P->tuner = true;
        int rc = enqueue(*P, stream);
        P->tuner = false;
        if (rc != RSVD_OK) {
            // a candidate's descriptors may be installed: let its copies finish, rebuild on the next execute
            (void)hipStreamSynchronize(stream);
            P->blob_valid = false;
            return rc;
        }
        HIPCHK(hipStreamSynchronize(stream));
        P->tuned = true;
        build_blob(*P, A, U, S, VT, w, kk, info);
        if (P->hb.bytes.size() != P->blob_bytes) return fail(RSVD_ERR_HIP, "descriptor layout changed");
        memcpy(P->hblob_pinned, P->hb.bytes.data(), P->blob_bytes);
        HIPCHK(hipMemcpyAsync(P->dblob, P->hblob_pinned, P->blob_bytes, hipMemcpyHostToDevice, stream));
        HIPCHK(hipEventRecord(P->upload_done, stream));
        P->upload_pending = true;
        ++P->fwd_gen;
    }
    if (P->flags & RSVD_PLAN_GRAPH) {
        if (!P->gexec) {
            HIPCHK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue(*P, P->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
            if (rc != RSVD_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(RSVD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            P->graph = g;
            HIPCHK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(P->gexec, stream));
    } else {
        int rc = enqueue(*P, stream);
        if (rc != RSVD_OK) return rc;
    }
    P->fwd_saved = (P->flags & RSVD_PLAN_SAVE) != 0 && !P->fullsvd;
    return RSVD_OK;
}

// ---------------------------------------------------------------- complex plans
}  // namespace

// RSVD_PLAN_COMPLEX: the problems are complex (A, U, VT interleaved complex
// double, S real).  Each runs as the real plan of its embedding
// At = [[Ar, -Ai], [Ai, Ar]] (2m x 2n, rank 2k, oversampling 2p, the same
// q and seed, the embedded complex Gaussian as test matrix, no truncation);
// the complex finishing step then picks one real triplet per pair, applies
// the truncation rule to the complex values and writes the complex outputs.
struct ComplexExt {
    rsvd_plan* inner = nullptr;
    char* ws = nullptr;  // per problem: At, the inner U, S, VT, sig; then the inner w, k_kept, info arrays
    size_t ws_bytes = 0;
    struct Prob {
        int64_t m, n, lda, k, ldu, ldvt;
        double delta;
        size_t o_at, o_u, o_s, o_vt, o_sig;
    };
    std::vector<Prob> probs;
    size_t o_w = 0, o_kk = 0, o_info = 0, o_info_local = 0;
    // descriptors of the embedding and finishing launches
    Blob hb;
    char* dblob = nullptr;
    char* hpinned = nullptr;
    size_t blob_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    IdxLaunch embed, cols;
    size_t off_cfin = 0;
    std::vector<const void*> lastA;
    std::vector<void*> lastU, lastS, lastVT;
    double* lastW = nullptr;
    int64_t* lastK = nullptr;
    int* lastInfo = nullptr;
    bool blob_valid = false;
};

namespace {

void complex_free(ComplexExt* X)
{
    if (!X) return;
    if (X->inner) plan_free(X->inner);
    if (X->ws) (void)hipFree(X->ws);
    if (X->dblob) (void)hipFree(X->dblob);
    if (X->hpinned) (void)hipHostFree(X->hpinned);
    if (X->upload_done) (void)hipEventDestroy(X->upload_done);
    delete X;
}

void complex_build_blob(rsvd_plan& P, const void* const* A, void* const* U, void* const* S, void* const* VT,
                        double* w, int64_t* kk, int* info)
{
    ComplexExt& X = *P.cx;
    const int np = P.nprob;
    Blob B;
    std::vector<CEmbedDesc> de(np);
    std::vector<CFinDesc> df(np);
    std::vector<int> ce(np), cc(np);
    for (int b = 0; b < np; ++b) {
        const ComplexExt::Prob& h = X.probs[b];
        CEmbedDesc& e = de[b];
        memset(&e, 0, sizeof(e));
        e.A = (const double*)A[b];
        e.At = (double*)(X.ws + h.o_at);
        e.lda = h.lda;
        e.ldt = 2 * h.n;
        e.m = (int)h.m;
        e.n = (int)h.n;
        ce[b] = (int)((h.m * h.n + 255) / 256);
        CFinDesc& f = df[b];
        memset(&f, 0, sizeof(f));
        f.Ur = (const double*)(X.ws + h.o_u);
        f.Sr = (const double*)(X.ws + h.o_s);
        f.VTr = (const double*)(X.ws + h.o_vt);
        f.normA2 = (const double*)(X.inner->ws + X.inner->probs[b].o_norm);
        f.wr = (const double*)(X.ws + X.o_w) + b;
        f.info_in = (const int*)(X.ws + X.o_info) + b;
        f.U = (double*)U[b];
        f.S = (double*)S[b];
        f.VT = (double*)VT[b];
        f.sig = (double*)(X.ws + h.o_sig);
        f.w_out = w + b;
        f.kkept_out = kk + b;
        f.info_out = info ? info + b : (int*)(X.ws + X.o_info_local) + b;
        f.ldu = h.ldu;
        f.ldvt = h.ldvt;
        f.m = (int)h.m;
        f.n = (int)h.n;
        f.k = (int)h.k;
        f.full = P.fullsvd ? 1 : 0;
        f.delta = h.delta;
        cc[b] = (int)h.k;
    }
    X.embed = add_idx(B, de, ce);
    X.cols = add_idx(B, df, cc);
    X.off_cfin = X.cols.off_desc;
    X.hb = std::move(B);
}

int complex_plan_create(const rsvd_problem_t* probs, int64_t batch, rsvd_dtype_t dt, rsvd_prec_t prec,
                        unsigned flags, rsvd_plan** out)
{
    if (!probs || batch < 1 || batch > (1 << 20)) return fail(RSVD_ERR_INVALID, "batch must be in [1, 2^20]");
    if (dt != RSVD_F64) return fail(RSVD_ERR_INVALID, "complex plans hold complex double (dtype RSVD_F64)");
    if (flags & RSVD_PLAN_SAVE) return fail(RSVD_ERR_INVALID, "complex plans have no adjoint (RSVD_PLAN_SAVE)");
    if (flags & RSVD_PLAN_SINGLE_VIEW) return fail(RSVD_ERR_INVALID, "complex plans have no single-view form");
    const bool full = (flags & RSVD_PLAN_FULLSVD) != 0;
    std::vector<rsvd_problem_t> in(batch);
    for (int64_t b = 0; b < batch; ++b) {
        const rsvd_problem_t& p = probs[b];
        int rc = validate_problem(p, full);
        if (rc != RSVD_OK) return fail(rc, "problem " + std::to_string(b) + ": " + g_err);
        const int64_t kk = std::min(p.k, std::min(p.m, p.n));
        rsvd_problem_t& q = in[b];
        q.m = 2 * p.m;
        q.n = 2 * p.n;
        q.lda = 2 * p.n;
        q.k = 2 * kk;
        q.p = 2 * p.p;
        q.q = p.q;
        q.seed = p.seed;
        q.delta_trunc = 0.0;  // the complex finishing step applies the cut
        q.ldu = 0;
        q.ldvt = 0;
    }
    rsvd_plan* P = new rsvd_plan();
    P->nprob = (int)batch;
    P->dt = dt;
    P->prec = full ? RSVD_PREC_F64 : prec;
    P->flags = flags;
    P->fullsvd = full;
    P->cx = new ComplexExt();
    ComplexExt& X = *P->cx;
    const unsigned inner_flags =
        (flags & (RSVD_PLAN_FULLSVD | RSVD_PLAN_NO_REFINE | RSVD_PLAN_ROUND_LAUNCHES | RSVD_PLAN_BLOCK_KRYLOV |
                  RSVD_PLAN_BLOCKED_QR)) |
        (full ? 0u : PLAN_CPLX_OMEGA);
    int rc = plan_create(in.data(), batch, RSVD_F64, prec, inner_flags, &X.inner);
    if (rc != RSVD_OK) {
        plan_free(P);
        return rc;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    X.probs.resize(batch);
    for (int64_t b = 0; b < batch; ++b) {
        const rsvd_problem_t& p = probs[b];
        ComplexExt::Prob& h = X.probs[b];
        h.m = p.m;
        h.n = p.n;
        h.lda = p.lda;
        h.k = std::min(p.k, std::min(p.m, p.n));
        h.ldu = p.ldu ? p.ldu : h.k;
        h.ldvt = p.ldvt ? p.ldvt : p.n;
        h.delta = p.delta_trunc;
        h.o_at = take(sizeof(double) * 4 * h.m * h.n);
        h.o_u = take(sizeof(double) * 2 * h.m * 2 * h.k);
        h.o_s = take(sizeof(double) * 2 * h.k);
        h.o_vt = take(sizeof(double) * 2 * h.k * 2 * h.n);
        h.o_sig = take(sizeof(double) * h.k);
    }
    X.o_w = take(sizeof(double) * batch);
    X.o_kk = take(sizeof(int64_t) * batch);
    X.o_info = take(sizeof(int) * batch);
    X.o_info_local = take(sizeof(int) * batch);
    X.ws_bytes = off;
    hipError_t e = hipMalloc(&X.ws, X.ws_bytes);
    if (e != hipSuccess) {
        plan_free(P);
        return fail(RSVD_ERR_ALLOC, std::string("complex workspace hipMalloc: ") + hipGetErrorString(e));
    }
    {
        std::vector<const void*> A(batch, (const void*)X.ws);
        std::vector<void*> O(batch, (void*)X.ws);
        complex_build_blob(*P, A.data(), O.data(), O.data(), O.data(), (double*)X.ws, (int64_t*)X.ws, nullptr);
        X.blob_bytes = X.hb.bytes.size();
    }
    e = hipMalloc(&X.dblob, std::max<size_t>(X.blob_bytes, 64));
    if (e == hipSuccess) e = hipHostMalloc(&X.hpinned, std::max<size_t>(X.blob_bytes, 64), 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&X.upload_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        plan_free(P);
        return fail(RSVD_ERR_ALLOC, std::string("complex plan allocation: ") + hipGetErrorString(e));
    }
    *out = P;
    return RSVD_OK;
}

// The embedding, the embedded plan's launches and the complex finishing step.
int complex_enqueue(rsvd_plan& P, hipStream_t s)
{
    ComplexExt& X = *P.cx;
    const int np = P.nprob;
    const char* db = X.dblob;
    PLAUNCH(RSVD_PHASE_STAGE, 0.0,
            launch_embed_complex((const CEmbedDesc*)(db + X.embed.off_desc), (const int*)(db + X.embed.off_begin), np,
                                 X.embed.total, s));
    X.inner->prof = P.prof;
    int rc = enqueue(*X.inner, s);
    X.inner->prof = nullptr;
    if (rc != RSVD_OK) return rc;
    PLAUNCH(RSVD_PHASE_FINISH, 0.0,
            launch_complex_finish((const CFinDesc*)(db + X.off_cfin), np, (const int*)(db + X.cols.off_begin),
                                  X.cols.total, s));
    return RSVD_OK;
}

int complex_execute(rsvd_plan* P, const void* const* A, void* const* U, void* const* S, void* const* VT, double* w,
                    int64_t* kk, int* info, hipStream_t stream, bool eager)
{
    ComplexExt& X = *P->cx;
    const int np = P->nprob;
    if (!A || !U || !S || !VT || !w || !kk) return fail(RSVD_ERR_INVALID, "null output or input array");
    for (int b = 0; b < np; ++b)
        if (!A[b] || !U[b] || !S[b] || !VT[b]) return fail(RSVD_ERR_INVALID, "null matrix pointer in batch");
    // the embedded plan's pointers are internal and never change
    {
        std::vector<const void*> Ai(np);
        std::vector<void*> Ui(np), Si(np), Vi(np);
        for (int b = 0; b < np; ++b) {
            Ai[b] = X.ws + X.probs[b].o_at;
            Ui[b] = X.ws + X.probs[b].o_u;
            Si[b] = X.ws + X.probs[b].o_s;
            Vi[b] = X.ws + X.probs[b].o_vt;
        }
        int rc = ensure_blob(X.inner, Ai.data(), Ui.data(), Si.data(), Vi.data(), (double*)(X.ws + X.o_w),
                             (int64_t*)(X.ws + X.o_kk), (int*)(X.ws + X.o_info), stream);
        if (rc != RSVD_OK) return rc;
    }
    bool same = X.blob_valid && X.lastW == w && X.lastK == kk && X.lastInfo == info;
    for (int b = 0; b < np && same; ++b)
        same = X.lastA[b] == A[b] && X.lastU[b] == U[b] && X.lastS[b] == S[b] && X.lastVT[b] == VT[b];
    if (!same) {
        if (X.upload_pending) HIPCHK(hipEventSynchronize(X.upload_done));
        complex_build_blob(*P, A, U, S, VT, w, kk, info);
        if (X.hb.bytes.size() != X.blob_bytes) return fail(RSVD_ERR_HIP, "descriptor layout changed");
        memcpy(X.hpinned, X.hb.bytes.data(), X.blob_bytes);
        HIPCHK(hipMemcpyAsync(X.dblob, X.hpinned, X.blob_bytes, hipMemcpyHostToDevice, stream));
        HIPCHK(hipEventRecord(X.upload_done, stream));
        X.upload_pending = true;
        X.lastA.assign(A, A + np);
        X.lastU.assign(U, U + np);
        X.lastS.assign(S, S + np);
        X.lastVT.assign(VT, VT + np);
        X.lastW = w;
        X.lastK = kk;
        X.lastInfo = info;
        X.blob_valid = true;
    }
    if ((P->flags & RSVD_PLAN_GRAPH) && !eager) {
        if (!P->gexec) {
            HIPCHK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = complex_enqueue(*P, P->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
            if (rc != RSVD_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(RSVD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            P->graph = g;
            HIPCHK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(P->gexec, stream));
        return RSVD_OK;
    }
    return eager ? RSVD_OK : complex_enqueue(*P, stream);
}

// ---------------------------------------------------------------- one-shot cache
struct CacheKey {
    int64_t m, n, lda, k, p, q, ldu, ldvt;
    int dt, prec, full;
    bool operator<(const CacheKey& o) const
    {
        return std::tie(m, n, lda, k, p, q, ldu, ldvt, dt, prec, full) <
               std::tie(o.m, o.n, o.lda, o.k, o.p, o.q, o.ldu, o.ldvt, o.dt, o.prec, o.full);
    }
};
struct CacheEntry {
    rsvd_plan* plan;
    int* info;  // device int for the status
    int device;
};
std::mutex g_cache_mu;
std::map<std::pair<int, CacheKey>, CacheEntry> g_cache;
constexpr size_t CACHE_MAX = 64;

int one_shot(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p, int64_t q,
             uint64_t seed, double delta, rsvd_prec_t prec, void* U, int64_t ldu, void* S, void* VT, int64_t ldvt,
             double* w, int64_t* kk, hipStream_t stream, bool full)
{
    if (!A || !U || !S || !VT || !w || !kk) return fail(RSVD_ERR_INVALID, "null pointer argument");
    rsvd_problem_t pr;
    pr.m = m;
    pr.n = n;
    pr.lda = lda;
    pr.k = k;
    pr.p = p;
    pr.q = q;
    pr.seed = seed;
    pr.delta_trunc = delta;
    pr.ldu = ldu;
    pr.ldvt = ldvt;
    int rc = validate_problem(pr, full);
    if (rc != RSVD_OK) return rc;
    if (ldu < std::min(k, std::min(m, n))) return fail(RSVD_ERR_INVALID, "ldu < k");
    if (ldvt < n) return fail(RSVD_ERR_INVALID, "ldvt < n");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    CacheKey key{m, n, lda, k, full ? 0 : p, full ? 0 : q, ldu, ldvt, (int)dt, full ? 0 : (int)prec, full ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find({dev, key});
    if (it == g_cache.end()) {
        if (g_cache.size() >= CACHE_MAX) {
            auto victim = g_cache.begin();
            int cur = dev;
            (void)hipSetDevice(victim->second.device);
            (void)hipDeviceSynchronize();
            plan_free(victim->second.plan);
            (void)hipFree(victim->second.info);
            (void)hipSetDevice(cur);
            g_cache.erase(victim);
        }
        rsvd_plan* P = nullptr;
        rc = plan_create(&pr, 1, dt, prec, RSVD_PLAN_GRAPH | (full ? RSVD_PLAN_FULLSVD : 0u), &P);
        if (rc != RSVD_OK) return rc;
        int* info = nullptr;
        hipError_t e = hipMalloc(&info, sizeof(int));
        if (e != hipSuccess) {
            plan_free(P);
            return fail(RSVD_ERR_ALLOC, "status allocation");
        }
        it = g_cache.emplace(std::make_pair(dev, key), CacheEntry{P, info, dev}).first;
    }
    rsvd_plan* P = it->second.plan;
    // per-call scalars live in the descriptors: force a rebuild when they change
    if (P->probs[0].seed != seed || P->probs[0].delta != delta) {
        P->probs[0].seed = seed;
        P->probs[0].delta = delta;
        P->blob_valid = false;
    }
    const void* Aa[1] = {A};
    void* Ua[1] = {U};
    void* Sa[1] = {S};
    void* Va[1] = {VT};
    rc = plan_execute(P, Aa, Ua, Sa, Va, w, kk, it->second.info, stream);
    if (rc != RSVD_OK) return rc;
    int h_info = 0;
    HIPCHK(hipMemcpyAsync(&h_info, it->second.info, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (h_info == RSVD_ERR_NONFINITE) return fail(RSVD_ERR_NONFINITE, "A contains NaN or Inf");
    if (h_info == RSVD_ERR_NOCONV) return fail(RSVD_ERR_NOCONV, "Jacobi sweep cap reached");
    return RSVD_OK;
}

}  // namespace

// ---------------------------------------------------------------- allocation-free one-shot
// Device memory of rsvd_truncate_noalloc: the workspace of one problem
// followed by its descriptor tables.  Each GPU holds its own copy of this
// array from the time the library is loaded until the process ends.
static __device__ __align__(256) char scratch[RSVD_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch;  // device -> address of that device's scratch

// The device address of the current device's scratch, taken once per device
// with that device current.  In host code the array's name is a stand-in, not
// a device address; only this pointer is passed to kernels.
int scratch_address(int dev, char** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(RSVD_ERR_HIP, "scratch symbol has no device address");
        it = g_scratch.emplace(dev, (char*)ptr).first;
    }
    *out = it->second;
    return RSVD_OK;
}

int noalloc_truncate(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
                     int64_t q, uint64_t seed, double delta, rsvd_prec_t prec, void* U, int64_t ldu, void* S,
                     void* VT, int64_t ldvt, double* w, int64_t* kk, int* info, hipStream_t stream)
{
    if (!A || !U || !S || !VT || !w || !kk) return fail(RSVD_ERR_INVALID, "null pointer argument");
    if (dt != RSVD_F64 && dt != RSVD_F32) return fail(RSVD_ERR_INVALID, "unknown dtype");
    if (prec != RSVD_PREC_F64 && prec != RSVD_PREC_F32 && prec != RSVD_PREC_BF16)
        return fail(RSVD_ERR_INVALID, "unknown precision");
    rsvd_problem_t pr;
    pr.m = m;
    pr.n = n;
    pr.lda = lda;
    pr.k = k;
    pr.p = p;
    pr.q = q;
    pr.seed = seed;
    pr.delta_trunc = delta;
    pr.ldu = ldu;
    pr.ldvt = ldvt;
    int rc = validate_problem(pr, false);
    if (rc != RSVD_OK) return rc;
    if (ldu < std::min(k, std::min(m, n))) return fail(RSVD_ERR_INVALID, "ldu < k");
    if (ldvt < n) return fail(RSVD_ERR_INVALID, "ldvt < n");
    // the host side of a one-problem plan, without graph, tuning or saved forward
    rsvd_plan P;
    if ((rc = plan_setup(&P, &pr, 1, dt, prec, 0u)) != RSVD_OK) return rc;
    const size_t ws = align_up(P.ws_bytes, 256);
    if (ws > (size_t)RSVD_NOALLOC_SCRATCH_BYTES)
        return fail(RSVD_ERR_INVALID, "problem needs " + std::to_string(ws) + " bytes of workspace; the scratch holds " +
                                          std::to_string((long long)RSVD_NOALLOC_SCRATCH_BYTES));
    if ((rc = kernels_ready()) != RSVD_OK) return rc;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    char* base = nullptr;
    if ((rc = scratch_address(dev, &base)) != RSVD_OK) return rc;
    P.ws = base;
    const void* Aa[1] = {A};
    void* Ua[1] = {U};
    void* Sa[1] = {S};
    void* Va[1] = {VT};
    build_blob(P, Aa, Ua, Sa, Va, w, kk, info);
    P.blob_bytes = P.hb.bytes.size();
    if (ws + P.blob_bytes > (size_t)RSVD_NOALLOC_SCRATCH_BYTES) {
        P.ws = nullptr;
        return fail(RSVD_ERR_INVALID, "problem needs " + std::to_string(ws + P.blob_bytes) +
                                          " bytes of workspace and descriptors; the scratch holds " +
                                          std::to_string((long long)RSVD_NOALLOC_SCRATCH_BYTES));
    }
    P.dblob = base + ws;
    hipError_t e = launch_upload(P.dblob, P.hb.bytes.data(), P.blob_bytes, stream);
    if (e == hipSuccess) rc = enqueue(P, stream);
    else rc = fail(RSVD_ERR_HIP, std::string("descriptor upload: ") + hipGetErrorString(e));
    // the scratch is not the plan's to free
    P.ws = nullptr;
    P.dblob = nullptr;
    return rc;
}

}  // namespace

extern "C" {

int rsvd_truncate_noalloc(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
                          int64_t q, uint64_t seed, double delta_trunc, rsvd_prec_t prec, void* U, int64_t ldu,
                          void* S, void* VT, int64_t ldvt, double* discarded_weight, int64_t* k_kept, int* info,
                          void* stream)
{
    g_err.clear();
    return noalloc_truncate(A, dt, m, n, lda, k, p, q, seed, delta_trunc, prec, U, ldu, S, VT, ldvt,
                            discarded_weight, k_kept, info, (hipStream_t)stream);
}

int rsvd_truncate(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
                  int64_t q, uint64_t seed, double delta_trunc, rsvd_prec_t prec, void* U, int64_t ldu, void* S,
                  void* VT, int64_t ldvt, double* discarded_weight, int64_t* k_kept, void* stream)
{
    g_err.clear();
    if (dt != RSVD_F64 && dt != RSVD_F32) return fail(RSVD_ERR_INVALID, "unknown dtype");
    if (prec != RSVD_PREC_F64 && prec != RSVD_PREC_F32 && prec != RSVD_PREC_BF16)
        return fail(RSVD_ERR_INVALID, "unknown precision");
    return one_shot(A, dt, m, n, lda, k, p, q, seed, delta_trunc, prec, U, ldu, S, VT, ldvt, discarded_weight,
                    k_kept, (hipStream_t)stream, false);
}

int rsvd_truncate_adaptive(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k0,
                           int64_t k_max, int64_t p, int64_t q, uint64_t seed, double delta_trunc,
                           rsvd_prec_t prec, void* U, int64_t ldu, void* S, void* VT, int64_t ldvt,
                           double* discarded_weight, int64_t* k_kept, int* attempts, void* stream)
{
    g_err.clear();
    if (dt != RSVD_F64 && dt != RSVD_F32) return fail(RSVD_ERR_INVALID, "unknown dtype");
    if (prec != RSVD_PREC_F64 && prec != RSVD_PREC_F32 && prec != RSVD_PREC_BF16)
        return fail(RSVD_ERR_INVALID, "unknown precision");
    if (!(delta_trunc > 0.0) || !(delta_trunc < INFINITY))
        return fail(RSVD_ERR_INVALID, "the adaptive rank needs a finite delta_trunc > 0");
    if (k0 < 1 || k_max < k0) return fail(RSVD_ERR_INVALID, "need 1 <= k0 <= k_max");
    if (m < 1 || n < 1) return fail(RSVD_ERR_INVALID, "m, n must be >= 1");
    if (!U || !S || !VT || !discarded_weight || !k_kept) return fail(RSVD_ERR_INVALID, "null pointer argument");
    const int64_t kcap = std::min(k_max, std::min(m, n));
    if (ldu < kcap) return fail(RSVD_ERR_INVALID, "ldu < min(k_max, m, n)");
    const hipStream_t s = (hipStream_t)stream;
    int64_t k = std::min(k0, kcap);
    int runs = 0;
    for (;;) {
        const int rc = one_shot(A, dt, m, n, lda, k, p, q, seed, delta_trunc, prec, U, ldu, S, VT, ldvt,
                                discarded_weight, k_kept, s, false);
        ++runs;
        if (rc != RSVD_OK) {
            if (attempts) *attempts = runs;
            return rc;
        }
        int64_t kk = 0;
        HIPCHK(hipMemcpy(&kk, k_kept, sizeof(int64_t), hipMemcpyDeviceToHost));
        if (kk < k || k >= kcap) break;  // the cut binds inside the sketch, or the rank cap is reached
        k = std::min(2 * k, kcap);
    }
    // triplets of the last run beyond its k_kept are zero; zero the ones beyond its k as well
    const size_t es = dt == RSVD_F64 ? sizeof(double) : sizeof(float);
    if (k < kcap) {
        HIPCHK(hipMemset2DAsync((char*)U + k * es, ldu * es, 0, (kcap - k) * es, m, s));
        HIPCHK(hipMemsetAsync((char*)S + k * es, 0, (kcap - k) * es, s));
        HIPCHK(hipMemset2DAsync((char*)VT + k * ldvt * es, ldvt * es, 0, n * es, kcap - k, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    if (attempts) *attempts = runs;
    return RSVD_OK;
}

int fullsvd_truncate(const void* A, rsvd_dtype_t dt, int64_t m, int64_t n, int64_t lda, int64_t k,
                     double delta_trunc, void* U, int64_t ldu, void* S, void* VT, int64_t ldvt,
                     double* discarded_weight, int64_t* k_kept, void* stream)
{
    g_err.clear();
    if (dt != RSVD_F64 && dt != RSVD_F32) return fail(RSVD_ERR_INVALID, "unknown dtype");
    return one_shot(A, dt, m, n, lda, k, 0, 0, 0, delta_trunc, RSVD_PREC_F64, U, ldu, S, VT, ldvt,
                    discarded_weight, k_kept, (hipStream_t)stream, true);
}

int rsvd_plan_create(const rsvd_problem_t* probs, int64_t batch, rsvd_dtype_t dt, rsvd_prec_t prec,
                     unsigned flags, rsvd_plan_t** plan)
{
    g_err.clear();
    if (flags & PLAN_CPLX_OMEGA) return fail(RSVD_ERR_INVALID, "unknown plan flag");
    if (flags & RSVD_PLAN_COMPLEX) {
        if (!plan) return fail(RSVD_ERR_INVALID, "plan output pointer is null");
        *plan = nullptr;
        return complex_plan_create(probs, batch, dt, prec, flags, plan);
    }
    return plan_create(probs, batch, dt, prec, flags, plan);
}

int rsvd_plan_execute(rsvd_plan_t* plan, const void* const* A, void* const* U, void* const* S, void* const* VT,
                      double* discarded_weight, int64_t* k_kept, int* info, void* stream)
{
    g_err.clear();
    if (plan && plan->cx)
        return complex_execute(plan, A, U, S, VT, discarded_weight, k_kept, info, (hipStream_t)stream, false);
    return plan_execute(plan, A, U, S, VT, discarded_weight, k_kept, info, (hipStream_t)stream);
}

int rsvd_gaussian(uint64_t seed, int64_t n, int64_t l, double* omega, void* stream)
{
    g_err.clear();
    if (n < 1 || l < 1 || n > (1 << 24) || l > (1 << 24) || !omega) return fail(RSVD_ERR_INVALID, "bad size or null");
    if ((n + 1) / 2 * l > ((int64_t)1 << 31) * 255) return fail(RSVD_ERR_INVALID, "too large");
    OmegaDesc d;
    memset(&d, 0, sizeof(d));
    d.Om = omega;
    d.seed = seed;
    d.n = (int)n;
    d.l = (int)l;
    d.elem = E_F64;
    const int64_t pairs = (n + 1) / 2 * l;
    const int nblk = (int)((pairs + 255) / 256);
    const std::vector<int> map = item_map(std::vector<int>(1, nblk));
    hipStream_t s = (hipStream_t)stream;
    OmegaDesc* dd = nullptr;
    int* db = nullptr;
    HIPCHK(hipMalloc(&dd, sizeof(d)));
    hipError_t e = hipMalloc(&db, sizeof(int) * map.size());
    if (e == hipSuccess) e = hipMemcpyAsync(dd, &d, sizeof(d), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(db, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_omega(dd, db, 1, nblk, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dd);
    if (db) (void)hipFree(db);
    if (e != hipSuccess) return fail(RSVD_ERR_HIP, std::string("rsvd_gaussian: ") + hipGetErrorString(e));
    return RSVD_OK;
}

int rsvd_philox4x32_10(const uint32_t* in, uint32_t* out, int64_t count, void* stream)
{
    g_err.clear();
    if (count < 0 || (count > 0 && (!in || !out))) return fail(RSVD_ERR_INVALID, "bad count or null");
    HIPCHK(launch_philox_words(in, out, count, (hipStream_t)stream));
    return RSVD_OK;
}

int rsvd_plan_profile(rsvd_plan_t* plan, const void* const* A, void* const* U, void* const* S, void* const* VT,
                      double* discarded_weight, int64_t* k_kept, int* info, double* ms, int64_t* launches,
                      double* flops, int ncat, void* stream)
{
    g_err.clear();
    if (!plan || !ms || !launches || !flops || ncat < 1) return fail(RSVD_ERR_INVALID, "null profile output");
    hipStream_t s = (hipStream_t)stream;
    const unsigned saved = plan->flags;
    plan->flags &= ~RSVD_PLAN_GRAPH;  // eager launches so that each can be timed
    Profiler prof;
    prof.s = s;
    int rc;
    if (plan->cx) {
        rc = complex_execute(plan, A, U, S, VT, discarded_weight, k_kept, info, s, true);  // uploads descriptors
        if (rc == RSVD_OK) {
            plan->prof = &prof;
            rc = complex_enqueue(*plan, s);
            plan->prof = nullptr;
        }
    } else {
        rc = plan_execute(plan, A, U, S, VT, discarded_weight, k_kept, info, s);  // uploads descriptors
        if (rc == RSVD_OK) {
            plan->prof = &prof;
            rc = enqueue(*plan, s);
            plan->prof = nullptr;
        }
    }
    plan->flags = saved;
    if (rc != RSVD_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 0; c < ncat; ++c) {
        ms[c] = 0.0;
        launches[c] = 0;
        flops[c] = 0.0;
    }
    for (size_t i = 0; i < prof.used; ++i) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, prof.ev[2 * i], prof.ev[2 * i + 1]));
        const int c = prof.cat[i];
        if (c < ncat) {
            ms[c] += t;
            launches[c] += 1;
            flops[c] += prof.flops[i];
        }
    }
    // Jacobi work from the device counters of the profiled execute
    if (RSVD_PHASE_JACOBI < ncat) {
        std::vector<int> st(2);
        const rsvd_plan* jp = plan->cx ? plan->cx->inner : plan;
        for (const ProbHost& h : jp->probs) {
            HIPCHK(hipMemcpy(st.data(), jp->ws + h.o_stats, 2 * sizeof(int), hipMemcpyDeviceToHost));
            flops[RSVD_PHASE_JACOBI] += 2.0 * (2 * JAC_B) * (2 * JAC_B) * (h.C * (double)st[0] + ((double)h.C + h.R) * st[1]);
        }
    }
    return RSVD_OK;
}

int rsvd_plan_backward(rsvd_plan_t* plan, const void* const* dU, const void* const* dS, const void* const* dVT,
                       void* const* dA, double broadening, void* stream)
{
    g_err.clear();
    return plan_backward(plan, dU, dS, dVT, dA, broadening, (hipStream_t)stream, false);
}

int rsvd_plan_profile_backward(rsvd_plan_t* plan, const void* const* dU, const void* const* dS,
                               const void* const* dVT, void* const* dA, double broadening, double* ms,
                               int64_t* launches, double* flops, int ncat, void* stream)
{
    g_err.clear();
    if (!plan || !ms || !launches || !flops || ncat < 1) return fail(RSVD_ERR_INVALID, "null profile output");
    hipStream_t s = (hipStream_t)stream;
    Profiler prof;
    prof.s = s;
    plan->prof = &prof;
    int rc = plan_backward(plan, dU, dS, dVT, dA, broadening, s, true);
    plan->prof = nullptr;
    if (rc != RSVD_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 0; c < ncat; ++c) {
        ms[c] = 0.0;
        launches[c] = 0;
        flops[c] = 0.0;
    }
    for (size_t i = 0; i < prof.used; ++i) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, prof.ev[2 * i], prof.ev[2 * i + 1]));
        const int c = prof.cat[i];
        if (c < ncat) {
            ms[c] += t;
            launches[c] += 1;
            flops[c] += prof.flops[i];
        }
    }
    return RSVD_OK;
}

int rsvd_plan_postselect(rsvd_plan_t* plan, int64_t chi, int64_t* chi_s, void* stream)
{
    g_err.clear();
    if (!plan) return fail(RSVD_ERR_INVALID, "plan is null");
    if (plan->cx) return fail(RSVD_ERR_INVALID, "post-selection is not available for complex plans");
    if (plan->single_view)
        return fail(RSVD_ERR_INVALID, "post-selection is not available for single-view plans (w is not sum sigma^2)");
    if (!chi_s) return fail(RSVD_ERR_INVALID, "chi_s is null");
    if (chi < 0) return fail(RSVD_ERR_INVALID, "chi must be >= 0");
    if (!plan->blob_valid) return fail(RSVD_ERR_INVALID, "postselect needs a preceding rsvd_plan_execute");
    if (plan->nprob > SELECT_MAX_SECTORS) return fail(RSVD_ERR_INVALID, "postselect supports at most 8192 problems");
    const hipStream_t s = (hipStream_t)stream;
    int64_t cand = 0;
    for (const ProbHost& h : plan->probs) cand += h.k;
    HIPCHK(launch_postselect(dp<FinDesc>(*plan, plan->signfix.off_desc), plan->nprob, cand, chi, chi_s,
                             plan->dt == RSVD_F64 ? 1 : 0, s));
    return RSVD_OK;
}

int64_t rsvd_plan_workspace_bytes(const rsvd_plan_t* plan)
{
    if (!plan) return 0;
    if (plan->cx) return (int64_t)(plan->cx->ws_bytes + plan->cx->inner->ws_bytes);
    return (int64_t)plan->ws_bytes;
}

int rsvd_plan_tiles(const rsvd_plan_t* plan, int32_t* tiles, int64_t cap, int64_t* count)
{
    g_err.clear();
    if (!plan || !count || cap < 0 || (cap > 0 && !tiles)) return fail(RSVD_ERR_INVALID, "null argument or negative cap");
    int64_t c = 0;
    for (int t : plan->slot_tile) {
        if (t < 0) continue;
        if (c < cap) {
            tiles[2 * c] = gemm_tile_m((GemmTile)t);
            tiles[2 * c + 1] = gemm_tile_n((GemmTile)t);
        }
        ++c;
    }
    *count = c;
    return RSVD_OK;
}

int rsvd_plan_set_tiles(rsvd_plan_t* plan, const int32_t* tiles, int64_t count)
{
    g_err.clear();
    if (!plan || (count > 0 && !tiles)) return fail(RSVD_ERR_INVALID, "null plan or tiles");
    int64_t n = 0;
    for (int t : plan->slot_tile) n += t >= 0;
    if (count != n) return fail(RSVD_ERR_INVALID, "count must equal the plan's number of tunable products (" +
                                                      std::to_string(n) + ")");
    std::vector<int> chosen((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int t = -1;
        for (int c = GT_64x64; c <= GT_128x128; ++c)
            if (gemm_tile_m((GemmTile)c) == tiles[2 * i] && gemm_tile_n((GemmTile)c) == tiles[2 * i + 1]) t = c;
        if (t < 0) return fail(RSVD_ERR_INVALID, "tile " + std::to_string(i) + " is not 64x64, 128x64, 64x128 or 128x128");
        chosen[(size_t)i] = t;
    }
    HIPCHK(hipDeviceSynchronize());  // no execute of this plan may still use its graph or descriptors
    plan->tile_ovr.assign(plan->slot_tile.size(), -1);
    int64_t i = 0;
    for (size_t slot = 0; slot < plan->slot_tile.size(); ++slot)
        if (plan->slot_tile[slot] >= 0) {
            plan->tile_ovr[slot] = chosen[(size_t)i];
            plan->slot_tile[slot] = chosen[(size_t)i++];
        }
    plan->tuned = true;
    plan->blob_valid = false;  // the next execute rebuilds and uploads the descriptors
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->gexec = nullptr;
    plan->graph = nullptr;
    return RSVD_OK;
}

void rsvd_plan_destroy(rsvd_plan_t* plan) { plan_free(plan); }

const char* rsvd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
