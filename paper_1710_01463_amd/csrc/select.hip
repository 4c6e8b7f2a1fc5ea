// Sector post-selection (paper Sec. III.A, symmetric tensor networks): a
// block-diagonal matrix is truncated block by block, each symmetry sector with
// its own RSVD of a guessed rank chi'_s; afterwards the chi largest singular
// values over all sectors are kept, which fixes the block dimensions chi_s.
//
// The candidates are the k_kept leading values of every problem of a plan
// (each sorted descending by the finishing step).  A single workgroup finds
// the chi-th largest by an 8-pass radix select on the bit patterns of the
// values (non-negative doubles order like their unsigned bit patterns), then
// counts per sector the values above it and hands the values equal to it to
// the sectors in index order, so the kept set is the first chi of the total
// order (value descending, sector ascending, index ascending) and is a prefix
// of every sector.  A second, per-sector launch drops the rest: it adds their
// squares to the discarded weight, zero-fills S, the columns of U and the rows
// of V^T, and lowers k_kept.
#include "common.hpp"
#include "kernels.hpp"

namespace rsvd {

constexpr int SEL_NT = 1024;

template <typename TO> __device__ __forceinline__ uint64_t sel_key(TO v)
{
    const double x = (double)v;
    return (x > 0.0) ? (uint64_t)__double_as_longlong(x) : 0ull;  // zero, -0 and NaN rank last
}

// sector of flat candidate e: the largest b with off[b] <= e
__device__ __forceinline__ int sel_sector(const int* off, int nprob, int e)
{
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int SEL_REG = 16;  // candidates per thread held in registers (total <= SEL_NT * SEL_REG)
constexpr int SEL_WAVES = SEL_NT / 64;

// In-place exclusive prefix sum of a[0..n) by all SEL_NT threads (each thread
// sums a contiguous chunk, the chunk totals are scanned by wave shuffles and
// across waves through LDS); returns the total.  Ends with a barrier.
__device__ int sel_exclusive_scan(int* a, int n, int* wave_tot)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + SEL_NT - 1) / SEL_NT, lo = tid * per, hi = min(n, lo + per);
    int own = 0;
    for (int i = lo; i < hi; ++i) own += a[i];
    int incl = own;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < SEL_WAVES; ++w) {
        before += (w < wave) ? wave_tot[w] : 0;
        total += wave_tot[w];
    }
    int run = before + incl - own;
    for (int i = lo; i < hi; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

template <typename TO, bool REG>
__global__ __launch_bounds__(SEL_NT) void select_kernel(const FinDesc* __restrict__ descs, int nprob, int64_t chi,
                                                        int64_t* __restrict__ chi_s)
{
    extern __shared__ int sel_lds[];
    int* off = sel_lds;         // nprob + 1 candidate offsets
    int* gt = off + nprob + 1;  // per sector: values above the threshold
    int* eq = gt + nprob;       // per sector: values equal to it (then: how many of them are kept)
    __shared__ unsigned int hist[SEL_WAVES][256];  // one histogram per wave: fewer colliding atomics
    __shared__ unsigned long long sh_prefix, sh_rem;
    __shared__ int wave_tot[SEL_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int b = tid; b < nprob; b += SEL_NT) {
        const int64_t kk = *to_glb(descs[b].kkept_out);
        off[b] = (int)(kk < 0 ? 0 : (kk > descs[b].k ? descs[b].k : kk));
    }
    __syncthreads();
    const int total = sel_exclusive_scan(off, nprob, wave_tot);
    if (tid == 0) off[nprob] = total;
    __syncthreads();
    if (chi <= 0 || total <= chi) {
        for (int b = tid; b < nprob; b += SEL_NT) chi_s[b] = chi <= 0 ? 0 : off[b + 1] - off[b];
        return;
    }
    // candidate e = tid + SEL_NT u: its key and sector, kept in registers when they fit
    uint64_t rkey[REG ? SEL_REG : 1];
    int rsec[REG ? SEL_REG : 1];
    auto fetch = [&](int e, uint64_t& key, int& b) {
        b = sel_sector(off, nprob, e);
        key = sel_key(((const GLB TO*)descs[b].S)[e - off[b]]);
    };
    if constexpr (REG) {
#pragma unroll
        for (int u = 0; u < SEL_REG; ++u) {
            const int e = tid + SEL_NT * u;
            rkey[u] = 0;
            rsec[u] = -1;
            if (e < total) fetch(e, rkey[u], rsec[u]);
        }
    }

    // radix select of the chi-th largest key, 8 bits at a time from the top
    uint64_t prefix = 0, mask = 0, rem = (uint64_t)chi;
    for (int dg = 7; dg >= 0; --dg) {
        for (int i = tid; i < SEL_WAVES * 256; i += SEL_NT) (&hist[0][0])[i] = 0;
        __syncthreads();
        auto count = [&](uint64_t key) {
            if ((key & mask) == prefix) atomicAdd(&hist[wave][(key >> (8 * dg)) & 255u], 1u);
        };
        if constexpr (REG) {
#pragma unroll
            for (int u = 0; u < SEL_REG; ++u)
                if (rsec[u] >= 0) count(rkey[u]);
        } else {
            for (int e = tid; e < total; e += SEL_NT) {
                uint64_t key;
                int b;
                fetch(e, key, b);
                count(key);
            }
        }
        __syncthreads();
        for (int i = tid; i < 256; i += SEL_NT) {
            unsigned int c = 0;
            for (int w = 0; w < SEL_WAVES; ++w) c += hist[w][i];
            hist[0][i] = c;
        }
        __syncthreads();
        if (wave == 0) {
            // lane L holds bins 255 - 4L .. 252 - 4L; the count above its bins
            // comes from a prefix sum over lanes; the lane whose bins reach rem
            // picks the bin (bin 0 if none does)
            unsigned int hb[4], own = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                hb[t] = hist[0][255 - 4 * lane - t];
                own += hb[t];
            }
            uint64_t incl = own;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint64_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            uint64_t cum = incl - own;
            if (cum < rem && (rem <= incl || lane == 63)) {
                int bin = 252 - 4 * lane;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (cum + hb[t] >= rem || t == 3) {
                        bin = 255 - 4 * lane - t;
                        break;
                    }
                    cum += hb[t];
                }
                sh_rem = rem - cum;
                sh_prefix = prefix | ((uint64_t)bin << (8 * dg));
            }
        }
        __syncthreads();
        prefix = sh_prefix;
        rem = sh_rem;
        mask |= 255ull << (8 * dg);
        __syncthreads();
    }

    // per sector: values above the chi-th key, and the equal ones in sector order
    for (int b = tid; b < nprob; b += SEL_NT) {
        gt[b] = 0;
        eq[b] = 0;
    }
    __syncthreads();
    auto classify = [&](uint64_t key, int b) {
        if (key > prefix) atomicAdd(&gt[b], 1);
        else if (key == prefix) atomicAdd(&eq[b], 1);
    };
    if constexpr (REG) {
#pragma unroll
        for (int u = 0; u < SEL_REG; ++u)
            if (rsec[u] >= 0) classify(rkey[u], rsec[u]);
    } else {
        for (int e = tid; e < total; e += SEL_NT) {
            uint64_t key;
            int b;
            fetch(e, key, b);
            classify(key, b);
        }
    }
    __syncthreads();
    // the equal values go to the sectors in order: sector b takes
    // clamp(rem - (equal values of the sectors before it), 0, eq[b])
    for (int b = tid; b < nprob; b += SEL_NT) off[b] = eq[b];
    __syncthreads();
    sel_exclusive_scan(off, nprob, wave_tot);
    for (int b = tid; b < nprob; b += SEL_NT) {
        const int64_t left = (int64_t)rem - off[b];
        const int take = left <= 0 ? 0 : (left < eq[b] ? (int)left : eq[b]);
        chi_s[b] = gt[b] + take;
    }
}

template <typename TO>
__global__ __launch_bounds__(256) void drop_kernel(const FinDesc* __restrict__ descs,
                                                   const int64_t* __restrict__ chi_s)
{
    __shared__ double red[256];
    const FinDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x;
    const int64_t kk64 = *to_glb(d.kkept_out);
    const int kk = (int)(kk64 < 0 ? 0 : (kk64 > d.k ? d.k : kk64));
    const int cs = (int)to_glb(chi_s)[blockIdx.x];
    if (cs >= kk) return;
    GLB TO* __restrict__ S = (GLB TO*)d.S;
    GLB TO* __restrict__ U = (GLB TO*)d.U;
    GLB TO* __restrict__ VT = (GLB TO*)d.VT;
    double part = 0.0;
    for (int j = cs + tid; j < kk; j += 256) {
        const double v = (double)S[j];
        part = fma(v, v, part);
    }
    red[tid] = part;
    __syncthreads();  // every read of S is done before it is zeroed below
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        *to_glb(d.w_out) += red[0];
        *to_glb(d.kkept_out) = cs;
    }
    const int n = d.n, m = d.m;
    GLB double* __restrict__ sgn = to_glb(d.sgn);
    for (int j = cs + tid; j < kk; j += 256) {
        S[j] = (TO)0;
        if (sgn) sgn[j] = 0.0;
    }
    const int lane = tid & 63, wave = tid >> 6;
    for (int r = cs + wave; r < kk; r += 4)
        for (int c = lane; c < n; c += 64) VT[(int64_t)r * d.ldvt + c] = (TO)0;
    for (int i = wave; i < m; i += 4)
        for (int c = cs + lane; c < kk; c += 64) U[(int64_t)i * d.ldu + c] = (TO)0;
}

size_t select_lds_bytes(int nprob) { return (size_t)(3 * nprob + 1) * sizeof(int); }

hipError_t launch_postselect(const FinDesc* d, int nprob, int64_t max_candidates, int64_t chi, int64_t* chi_s,
                             int out_f64, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    const size_t lds = select_lds_bytes(nprob);
    const bool reg = max_candidates <= (int64_t)SEL_NT * SEL_REG;
    if (out_f64) {
        if (reg)
            hipLaunchKernelGGL((select_kernel<double, true>), dim3(1), dim3(SEL_NT), lds, s, d, nprob, chi, chi_s);
        else
            hipLaunchKernelGGL((select_kernel<double, false>), dim3(1), dim3(SEL_NT), lds, s, d, nprob, chi, chi_s);
        hipLaunchKernelGGL(drop_kernel<double>, dim3(nprob), dim3(256), 0, s, d, chi_s);
    } else {
        if (reg)
            hipLaunchKernelGGL((select_kernel<float, true>), dim3(1), dim3(SEL_NT), lds, s, d, nprob, chi, chi_s);
        else
            hipLaunchKernelGGL((select_kernel<float, false>), dim3(1), dim3(SEL_NT), lds, s, d, nprob, chi, chi_s);
        hipLaunchKernelGGL(drop_kernel<float>, dim3(nprob), dim3(256), 0, s, d, chi_s);
    }
    return hipGetLastError();
}

hipError_t init_select_kernels()
{
    const int bytes = (int)select_lds_bytes(SELECT_MAX_SECTORS);
    const void* fns[4] = {(const void*)select_kernel<double, true>, (const void*)select_kernel<double, false>,
                          (const void*)select_kernel<float, true>, (const void*)select_kernel<float, false>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rsvd
