// Input staging, the Gaussian test matrix, and small fills.
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"
#include "philox.hpp"

namespace rsvd {

template <typename T> __device__ __forceinline__ double ldv(const void* p, int64_t i)
{
    return to_f64(((const GLB T*)p)[i]);
}
__device__ __forceinline__ double load_elem(const void* p, int elem, int64_t i)
{
    if (elem == E_F64) return ldv<double>(p, i);
    if (elem == E_F32) return ldv<float>(p, i);
    return ldv<__bf16>(p, i);
}
__device__ __forceinline__ void store_elem(void* p, int elem, int64_t i, double v)
{
    if (elem == E_F64)
        ((GLB double*)p)[i] = v;
    else if (elem == E_F32)
        ((GLB float*)p)[i] = (float)v;
    else
        ((GLB __bf16*)p)[i] = from_f64<__bf16>(v);
}

// ||A||_F^2 over a chunk of STAGE_ROWS rows (fixed reduction order), plus the
// optional cast of those rows into the compact copy used by the low-precision
// products.  A stored FP32 is cast from its exact FP32 value.
__global__ __launch_bounds__(256) void stage_kernel(const StageDesc* __restrict__ descs,
                                                    const int* __restrict__ chunk_begin, int nprob)
{
    __shared__ double red[4];
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(chunk_begin, t);
    const int b = wi_.x;
    const StageDesc& d = descs[b];
    const int c = wi_.y;
    const int r0 = c * STAGE_ROWS;
    const int nr = min(STAGE_ROWS, d.m - r0);
    const int n = d.n;
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int base = tid; base < nr * n; base += 256 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + 256 * u;
            v[u] = (e < nr * n) ? load_elem(d.A, d.a_elem, (int64_t)(r0 + e / n) * d.lda + e % n) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = base + 256 * u;
            s = fma(v[u], v[u], s);
            if (d.Acast && e < nr * n) store_elem(d.Acast, d.cast_elem, (int64_t)(r0 + e / n) * n + e % n, v[u]);
        }
    }
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) to_glb(d.partial)[c] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void stage_final_kernel(const StageDesc* __restrict__ descs, int nprob)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    const StageDesc& d = descs[b];
    double s = 0.0, c = 0.0;
    for (int i = 0; i < d.nchunks; ++i) {
        const double x = to_glb(d.partial)[i];
        const double tsum = s + x;
        if (fabs(s) >= fabs(x)) c += (s - tsum) + x; else c += (x - tsum) + s;
        s = tsum;
    }
    *to_glb(d.normA2) = s + c;
}

hipError_t launch_stage(const StageDesc* d, const int* chunk_begin, int nprob, int total_chunks,
                        hipStream_t s)
{
    if (total_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(stage_kernel, dim3(total_chunks), dim3(256), 0, s, d, chunk_begin, nprob);
    return hipGetLastError();
}

hipError_t launch_stage_final(const StageDesc* d, int nprob, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(stage_final_kernel, dim3((nprob + 63) / 64), dim3(64), 0, s, d, nprob);
    return hipGetLastError();
}

// Omega (n x l) of every problem: thread = one (row pair, column) Philox draw.
__global__ __launch_bounds__(256) void omega_kernel(const OmegaDesc* __restrict__ descs,
                                                    const int* __restrict__ blk_begin, int nprob)
{
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(blk_begin, t);
    const int b = wi_.x;
    const OmegaDesc& d = descs[b];
    const int64_t idx = (int64_t)wi_.y * 256 + threadIdx.x;
    const int l = d.l, n = d.n;
    if (d.complex_embed) {
        // entry (i, j) of the complex test matrix -> its 2 x 2 real block
        if (idx >= (int64_t)n * l) return;
        const int i = (int)(idx / l), j = (int)(idx % l);
        double re, im;
        gaussian_complex(d.seed, (uint32_t)i, (uint32_t)j, &re, &im);
        const int64_t ld = 2 * (int64_t)l;
        store_elem(d.Om, d.elem, (int64_t)i * ld + j, re);
        store_elem(d.Om, d.elem, (int64_t)i * ld + l + j, -im);
        store_elem(d.Om, d.elem, (int64_t)(n + i) * ld + j, im);
        store_elem(d.Om, d.elem, (int64_t)(n + i) * ld + l + j, re);
        return;
    }
    const int64_t pairs = (int64_t)((n + 1) / 2) * l;
    if (idx >= pairs) return;
    const int ip = (int)(idx / l), j = (int)(idx % l);
    double g0, g1;
    gaussian_pair(d.seed, (uint32_t)ip, (uint32_t)j, &g0, &g1);
    store_elem(d.Om, d.elem, (int64_t)(2 * ip) * l + j, g0);
    if (2 * ip + 1 < n) store_elem(d.Om, d.elem, (int64_t)(2 * ip + 1) * l + j, g1);
}

hipError_t launch_omega(const OmegaDesc* d, const int* blk_begin, int nprob, int total_blocks,
                        hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(omega_kernel, dim3(total_blocks), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

// At = [[Ar, -Ai], [Ai, Ar]] from the interleaved complex A: thread = one complex entry.
__global__ __launch_bounds__(256) void embed_complex_kernel(const CEmbedDesc* __restrict__ descs,
                                                            const int* __restrict__ blk_begin, int nprob)
{
    const int2 wi_ = wg_item(blk_begin, blockIdx.x);
    const CEmbedDesc& d = descs[wi_.x];
    const int64_t idx = (int64_t)wi_.y * 256 + threadIdx.x;
    const int m = d.m, n = d.n;
    if (idx >= (int64_t)m * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    const GLB double* a = to_glb(d.A) + 2 * ((int64_t)i * d.lda + j);
    const double re = a[0], im = a[1];
    GLB double* t = to_glb(d.At);
    const int64_t ld = d.ldt;
    t[(int64_t)i * ld + j] = re;
    t[(int64_t)i * ld + n + j] = -im;
    t[(int64_t)(m + i) * ld + j] = im;
    t[(int64_t)(m + i) * ld + n + j] = re;
}

hipError_t launch_embed_complex(const CEmbedDesc* d, const int* blk_begin, int nprob, int total_blocks,
                                hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(embed_complex_kernel, dim3(total_blocks), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

// Raw Philox4x32-10 words for count (counter, key) inputs, 6 words each.
__global__ void philox_words_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t* c = in + 6 * i;
    PhiloxWords w = philox4x32_10(c[0], c[1], c[2], c[3], c[4], c[5]);
    for (int t = 0; t < 4; ++t) out[4 * i + t] = w.w[t];
}

hipError_t launch_philox_words(const uint32_t* in, uint32_t* out, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_words_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, in, out,
                       count);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int* p, int value, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

hipError_t launch_fill_i32(int* p, int value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, value,
                       count);
    return hipGetLastError();
}

// Host bytes to device memory through kernel arguments: each launch carries
// one chunk by value, so the copy needs no pinned staging buffer and a
// captured graph keeps the bytes of the call that recorded it.
struct UploadChunk {
    unsigned char bytes[UPLOAD_CHUNK_BYTES];
};

__global__ __launch_bounds__(256) void upload_kernel(unsigned char* dst, UploadChunk c, int nbytes)
{
    for (int i = threadIdx.x; i < nbytes; i += 256) dst[i] = c.bytes[i];
}

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    UploadChunk c;
    for (size_t off = 0; off < bytes; off += UPLOAD_CHUNK_BYTES) {
        const size_t nb = bytes - off < (size_t)UPLOAD_CHUNK_BYTES ? bytes - off : (size_t)UPLOAD_CHUNK_BYTES;
        memcpy(c.bytes, (const unsigned char*)src + off, nb);
        hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, s, (unsigned char*)dst + off, c, (int)nb);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// X = A (m x n) or A^T (n x m) in FP64; 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void copy_f64_kernel(const CopyDesc* __restrict__ descs,
                                                       const int* __restrict__ blk_begin, int nprob)
{
    __shared__ double T[64][65];
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(blk_begin, t);
    const int b = wi_.x;
    const CopyDesc& d = descs[b];
    const int local = wi_.y;
    const int tn = (d.n + 63) / 64;
    const int i0 = (local / tn) * 64, j0 = (local % tn) * 64;
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int i = e / 64, j = e % 64;
        const int gi = i0 + i, gj = j0 + j;
        T[i][j] = (gi < d.m && gj < d.n) ? load_elem(d.A, d.a_elem, (int64_t)gi * d.lda + gj) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        if (!d.transpose) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < d.m && gj < d.n) to_glb(d.X)[(int64_t)gi * d.ldx + gj] = T[r][c];
        } else {
            const int gj = j0 + r, gi = i0 + c;  // X row = column of A
            if (gi < d.m && gj < d.n) to_glb(d.X)[(int64_t)gj * d.ldx + gi] = T[c][r];
        }
    }
}

hipError_t launch_copy_f64(const CopyDesc* d, const int* blk_begin, int nprob, int total_blocks,
                           hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_f64_kernel, dim3(total_blocks), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void eye_kernel(const EyeDesc* __restrict__ descs,
                                                  const int* __restrict__ blk_begin, int nprob)
{
    const int t = blockIdx.x;
    const int2 wi_ = wg_item(blk_begin, t);
    const int b = wi_.x;
    const EyeDesc& d = descs[b];
    const int64_t idx = (int64_t)wi_.y * 256 + threadIdx.x;
    const int64_t R = d.R;
    if (idx >= R * R) return;
    const int64_t i = idx / R, j = idx % R;
    to_glb(d.P)[i * d.ldp + j] = (i == j) ? 1.0 : 0.0;
}

hipError_t launch_eye(const EyeDesc* d, const int* blk_begin, int nprob, int total_blocks, hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(eye_kernel, dim3(total_blocks), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void rowdot_kernel(const RowDotDesc* __restrict__ descs,
                                                     const int* __restrict__ blk_begin, int nprob)
{
    const int2 wi_ = wg_item(blk_begin, blockIdx.x);
    const RowDotDesc& d = descs[wi_.x];
    const int lane = threadIdx.x & 63, i = 4 * wi_.y + (threadIdx.x >> 6);
    if (i >= d.rows) return;
    const GLB double* __restrict__ x = to_glb(d.X) + (int64_t)i * d.ldx;
    const GLB double* __restrict__ y = to_glb(d.Y) + (int64_t)i * d.ldy;
    double acc = 0.0;
    for (int j = lane; j < d.cols; j += 64) acc = fma(x[j], y[j], acc);
    acc = wave_sum(acc);
    if (lane == 0) to_glb(d.out)[i] = d.alpha * acc;
}

hipError_t launch_rowdot(const RowDotDesc* d, const int* blk_begin, int nprob, int total_blocks, hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(rowdot_kernel, dim3(total_blocks), dim3(256), 0, s, d, blk_begin, nprob);
    return hipGetLastError();
}

}  // namespace rsvd
