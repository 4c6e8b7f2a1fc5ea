// Shared device-side definitions for librsvd (gfx950 / CDNA4 only).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

#define RSVD_WAVE 64

// Pointers read from descriptor tables are generic; casting them to the global
// address space lets the compiler emit global_load/store instead of flat
// accesses (which share the LDS wait counter and serialise with LDS traffic).
#define GLB __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GLB T* to_glb(T* p) { return (GLB T*)p; }
template <typename T> __device__ __forceinline__ const GLB T* to_glb(const T* p) { return (const GLB T*)p; }

// Element storage kinds used by kernel templates.
enum ElemKind : int { EK_F64 = 0, EK_F32 = 1, EK_BF16 = 2 };

template <int K> struct ElemT;
template <> struct ElemT<EK_F64> { typedef double type; };
template <> struct ElemT<EK_F32> { typedef float type; };
template <> struct ElemT<EK_BF16> { typedef __bf16 type; };

__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(float x) { return (double)x; }
__device__ __forceinline__ double to_f64(__bf16 x) { return (double)(float)x; }
__device__ __forceinline__ float to_f32(double x) { return (float)x; }
__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(__bf16 x) { return (float)x; }

template <typename T> __device__ __forceinline__ T from_f64(double x);
template <> __device__ __forceinline__ double from_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_f64<float>(double x) { return (float)x; }
// double -> bf16, round to nearest even in one step: first round toward zero
// to float and mark inexactness in the float's last bit (round-to-odd keeps
// the sticky information), then round that float to bf16 to nearest even.
template <> __device__ __forceinline__ __bf16 from_f64<__bf16>(double x)
{
    float t = __double2float_rz(x);
    uint32_t fb = __float_as_uint(t);
    if ((fb & 0x7f800000u) == 0x7f800000u) return (__bf16)(float)x;  // inf / nan
    if ((double)t != x) fb |= 1u;
    uint32_t lsb = (fb >> 16) & 1u;
    uint32_t rounded = fb + 0x7fffu + lsb;
    unsigned short hi = (unsigned short)(rounded >> 16);
    return __builtin_bit_cast(__bf16, hi);
}
template <typename T> __device__ __forceinline__ T from_f32(float x);
template <> __device__ __forceinline__ double from_f32<double>(float x) { return (double)x; }
template <> __device__ __forceinline__ float from_f32<float>(float x) { return x; }
template <> __device__ __forceinline__ __bf16 from_f32<__bf16>(float x)
{
    uint32_t fb = __float_as_uint(x);
    if ((fb & 0x7f800000u) == 0x7f800000u) return (__bf16)x;
    uint32_t lsb = (fb >> 16) & 1u;
    uint32_t rounded = fb + 0x7fffu + lsb;
    unsigned short hi = (unsigned short)(rounded >> 16);
    return __builtin_bit_cast(__bf16, hi);
}

// p[idx] if ok, else 0, as an unconditional load from a clamped address: no
// branch around the load, so that a group of such loads is issued back to
// back and waited for once (a load under a branch ends the branch with a wait).
template <typename T> __device__ __forceinline__ T ld_or0(const GLB T* p, int64_t idx, bool ok)
{
    const T v = p[ok ? idx : 0];
    return ok ? v : (T)0;
}

// Store written through this XCD's L2 (an agent-scope relaxed store): the
// line is not left dirty in L2, where the end-of-kernel write-back, which the
// next kernel waits for, would have to flush it.  Used for the rows the
// Jacobi rounds rotate (measured: the other large outputs gain nothing).
template <typename T> __device__ __forceinline__ void st_through(GLB T* p, T v)
{
    if constexpr (sizeof(T) == 8 || sizeof(T) == 4)
        __hip_atomic_store((T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// Wave-level reductions (64 lanes) with shuffles.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Work-item map of a batched launch: workgroup t serves problem map[t].x,
// local item map[t].y (one load instead of a search over prefix sums, which
// would put several dependent global loads at the start of every workgroup).
__device__ __forceinline__ int2 wg_item(const int* __restrict__ map, int t)
{
    const GLB int* m = to_glb(map) + 2 * (int64_t)t;
    return make_int2(m[0], m[1]);
}
