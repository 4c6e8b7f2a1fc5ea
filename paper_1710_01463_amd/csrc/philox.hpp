// Counter-based Gaussian test matrix for the sketch (paper Sec. II.B,
// Alg. RSVD step 1: an n x l matrix of i.i.d. standard normal entries).
//
// Generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11),
// i.e. the 4x32 multiply-xor S-box with multipliers 0xD2511F53 / 0xCD9E8D57
// and key schedule increments 0x9E3779B9 / 0xBB67AE85.
//
// Layout: entry (i, j) of the test matrix of a problem with seed s uses
//   key = (s mod 2^32, s >> 32), counter = (i/2, j, 0, 0).
// The four output words w0..w3 form two 53-bit uniforms
//   u1 = 1 - ((w0:w1) >> 11) 2^-53  in (0, 1],   u2 = ((w2:w3) >> 11) 2^-53,
// and the Box-Muller pair r cos(2 pi u2) (even i), r sin(2 pi u2) (odd i),
// r = sqrt(-2 ln u1).  The entry depends only on (seed, i, j), so any tile can
// regenerate its block and the batch position of a problem does not matter.
#pragma once
#include "common.hpp"

struct PhiloxWords {
    uint32_t w[4];
};

__device__ __forceinline__ PhiloxWords philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                     uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0;
        uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    PhiloxWords out;
    out.w[0] = c0; out.w[1] = c1; out.w[2] = c2; out.w[3] = c3;
    return out;
}

// Both normals of the pair (2*ip, j), (2*ip+1, j).
__device__ __forceinline__ void gaussian_pair(uint64_t seed, uint32_t ip, uint32_t j, double* g_even,
                                              double* g_odd)
{
    PhiloxWords x = philox4x32_10(ip, j, 0u, 0u, (uint32_t)(seed & 0xffffffffu),
                                  (uint32_t)(seed >> 32));
    uint64_t a = ((uint64_t)x.w[0] << 32) | x.w[1];
    uint64_t b = ((uint64_t)x.w[2] << 32) | x.w[3];
    double u1 = 1.0 - (double)(a >> 11) * 0x1.0p-53;
    double u2 = (double)(b >> 11) * 0x1.0p-53;
    double r = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    double sn, cs;
    sincos(ang, &sn, &cs);
    *g_even = r * cs;
    *g_odd = r * sn;
}

// Complex entry (i, j) of the circular Gaussian test matrix of the complex
// path: the Box-Muller pair of counter (i, j, 1, 0) (third word 1, so these
// draws never share a counter with the real ones) as real and imaginary
// parts, each divided by sqrt(2) so that E|w|^2 = 1.
__device__ __forceinline__ void gaussian_complex(uint64_t seed, uint32_t i, uint32_t j, double* re, double* im)
{
    PhiloxWords x = philox4x32_10(i, j, 1u, 0u, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    uint64_t a = ((uint64_t)x.w[0] << 32) | x.w[1];
    uint64_t b = ((uint64_t)x.w[2] << 32) | x.w[3];
    double u1 = 1.0 - (double)(a >> 11) * 0x1.0p-53;
    double u2 = (double)(b >> 11) * 0x1.0p-53;
    double r = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    double sn, cs;
    sincos(ang, &sn, &cs);
    const double s2 = sqrt(2.0);
    *re = r * cs / s2;
    *im = r * sn / s2;
}
