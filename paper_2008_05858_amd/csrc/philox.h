// Photon-noise streams (Sec. 2.2): Philox-4x32-10 (Salmon, Moraes, Dror,
// Shaw, SC'11) with key = seed and counter = (pixel lo, pixel hi, frame
// index, draw block), and the Poisson sampler drawn from it -- Knuth's
// multiplication method (TAOCP vol. 2, 3.4.1) below a mean of 10, Hormann's
// PTRS transformed rejection (Insurance: Math. & Econ. 12, 1993) above.
// Shared by the noise and detector kernels.
#pragma once

#include "dev_common.h"

namespace e2e {

struct Stream {
    uint32_t k0, k1;
    uint32_t c0, c1, c2, c3;
    uint32_t b0, b1, b2, b3;
    int have;
};

__device__ __forceinline__ void philox10(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
        uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
        uint32_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double to_unit(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ inline double next_u(Stream &s)
{
    if (s.have == 0) {
        uint32_t x0 = s.c0, x1 = s.c1, x2 = s.c2, x3 = s.c3;
        philox10(x0, x1, x2, x3, s.k0, s.k1);
        s.b0 = x0; s.b1 = x1; s.b2 = x2; s.b3 = x3;
        s.c3 += 1u;
        s.have = 2;
    }
    double u = s.have == 2 ? to_unit(s.b0, s.b1) : to_unit(s.b2, s.b3);
    s.have -= 1;
    return u;
}

// log(k!) for integer k >= 0: exact factorials (all below 2^53) up to 15,
// then Stirling's series for log Gamma(z), z = k + 1 >= 16, through the
// z^-9 term (the first omitted term is below 1.2e-16); within a few ulps of
// the exact value.
__device__ __forceinline__ double log_factorial(double k)
{
    if (k < 16.0) {
        double f = 1.0;
        for (double m = 2.0; m <= k; m += 1.0) f *= m;
        return log(f);
    }
    const double z = k + 1.0, r = 1.0 / z, r2 = r * r;
    double t = 1.0 / 1188.0;
    t = fma(t, r2, -1.0 / 1680.0);
    t = fma(t, r2, 1.0 / 1260.0);
    t = fma(t, r2, -1.0 / 360.0);
    t = fma(t, r2, 1.0 / 12.0);
    return (z - 0.5) * log(z) - z + 0.91893853320467274178 + t * r;
}

// Poisson draw of mean `mean` from the stream: multiplication of uniforms
// below 10, the transformed rejection with squeeze of Hormann (1993, PTRS)
// above.  The acceptance test is the one of the method, evaluated as
// log(V alpha^-1 / (a / us^2 + b)) against k log(mean) - mean - log(k!),
// with log(k!) from log_factorial(); decisions differ from a plain lgamma
// evaluation only when the two sides agree to a few ulps.
__device__ inline double poisson(double mean, Stream &st)
{
    if (!(mean > 0.0)) return 0.0;
    if (mean < 10.0) {
        double L = exp(-mean), prod = next_u(st), k = 0.0;
        for (int guard = 0; prod > L && guard < 100000; ++guard) {
            k += 1.0;
            prod *= next_u(st);
        }
        return k;
    }
    double slam = sqrt(mean), loglam = log(mean);
    double b = 0.931 + 2.53 * slam;
    double a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    double vr = 0.9277 - 3.6224 / (b - 2.0);
    double k = floor(mean);
    for (int guard = 0; guard < 100000; ++guard) {
        double U = next_u(st) - 0.5;
        double V = next_u(st);
        double us = 0.5 - fabs(U);
        k = floor((2.0 * a / us + b) * U + mean + 0.43);
        if (us >= 0.07 && V <= vr) return k;
        if (k < 0.0 || (us < 0.013 && V > us)) continue;
        if (log(V * invalpha / (a / (us * us) + b)) <= -mean + k * loglam - log_factorial(k))
            return k;
    }
    return k;
}

__device__ __forceinline__ Stream make_stream(uint64_t seed, uint32_t frame, uint64_t p)
{
    Stream s;
    s.k0 = (uint32_t)seed;
    s.k1 = (uint32_t)(seed >> 32);
    s.c0 = (uint32_t)p;
    s.c1 = (uint32_t)(p >> 32);
    s.c2 = frame;
    s.c3 = 0u;
    s.have = 0;
    return s;
}

// 53-bit uniform pair of draw block `block` of a pixel's stream (a block
// index the Poisson draws of that pixel never reach when >= 2^31).
__device__ __forceinline__ void uniform_pair(uint64_t seed, uint32_t frame, uint64_t p,
                                             uint32_t block, double *u1, double *u2)
{
    uint32_t x0 = (uint32_t)p, x1 = (uint32_t)(p >> 32), x2 = frame, x3 = block;
    philox10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    *u1 = to_unit(x0, x1);
    *u2 = to_unit(x2, x3);
}

}  // namespace e2e
