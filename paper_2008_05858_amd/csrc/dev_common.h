// Device helpers shared by the render kernels: the wavelength -> t map and
// the spectral-format polynomials (FP64), spectrum loads, small wave
// utilities.
#pragma once

#include <hip/hip_runtime.h>

#include "e2e_impl.h"

namespace e2e {

// Address-space views: constant (scalar loads of wave-uniform data through
// the scalar cache) and global (vector loads without the flat path).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)p; }
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) { return (gptr<T>)p; }

// Sample k of a trace sits at lambda_k = lmin + (k + 1/2) dl, dl = span / n,
// and is seen at lambda_k (1 + beta).  Its normalised wavelength
//   t = (2 lambda_k (1 + beta) - lmin - lmax) / span
// is affine in k: t = t0 + k dt.
__device__ __host__ inline void trace_affine(const TraceDev &T, double beta, double *t0,
                                             double *dt)
{
    double span = T.lmax - T.lmin;
    double dl = span / (double)T.n;
    double g = 1.0 + beta;
    *t0 = (2.0 * (T.lmin + 0.5 * dl) * g - T.lmin - T.lmax) / span;
    *dt = 2.0 * dl * g / span;
}

// Horner evaluation of sum_j c[j] t^j with coefficients padded by zeros up
// to degree D (a zero leading coefficient leaves the value bit-identical).
template <int D>
__device__ __forceinline__ double horner(const double *c, double t)
{
    double v = c[D];
#pragma unroll
    for (int j = D - 1; j >= 0; --j) v = fma(v, t, c[j]);
    return v;
}

template <int D>
__device__ __forceinline__ double horner_d(const double *c, double t, double *dv)
{
    double v = c[D], d = 0.0;
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
        d = fma(d, t, v);
        v = fma(v, t, c[j]);
    }
    *dv = d;
    return v;
}

template <typename ST>
__device__ __forceinline__ double spec_at(const ST *p, int k) { return (double)p[k]; }
template <typename ST>
__device__ __forceinline__ double spec_at(gptr<ST> p, int k) { return (double)p[k]; }

// Bilinear node fraction along one axis: node m at m (n-1)/(g-1); returns
// the lower node index (<= g-2) and the fraction towards the next node,
// clamped at the detector edges.  g == 1: one node, fraction 0.
__device__ __forceinline__ int node_cell(double p, double gs, int g, double *f)
{
    if (g < 2) { *f = 0.0; return 0; }
    double sp = fmin(fmax(p * gs, 0.0), (double)(g - 1));
    double c = floor(sp);
    int ci = (int)c;
    if (ci > g - 2) ci = g - 2;
    *f = sp - (double)ci;
    return ci;
}

// Fraction towards node c+1 of position p on a g-node axis, and whether p
// falls in node cell c (the same cell node_cell() would pick).
__device__ __forceinline__ double node_frac_in(double p, double gs, int g, int c, bool *in)
{
    if (g < 2) { *in = true; return 0.0; }
    double sp = fmin(fmax(p * gs, 0.0), (double)(g - 1));
    double f = sp - (double)c;
    *in = (f >= 0.0) && (f < 1.0 || c == g - 2);
    return f;
}

// Extended node cell of position p on a g-node axis: -1 left of node 0 (the
// clamped edge region, fraction 0), g-1 right of the last node (fraction 1),
// otherwise floor(p (g-1)/(n-1)).  Within one extended cell the fraction
// towards the next node is affine in p (or constant), which is what lets a
// column's samples be summed as moments.  g == 1: always cell 0, fraction 0.
__device__ __host__ inline int ext_cell(double p, double gs, int g)
{
    if (g < 2) return 0;
    double v = floor(p * gs);
    if (v < 0.0) return -1;
    if (v > (double)(g - 1)) return g - 1;
    return (int)v;
}

// Node-weight line of an extended cell: fraction towards node base+1 is
// a0 + a1 * p, with the lower node index in *base.
__device__ __host__ inline void cell_line(int c, double gs, int g, int *base, double *a0,
                                          double *a1)
{
    if (g < 2) { *base = 0; *a0 = 0.0; *a1 = 0.0; return; }
    if (c < 0) { *base = 0; *a0 = 0.0; *a1 = 0.0; return; }
    if (c >= g - 1) { *base = g - 2; *a0 = 1.0; *a1 = 0.0; return; }
    *base = c; *a0 = -(double)c; *a1 = gs;
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double uniform_d(double v)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const void *p)
{
    const unsigned long long b = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffull));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return (const T *)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ int floordiv(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

}  // namespace e2e
