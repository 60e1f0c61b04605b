// Pixel integrals of an axis-aligned Gaussian PSF (Sec. 2.1's analytic
// aberration model), shared by the VALU and MFMA separable paths.
#pragma once

#include "dev_common.h"

namespace e2e {

constexpr int kMaxH = 8;

// Per-axis weights of a Gaussian centred at pixel offset d in [-1/2, 1/2)
// from anchor pixel 0: w[m] = (Phi(e_{m+1}) - Phi(e_m)) / norm for pixels
// m - H, with e_m = (m - H - 1/2 - d) / sg.  Each edge uses one erfc of its
// absolute value: c_m = Phi(-|e_m|).
__device__ inline void axis_weights(float d, float sg, int H, float scale, float *w)
{
    const float r = 0.70710678118654752f;
    float inv = 1.0f / sg;
    float cprev = 0.f;
    bool pprev = false;
    float c0 = 0.f, clast = 0.f;
    for (int m = 0; m <= 2 * H + 1; ++m) {
        float e = ((float)(m - H) - 0.5f - d) * inv;
        float c = 0.5f * erfcf(fabsf(e) * r);
        bool pos = e >= 0.0f;
        if (m > 0) {
            float v;
            if (pprev) v = cprev - c;            // both edges right of the centre
            else if (!pos) v = c - cprev;        // both left
            else v = (1.0f - cprev) - c;         // straddles the centre
            w[m - 1] = v;
        } else {
            c0 = c;
        }
        cprev = c;
        pprev = pos;
        clast = c;
    }
    float norm = (1.0f - c0) - clast;
    float f = scale / norm;
    for (int m = 0; m <= 2 * H; ++m) w[m] *= f;
}


// Normal tail Phi(-|z|) = erfc(|z| / sqrt 2) / 2 in FP32, branch free: the
// Chebyshev-fitted form erfc(x) = t exp(-x^2 + P(t)), t = 1 / (1 + x/2)
// (Numerical Recipes, Press et al., 2nd ed., Sec. 6.2; fractional error
// below 1.2e-7 for x >= 0 in exact arithmetic), evaluated in FP32 with the
// hardware reciprocal and base-2 exponential.  About 2e-7 absolute error in
// Phi near z = 0 (P sums terms of order one), against erfcf's few ulp: used
// by the FP32 precision variant only.
__device__ __forceinline__ float phi_tail_f32(float z)
{
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
    float p = 0.17087277f;
    p = fmaf(p, t, -0.82215223f);
    p = fmaf(p, t, 1.48851587f);
    p = fmaf(p, t, -1.13520398f);
    p = fmaf(p, t, 0.27886807f);
    p = fmaf(p, t, -0.18628806f);
    p = fmaf(p, t, 0.09678418f);
    p = fmaf(p, t, 0.37409196f);
    p = fmaf(p, t, 1.00002368f);
    p = fmaf(p, t, -1.26551223f);
    return 0.5f * t * __builtin_amdgcn_exp2f(fmaf(-x, x, p) * 1.4426950408889634f);
}

// Phi(-|z|) in FP32 from two fitted forms (coefficients: least-squares fits
// to the exact function, made by fit_normal_tail.py beside this file):
//   |z| < 1:  1/2 - |z| Q(z^2), Q of degree 5 (the odd series of the CDF);
//   |z| >= 1: exp(-z^2 / 2) S(1 / (1 + 0.35 |z|)), S of degree 9, fitted in
//             relative error up to |z| = 9.
// Absolute error below 1e-7 over the whole range (about one FP32 ulp of
// 1/2, as erfcf), in 24 instructions without branches.
__device__ __forceinline__ float phi_lower_f32(float z)
{
    const float x = fabsf(z);
    const float u = x * x;
    float q = -7.661413292e-06f;
    q = fmaf(q, u, 1.134861668e-04f);
    q = fmaf(q, u, -1.186309266e-03f);
    q = fmaf(q, u, 9.973305278e-03f);
    q = fmaf(q, u, -6.649035215e-02f);
    q = fmaf(q, u, 3.989422917e-01f);
    const float centre = fmaf(-x, q, 0.5f);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.35f, x, 1.0f));
    float p = -3.970254585e-02f;
    p = fmaf(p, t, 1.906433702e-01f);
    p = fmaf(p, t, -3.446725309e-01f);
    p = fmaf(p, t, 2.548686564e-01f);
    p = fmaf(p, t, -8.698244393e-02f);
    p = fmaf(p, t, 1.328877807e-01f);
    p = fmaf(p, t, 1.123037711e-01f);
    p = fmaf(p, t, 1.411426216e-01f);
    p = fmaf(p, t, 1.394989341e-01f);
    p = fmaf(p, t, 5.031029559e-06f);
    // exp(-u / 2) = 2^(-u / (2 ln 2))
    const float tail = __builtin_amdgcn_exp2f(u * -0.7213475204f) * p;
    return x < 1.0f ? centre : tail;
}

// Phi(-|e|): library erfcf, or the FP32 fitted tail when FAST.
template <bool FAST>
__device__ __forceinline__ float normal_tail(float e)
{
    if (FAST) return phi_tail_f32(e);
    return 0.5f * erfcf(fabsf(e) * 0.70710678118654752f);
}

// The same weights, written aligned to a tile edge of TWD pixels: window
// pixel m (0 .. 2H) lands in w16[(off + m) * STRIDE] when off + m is inside
// the tile, every other entry is 0.  The window sum is taken
// from the two outer edges first (through the fitted tail, see below), so
// each weight is stored once, already scaled; the other edges are as in
// axis_weights() (erfcf unless FAST).
template <int TWD = 16, int STRIDE = 1, bool FAST = false>
__device__ inline void axis_weights_tile(float d, float sg, int H, float scale, int off,
                                         float *w16)
{
    float inv = 1.0f / sg;
#pragma unroll
    for (int c = 0; c < TWD; ++c) w16[c * STRIDE] = 0.0f;
    // the window's outer edges lie at |e| >= H / sg, in the far tail, where the
    // fitted tail's relative error (~2e-7) is an absolute error below
    // 2e-7 Phi(-H / sg): it takes them on every path
    const float c0 = phi_tail_f32(((float)(0 - H) - 0.5f - d) * inv);
    const float clast = phi_tail_f32(((float)(2 * H + 1 - H) - 0.5f - d) * inv);
    const float f = scale / ((1.0f - c0) - clast);
    float cprev = c0;
    bool pprev = false;  // the first edge lies left of the centre
    const int m0 = max(1, 1 - off), m1 = min(2 * H + 1, TWD - off);
    if (m0 > 1) {
        const float e = ((float)(m0 - 1 - H) - 0.5f - d) * inv;
        cprev = normal_tail<FAST>(e);
        pprev = e >= 0.0f;
    }
    for (int m = m0; m <= m1; ++m) {
        const float e = ((float)(m - H) - 0.5f - d) * inv;
        const float c = m == 2 * H + 1 ? clast : normal_tail<FAST>(e);
        const bool pos = e >= 0.0f;
        float v;
        if (pprev) v = cprev - c;
        else if (!pos) v = c - cprev;
        else v = (1.0f - cprev) - c;
        w16[(off + m - 1) * STRIDE] = v * f;
        cprev = c;
        pprev = pos;
    }
}

// (sigma_x, sigma_y) of a sample: bilinear in the field over the node grid.
__device__ inline void sigma_at(const float *sxy, int gx, int gy, double gsx, double gsy,
                                double x, double y, float *sx, float *sy)
{
    double fx, fy;
    int cx = node_cell(x, gsx, gx, &fx);
    int cy = node_cell(y, gsy, gy, &fy);
    int cx1 = min(cx + 1, gx - 1), cy1 = min(cy + 1, gy - 1);
    auto S = [&](int l, int m, int c) { return (double)sxy[((size_t)l * gx + m) * 2 + c]; };
    double gx0 = 1.0 - fx, gy0 = 1.0 - fy;
    *sx = (float)(gx0 * gy0 * S(cy, cx, 0) + fx * gy0 * S(cy, cx1, 0) + gx0 * fy * S(cy1, cx, 0) +
                  fx * fy * S(cy1, cx1, 0));
    *sy = (float)(gx0 * gy0 * S(cy, cx, 1) + fx * gy0 * S(cy, cx1, 1) + gx0 * fy * S(cy1, cx, 1) +
                  fx * fy * S(cy1, cx1, 1));
}

}  // namespace e2e
