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
