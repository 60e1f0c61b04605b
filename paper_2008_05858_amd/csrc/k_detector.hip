// Detector stage on the final frame (Sec. 2.2: photon noise plus the
// detector's own effects -- dark current, read-out noise, pixel response
// non-uniformity, cross-talk -- added on the synthetic echellogram).
//
// One kernel, one 64 x 64 pixel tile per workgroup:
//  1. electrons of the tile and its one-pixel border into LDS: the mean
//     mu = G F + dark t (G the response map, 1 if absent), then the Poisson
//     draw of the pixel's own counter stream (or mu itself without shot
//     noise); border pixels are recomputed by each neighbouring tile (the
//     draw is a pure function of the pixel, so every copy is the same);
//  2. per output pixel: the 3 x 3 inter-pixel cross-talk gathered in a
//     fixed order (charge moving from a pixel to its neighbour at offset
//     (dx, dy) with weight K[dy+1][dx+1], charge leaving the chip lost),
//     read noise from a Box-Muller pair of the pixel's stream at draw block
//     2^31, then the ADC: floor(R / gain + bias + 1/2) clipped to
//     [0, 2^bits - 1], stored as uint16.
// HBM traffic is the frame and gain map read once plus the ADU written once
// (10 bytes per pixel with an FP32 frame); with shot noise the Poisson
// sampler's FP64 arithmetic sets the pace.
#include "philox.h"

namespace e2e {

namespace {

constexpr int DT = 64;          // tile edge
constexpr int DH = DT + 2;      // with its border
constexpr int DN = DH * DH;     // electrons held in LDS per tile

struct DetArgs {
    double k[9];
    double dark, ron, gain, bias, top;
    uint64_t seed;
    uint32_t fidx;
    int nx, ny;
};

template <typename T, bool SHOT>
__global__ __launch_bounds__(256) void k_detector(const T *__restrict__ frame,
                                                  const float *__restrict__ prnu, DetArgs a,
                                                  uint16_t *__restrict__ adu)
{
    __shared__ double el[DN];
    const int x0 = blockIdx.x * DT - 1, y0 = blockIdx.y * DT - 1;
    for (int c = threadIdx.x; c < DN; c += 256) {
        const int gy = y0 + c / DH, gx = x0 + c % DH;
        double v = 0.0;
        if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny) {
            const int64_t p = (int64_t)gy * a.nx + gx;
            const double g = prnu ? (double)prnu[p] : 1.0;
            const double mu = fma(g, (double)frame[p], a.dark);
            if (SHOT) {
                Stream st = make_stream(a.seed, a.fidx, (uint64_t)p);
                v = poisson(mu, st);
            } else {
                v = mu;
            }
        }
        el[c] = v;
    }
    __syncthreads();
    const int lx = threadIdx.x & 63, gx = x0 + 1 + lx;
    if (gx >= a.nx) return;
    for (int ly = threadIdx.x >> 6; ly < DT; ly += 4) {
        const int gy = y0 + 1 + ly;
        if (gy >= a.ny) break;
        double e = 0.0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)  // the pixel the charge comes from
                e = fma(a.k[(dy + 1) * 3 + (dx + 1)], el[(ly + 1 - dy) * DH + (lx + 1 - dx)], e);
        const int64_t p = (int64_t)gy * a.nx + gx;
        double r = e;
        if (a.ron > 0.0) {
            double u1, u2;
            uniform_pair(a.seed, a.fidx, (uint64_t)p, 0x80000000u, &u1, &u2);
            const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            r = fma(a.ron, z, e);
        }
        double v = floor(r / a.gain + a.bias + 0.5);
        v = fmin(fmax(v, 0.0), a.top);
        adu[p] = (uint16_t)v;
    }
}

template <typename T>
void launch_t(const T *frame, const float *prnu, const DetArgs &a, int shot, uint16_t *adu,
              hipStream_t s)
{
    const dim3 grid((a.nx + DT - 1) / DT, (a.ny + DT - 1) / DT);
    if (shot)
        hipLaunchKernelGGL((k_detector<T, true>), grid, dim3(256), 0, s, frame, prnu, a, adu);
    else
        hipLaunchKernelGGL((k_detector<T, false>), grid, dim3(256), 0, s, frame, prnu, a, adu);
}

}  // namespace

hipError_t launch_detector(const void *frame, int f64, const float *prnu, int nx, int ny,
                           double dark, int shot, const double *xtalk, double ron, double gain,
                           double bias, int bits, uint64_t seed, uint32_t fidx, uint16_t *adu,
                           hipStream_t s)
{
    if (nx <= 0 || ny <= 0) return hipSuccess;
    if ((ny + DT - 1) / DT > 65535) return hipErrorInvalidValue;
    DetArgs a;
    for (int q = 0; q < 9; ++q) a.k[q] = xtalk[q];
    a.dark = dark;
    a.ron = ron;
    a.gain = gain;
    a.bias = bias;
    a.top = (double)((1u << bits) - 1u);
    a.seed = seed;
    a.fidx = fidx;
    a.nx = nx;
    a.ny = ny;
    if (f64)
        launch_t((const double *)frame, prnu, a, shot, adu, s);
    else
        launch_t((const float *)frame, prnu, a, shot, adu, s);
    return hipGetLastError();
}

}  // namespace e2e
