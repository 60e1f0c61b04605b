// Detector stage on the final frame (Sec. 2.2: photon noise plus the
// detector's own effects -- dark current, read-out noise, pixel response
// non-uniformity, cross-talk -- added on the synthetic echellogram).
//
// Pass 1, one thread per pixel: mean electrons mu = G F + dark t (G the
// response map, 1 if absent), then the Poisson draw of the pixel's own
// stream (or mu itself without shot noise), into an FP64 scratch frame.
// Pass 2, 16 x 16 pixel blocks: the 3 x 3 inter-pixel cross-talk gathered
// in a fixed order (charge moving from a pixel to its neighbour at offset
// (dx, dy) with weight K[dy+1][dx+1], charge leaving the chip lost), read
// noise from a Box-Muller pair of the pixel's stream at draw block 2^31,
// then the ADC: floor(R / gain + bias + 1/2) clipped to [0, 2^bits - 1].
// Both passes read and write each pixel once (HBM bound apart from the
// Poisson sampler's arithmetic).
#include "philox.h"

namespace e2e {

namespace {

template <typename T>
__global__ void k_det_electrons(const T *__restrict__ frame, const float *__restrict__ prnu,
                                int64_t n, double dt, int shot, uint64_t seed, uint32_t fidx,
                                double *__restrict__ el)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double g = prnu ? (double)prnu[p] : 1.0;
        const double mu = fma(g, (double)frame[p], dt);
        if (shot) {
            Stream st = make_stream(seed, fidx, (uint64_t)p);
            el[p] = poisson(mu, st);
        } else {
            el[p] = mu;
        }
    }
}

struct DetAdc {
    double k[9];
    double ron, gain, bias, top;
    uint64_t seed;
    uint32_t fidx;
};

__global__ __launch_bounds__(256) void k_det_adc(const double *__restrict__ el, int nx, int ny,
                                                 DetAdc a, uint16_t *__restrict__ adu)
{
    const int gx = blockIdx.x * 16 + (threadIdx.x & 15);
    const int gy = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (gx >= nx || gy >= ny) return;
    double e = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int sx = gx - dx, sy = gy - dy;  // the pixel the charge comes from
            const double v =
                (sx >= 0 && sx < nx && sy >= 0 && sy < ny) ? el[(int64_t)sy * nx + sx] : 0.0;
            e = fma(a.k[(dy + 1) * 3 + (dx + 1)], v, e);
        }
    const int64_t p = (int64_t)gy * nx + gx;
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

}  // namespace

hipError_t launch_det_electrons(const void *frame, int f64, const float *prnu, int64_t n,
                               double dt, int shot, uint64_t seed, uint32_t fidx, double *el,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t nb64 = (n + 255) / 256;
    int nb = (int)(nb64 < 65536 ? nb64 : 65536);
    if (f64)
        hipLaunchKernelGGL(k_det_electrons<double>, dim3(nb), dim3(256), 0, s,
                           (const double *)frame, prnu, n, dt, shot, seed, fidx, el);
    else
        hipLaunchKernelGGL(k_det_electrons<float>, dim3(nb), dim3(256), 0, s,
                           (const float *)frame, prnu, n, dt, shot, seed, fidx, el);
    return hipGetLastError();
}

hipError_t launch_det_adc(const double *el, int nx, int ny, const double *xtalk, double ron,
                          double gain, double bias, int bits, uint64_t seed, uint32_t fidx,
                          uint16_t *adu, hipStream_t s)
{
    if ((int64_t)nx * ny <= 0) return hipSuccess;
    DetAdc a;
    for (int q = 0; q < 9; ++q) a.k[q] = xtalk[q];
    a.ron = ron;
    a.gain = gain;
    a.bias = bias;
    a.top = (double)((1u << bits) - 1u);
    a.seed = seed;
    a.fidx = fidx;
    hipLaunchKernelGGL(k_det_adc, dim3((nx + 15) / 16, (ny + 15) / 16), dim3(256), 0, s, el, nx,
                       ny, a, adu);
    return hipGetLastError();
}

}  // namespace e2e
