// Photon noise on the final frame (Sec. 2.2): every pixel's expected count
// becomes a Poisson draw.  Uniforms come from Philox-4x32-10 (Salmon,
// Moraes, Dror, Shaw, SC'11) with key = seed and counter = (pixel lo, pixel
// hi, frame index, draw block), so a pixel's draws depend only on
// (seed, frame, pixel): identical alone or inside any batch.  Means below 10
// use Knuth's multiplication method (TAOCP vol. 2, 3.4.1); larger means use
// Hormann's PTRS transformed rejection (Insurance: Math. & Econ. 12, 1993).
// One thread per pixel; the frame is read and written once (HBM bound).
#include "dev_common.h"

namespace e2e {

namespace {

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

__device__ double next_u(Stream &s)
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

__device__ double poisson(double mean, Stream &st)
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
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <=
            -mean + k * loglam - lgamma(k + 1.0))
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

template <typename T>
__global__ void k_noise(T *frame, int64_t n, uint64_t seed, uint32_t fidx)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        Stream st = make_stream(seed, fidx, (uint64_t)p);
        frame[p] = (T)poisson((double)frame[p], st);
    }
}

__global__ void k_noise_frames(const FrameDev *__restrict__ frames)
{
    const FrameDev &F = frames[blockIdx.y];
    if (!F.poisson) return;
    int64_t n = (int64_t)F.nx * F.ny;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        Stream st = make_stream(F.seed, F.frame_index, (uint64_t)p);
        if (F.out_f64) {
            double *o = (double *)F.out;
            o[p] = poisson(o[p], st);
        } else {
            float *o = (float *)F.out;
            o[p] = (float)poisson((double)o[p], st);
        }
    }
}

__global__ void k_philox(uint64_t seed, uint32_t frame, uint64_t pixel0, int64_t n,
                         uint32_t blocks, uint32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * (int64_t)blocks) return;
    uint64_t p = pixel0 + (uint64_t)(i / blocks);
    uint32_t b = (uint32_t)(i % blocks);
    uint32_t x0 = (uint32_t)p, x1 = (uint32_t)(p >> 32), x2 = frame, x3 = b;
    philox10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[i * 4 + 0] = x0;
    out[i * 4 + 1] = x1;
    out[i * 4 + 2] = x2;
    out[i * 4 + 3] = x3;
}

}  // namespace

hipError_t launch_noise(void *frame, int f64, int64_t n, uint64_t seed, uint32_t frame_index,
                        hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t nb64 = (n + 255) / 256;
    int nb = (int)(nb64 < 65536 ? nb64 : 65536);
    if (f64)
        hipLaunchKernelGGL(k_noise<double>, dim3(nb), dim3(256), 0, s, (double *)frame, n, seed,
                           frame_index);
    else
        hipLaunchKernelGGL(k_noise<float>, dim3(nb), dim3(256), 0, s, (float *)frame, n, seed,
                           frame_index);
    return hipGetLastError();
}

hipError_t launch_noise_frames(const FrameDev *frames_dev, const FrameDev *frames_host,
                               int n_frames, hipStream_t s)
{
    int64_t maxn = 0;
    bool any = false;
    for (int f = 0; f < n_frames; ++f) {
        if (!frames_host[f].poisson) continue;
        any = true;
        int64_t n = (int64_t)frames_host[f].nx * frames_host[f].ny;
        if (n > maxn) maxn = n;
    }
    if (!any) return hipSuccess;
    int64_t nb64 = (maxn + 255) / 256;
    int nb = (int)(nb64 < 8192 ? nb64 : 8192);
    hipLaunchKernelGGL(k_noise_frames, dim3(nb, n_frames), dim3(256), 0, s, frames_dev);
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, uint32_t frame, uint64_t pixel0, int64_t n,
                         uint32_t blocks, uint32_t *out, hipStream_t s)
{
    int64_t tot = n * (int64_t)blocks;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, seed,
                       frame, pixel0, n, blocks, out);
    return hipGetLastError();
}

}  // namespace e2e
