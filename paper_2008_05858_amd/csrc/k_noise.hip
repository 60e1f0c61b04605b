// Photon noise on the final frame (Sec. 2.2): every pixel's expected count
// becomes a Poisson draw.  Uniforms come from Philox-4x32-10 (Salmon,
// Moraes, Dror, Shaw, SC'11) with key = seed and counter = (pixel lo, pixel
// hi, frame index, draw block), so a pixel's draws depend only on
// (seed, frame, pixel): identical alone or inside any batch.  Means below 10
// use Knuth's multiplication method (TAOCP vol. 2, 3.4.1); larger means use
// Hormann's PTRS transformed rejection (Insurance: Math. & Econ. 12, 1993).
// One thread per pixel; the frame is read and written once (HBM bound).
#include "philox.h"

namespace e2e {

namespace {

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
