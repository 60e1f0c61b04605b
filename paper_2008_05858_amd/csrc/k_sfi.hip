// Explicit spectral-fiber-image render path (Sec. 2.2: every SFI is the
// surface integral of the fiber's spatial profile convolved with the PSF,
// computed on a sub-pixel grid; Sec. 2.1's axis-aligned Gaussian as the
// PSF, with (sigma_x, sigma_y) interpolated across the field).
//
// The fiber image is a uniform disc of radius rho (or one half of it) on
// the sample position.  Its convolution with the Gaussian at offset (u, v)
// is, with the disc parametrised by the chord angle th (a = rho sin th,
// chord b in [-h, h], h = rho cos th, or [0, h] / [-h, 0] for a half),
//   C(u, v) ~ int cos(th) N(u - a) [Phi((v - lo)/sy) - Phi((v - hi)/sy)] dth,
// taken with Gauss-Legendre points th_p (chosen at load so the rule agrees
// with the converged integral to rounding).  Each point is separable in
// (u, v), so the sub-pixel mean of C over pixel (i, j) is
//   W(i, j) ~ sum_p X_p[i] Y_p[j],
//   X_p[i] = w_p cos th_p sum_s [N(u_is - a_p) + N(u_is + a_p)]  (th, -th pair)
//   Y_p[j] = sum_t [Phi((v_jt - lo_p)/sy) - Phi((v_jt - hi_p)/sy)]
// over the S sub-pixel centres u_is, v_jt of the pixel, and the window sum
// is sum_p (sum_i X_p[i]) (sum_j Y_p[j]), which renormalises the weights
// (constant factors cancel).  So one sample costs R (N S) Gaussians per
// side of a pair and 2 R N S normal CDFs, then a rank-R product per pixel,
// instead of the N^2 S^2 quadratures of the direct form.
//
// One workgroup owns a 64 x 32 tile (wide along the dispersion, so fewer
// tiles share a sample: a window meets 1.5 tiles on average against 2.6
// with 16 x 16).  Per chunk of 16 samples: positions in
// FP64 (one thread per sample); the X_p row of every (sample, point) and
// the Y_p entry of every (sample, point, pixel row) by one thread each
// (FP32 Gaussians and normal tails on pixel-relative offsets, each CDF
// difference taken on the side where nothing cancels); each sample's scale
// photons / window sum; then every
// thread adds its 8 pixels' rank-R products times the scale, in sample
// order, into FP64 sums.  Deterministic; each pixel written once.
#include "psf_gauss.h"

namespace e2e {

namespace {

constexpr int CH = 16;                   // samples per chunk
constexpr int PB = 64;                   // samples positioned together
constexpr int NW = 2 * kSfiMaxH + 1;     // window edge, max

// Normal tail Phi(-|z|) = erfc(|z| / sqrt 2) / 2, branch free: the
// Chebyshev-fitted form erfc(x) = t exp(-x^2 + P(t)), t = 1 / (1 + x/2),
// of Numerical Recipes (Press et al., 2nd ed., Sec. 6.2; fractional error
// below 1.2e-7 for all x >= 0), with t and P in FP64 (P sums terms of order
// one that cancel near x = 0) and the exponential in FP32.  A whole wave
// runs one instruction stream whatever mix of arguments its lanes hold.
__device__ __forceinline__ float phi_tail(float z)
{
    const double x = (double)fabsf(z) * 0.70710678118654752;
    // 1 / d for d in [1, 9]: hardware reciprocal refined by one Newton step
    const double d = fma(0.5, x, 1.0);
    const double r0 = __builtin_amdgcn_rcp(d);
    const double t = fma(r0, fma(-d, r0, 1.0), r0);
    double p = 0.17087277;
    p = fma(p, t, -0.82215223);
    p = fma(p, t, 1.48851587);
    p = fma(p, t, -1.13520398);
    p = fma(p, t, 0.27886807);
    p = fma(p, t, -0.18628806);
    p = fma(p, t, 0.09678418);
    p = fma(p, t, 0.37409196);
    p = fma(p, t, 1.00002368);
    p = fma(p, t, -1.26551223);
    const float l2 = (float)(fma(-x, x, p) * 1.4426950408889634);
    return 0.5f * (float)t * __builtin_amdgcn_exp2f(l2);
}

// exp(-e^2 / 2) through the hardware base-2 exponential.
__device__ __forceinline__ float gauss(float e)
{
    return __builtin_amdgcn_exp2f(-0.72134752044448170f * e * e);
}

// Phi(z1) - Phi(z2), z1 >= z2, from the tails (no cancellation of values
// near 1).
__device__ __forceinline__ float cdf_diff(float z1, float z2)
{
    const float c1 = phi_tail(z1), c2 = phi_tail(z2);
    if (z2 >= 0.0f) return c2 - c1;
    if (z1 <= 0.0f) return c1 - c2;
    return (1.0f - c1) - c2;
}

template <int DX, int DY, typename ST>
__global__ __launch_bounds__(256) void k_render_sfi(const FrameDev *__restrict__ frames,
                                                    const int2 *__restrict__ work, int n_work,
                                                    int *__restrict__ counter,
                                                    int *__restrict__ err)
{
    constexpr int TW = kSfiTW, TH = kSfiTH;
    __shared__ float sX[CH][kSfiMaxR][NW + 1], sY[CH][kSfiMaxR][NW + 1];
    __shared__ float sSX[CH][kSfiMaxR];
    __shared__ double sprod[CH][kSfiMaxR];
    __shared__ float sdx[PB], sdy[PB], ssx[PB], ssy[PB], sphi[PB];
    __shared__ double sscale[PB];
    __shared__ int sax[PB], say[PB];
    __shared__ int tlist[kMaxTileTraces];
    __shared__ int sh_count, sh_item;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    for (int iter = 0;; ++iter) {
        int fi, tile_id;
        if (work == nullptr) {
            if (iter > 0) break;
            fi = 0;
            tile_id = xcd_remap(blockIdx.x, gridDim.x);
        } else {
            if (tid == 0) sh_item = atomicAdd(counter, 1);
            __syncthreads();
            int w = uniform_i(sh_item);
            if (w >= n_work) break;
            int2 wk = work[w];
            fi = uniform_i(wk.x);
            tile_id = uniform_i(wk.y);
        }
        const FrameDev &F = frames[fi];
        const int ntr = F.ntr, H = F.H, N = 2 * F.H + 1;
        const int R = F.sfi_R, S = F.sfi_S, shape = F.sfi_shape;
        const float invS = 1.0f / (float)S;
        const int tx = tile_id % F.ntx, ty = tile_id / F.ntx;
        const int X0 = tx * TW, Y0 = ty * TH;
        const SegDev *segs = F.segs + (size_t)tx * ntr;
        if (tid < 64) {
            int cnt = 0;
            for (int base = 0; base < ntr; base += 64) {
                int tr = base + lane;
                bool ok = false;
                if (tr < ntr) {
                    SegDev s = segs[tr];
                    ok = s.k0 < s.k1 && s.ty0 <= ty && ty <= s.ty1;
                }
                unsigned long long m = __ballot(ok);
                int pos = cnt + __popcll(m & ((1ull << lane) - 1ull));
                if (ok) {
                    if (pos < kMaxTileTraces) tlist[pos] = tr;
                    else atomicOr(err, kErrTileTraces);
                }
                cnt += __popcll(m);
            }
            if (lane == 0) sh_count = min(cnt, kMaxTileTraces);
        }
        __syncthreads();
        const int count = uniform_i(sh_count);
        // this thread's pixels: column pi, rows pj .. pj+7 (a wave covers 16
        // columns x 32 rows, so a window touches one or two waves)
        const int pi = X0 + 16 * (tid >> 6) + (lane & 15), pj = Y0 + 8 * (lane >> 4);
        double acc[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r] = 0.0;

        for (int li = 0; li < count; ++li) {
            const int tr = uniform_i(tlist[li]);
            const TraceDev &T = F.tr[tr];
            const SegDev sg = segs[tr];
            double cxr[DX + 1], cyr[DY + 1];
#pragma unroll
            for (int j = 0; j <= DX; ++j) cxr[j] = T.cx[j];
#pragma unroll
            for (int j = 0; j <= DY; ++j) cyr[j] = T.cy[j];
            double t0, dt;
            trace_affine(T, F.beta, &t0, &dt);
            const float scale = (float)(T.thr * F.flux_scale);
            const ST *spec = (const ST *)F.spec[T.slot];
            for (int kb = sg.k0; kb < sg.k1; kb += PB) {
                const int nb = min(PB, sg.k1 - kb);
                // 1. positions, anchors, sigmas, photons of up to 64 samples
                if (tid < nb) {
                    const int k = kb + tid;
                    const double t = fma((double)k, dt, t0);
                    const double x = horner<DX>(cxr, t);
                    const double y = horner<DY>(cyr, t);
                    const double axd = floor(x + 0.5), ayd = floor(y + 0.5);
                    float sgx, sgy;
                    sigma_at(F.sxy, F.gx, F.gy, F.gsx, F.gsy, x, y, &sgx, &sgy);
                    sdx[tid] = (float)(x - axd);
                    sdy[tid] = (float)(y - ayd);
                    ssx[tid] = sgx;
                    ssy[tid] = sgy;
                    sphi[tid] = (float)spec_at(spec, k) * scale;
                    sax[tid] = (int)axd - H;
                    say[tid] = (int)ayd - H;
                }
                __syncthreads();
                for (int c0 = 0; c0 < nb; c0 += CH) {
                    const int nk = min(CH, nb - c0);
                    // 2. X_p rows (one (sample, point) per task) and Y_p
                    //    entries (one (sample, point, pixel row) per task: the
                    //    normal tails are the costly part, so they are spread
                    //    finest); s indexes the chunk, c0 + s the block
                    const int nX = nk * R, nT = nX + nk * R * N;
                    for (int q = tid; q < nT; q += 256) {
                        if (q < nX) {
                            const int s = q / R, p = q % R;
                            const float a = F.sfq[3 * p], wp = F.sfq[3 * p + 2];
                            const float inv = 1.0f / ssx[c0 + s], d = sdx[c0 + s];
                            float tot = 0.0f;
                            for (int i = 0; i < N; ++i) {
                                float g = 0.0f;
                                for (int t = 0; t < S; ++t) {
                                    const float u =
                                        (float)(i - H) - 0.5f + ((float)t + 0.5f) * invS - d;
                                    g += gauss((u - a) * inv) + gauss((u + a) * inv);
                                }
                                g *= wp;
                                sX[s][p][i] = g;
                                tot += g;
                            }
                            sSX[s][p] = tot;
                        } else {
                            const int e = q - nX, s = e / (R * N), rem = e % (R * N);
                            const int p = rem / N, j = rem % N;
                            const float h = F.sfq[3 * p + 1];
                            const float inv = 1.0f / ssy[c0 + s];
                            const float lo = shape == E2E_FIBER_HALF_UP ? 0.0f : -h;
                            const float hi = shape == E2E_FIBER_HALF_DOWN ? 0.0f : h;
                            const float v0 = (float)(j - H) - 0.5f - sdy[c0 + s];
                            float g0 = 0.0f, g1 = 0.0f;
                            int t = 0;
                            for (; t + 1 < S; t += 2) {   // two sub-rows: four independent tails
                                const float va = v0 + ((float)t + 0.5f) * invS;
                                const float vb = v0 + ((float)t + 1.5f) * invS;
                                g0 += cdf_diff((va - lo) * inv, (va - hi) * inv);
                                g1 += cdf_diff((vb - lo) * inv, (vb - hi) * inv);
                            }
                            if (t < S) {
                                const float va = v0 + ((float)t + 0.5f) * invS;
                                g0 += cdf_diff((va - lo) * inv, (va - hi) * inv);
                            }
                            sY[s][p][j] = g0 + g1;
                        }
                    }
                    __syncthreads();
                    // 3. scale of each sample: photons over its window sum
                    //    sum_p (sum_i X_p[i]) (sum_j Y_p[j]), one (sample, point)
                    //    per thread, then the sums over the points in order
                    if (tid < nX) {
                        const int s = tid / R, p = tid % R;
                        float sy = 0.0f;
                        for (int j = 0; j < N; ++j) sy += sY[s][p][j];
                        sprod[s][p] = (double)sSX[s][p] * (double)sy;
                    }
                    __syncthreads();
                    if (tid < nk) {
                        double z = 0.0;
                        for (int p = 0; p < R; ++p) z += sprod[tid][p];
                        sscale[c0 + tid] = (double)sphi[c0 + tid] / z;
                    }
                    __syncthreads();
                    // 4. this thread's pixels, samples in order
                    for (int s = 0; s < nk; ++s) {
                        const int di = pi - sax[c0 + s], dj0 = pj - say[c0 + s];
                        if ((unsigned)di < (unsigned)N && dj0 > -8 && dj0 < N) {
                            const double sc = sscale[c0 + s];
#pragma unroll
                            for (int r = 0; r < 8; ++r) {
                                const int dj = dj0 + r;
                                if ((unsigned)dj < (unsigned)N) {
                                    float v = 0.0f;
                                    for (int p = 0; p < R; ++p)
                                        v = fmaf(sX[s][p][di], sY[s][p][dj], v);
                                    acc[r] = fma((double)v, sc, acc[r]);
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (pi < F.nx && pj + r < F.ny) {
                const size_t o = (size_t)(pj + r) * F.nx + pi;
                if (F.out_f64) ((double *)F.out)[o] = acc[r];
                else ((float *)F.out)[o] = (float)acc[r];
            }
        }
        __syncthreads();
    }
}

template <int DX, int DY>
hipError_t launch_deg(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                      int n_work, int *counter, int *err, int nb, hipStream_t s)
{
    if (cfg.spec_f64)
        hipLaunchKernelGGL((k_render_sfi<DX, DY, double>), dim3(nb), dim3(256), 0, s,
                           frames_dev, work, n_work, counter, err);
    else
        hipLaunchKernelGGL((k_render_sfi<DX, DY, float>), dim3(nb), dim3(256), 0, s,
                           frames_dev, work, n_work, counter, err);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sfi(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                      int n_work, int *counter, int *err, hipStream_t s)
{
    int nb = work == nullptr ? cfg.plain_tiles : (n_work < 1024 ? n_work : 1024);
    if (nb <= 0) return hipSuccess;
    if (cfg.degx <= 3 && cfg.degy <= 2)
        return launch_deg<3, 2>(frames_dev, cfg, work, n_work, counter, err, nb, s);
    if (cfg.degx <= 4 && cfg.degy <= 3)
        return launch_deg<4, 3>(frames_dev, cfg, work, n_work, counter, err, nb, s);
    return launch_deg<7, 7>(frames_dev, cfg, work, n_work, counter, err, nb, s);
}

}  // namespace e2e
