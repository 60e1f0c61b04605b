// Separable-PSF render path on the matrix cores (Sec. 2.1's axis-aligned
// Gaussian aberration model with field-dependent (sigma_x, sigma_y)).
//
// With a separable PSF the samples reaching a TY x TX tile contribute
//   F[j][i] = sum_k gy_k[j] phi_k gx_k[i],   i.e.  F = Gy diag(phi) Gx^T,
// a dense contraction over the samples, which is what MFMA computes.  Per
// 32-sample slice a wave builds the A (TY x 32) and B (32 x TX) fragments
// from the per-axis pixel integrals staged in LDS and issues
// v_mfma_f32_16x16x32_{f16,bf16}.  Each operand is split into hi + lo
// halves (hi = round(v), lo = round(v - hi)) and the product is
// hi*hi + hi*lo + lo*hi with FP32 accumulation; phi is scaled per slice by
// an exact power of two so every operand lies in [0, 1].  The four waves
// own disjoint sample slices and their FP32 partial tiles are summed in a
// fixed order, so the result is deterministic.
#include "psf_gauss.h"

namespace e2e {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TX = kMfmaTW;   // 64 columns = 4 blocks of 16
constexpr int TY = kMfmaTH;   // 32 rows = 2 blocks of 16
constexpr int CH = 128;       // samples per chunk: 4 waves x 32

template <bool BF16>
struct Op;
template <>
struct Op<false> {
    using V = h8;
    using E = _Float16;
    __device__ static E hi(float v) { return (E)v; }
    __device__ static f4 mfma(const V &a, const V &b, const f4 &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Op<true> {
    using V = b8;
    using E = __bf16;
    __device__ static E hi(float v) { return (E)v; }
    __device__ static f4 mfma(const V &a, const V &b, const f4 &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <int DX, int DY, typename ST, bool BF16>
__global__ __launch_bounds__(256) void k_render_sep_mfma(const FrameDev *__restrict__ frames,
                                                         const int2 *__restrict__ work,
                                                         int n_work, int *__restrict__ counter,
                                                         int *__restrict__ err)
{
    using O = Op<BF16>;
    using V = typename O::V;
    constexpr int WMAX = 2 * kMaxH + 1;
    __shared__ float swx[CH][WMAX + 1], swy[CH][WMAX + 1];
    __shared__ int sax[CH], say[CH];
    __shared__ float sphi[CH];
    __shared__ float red[4][8][4][64];
    __shared__ int tlist[kMaxTileTraces];
    __shared__ int sh_count, sh_item;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, lg = lane >> 4;

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
        const int ntr = F.ntr, H = F.H;
        const int tx = tile_id % F.ntx, ty = tile_id / F.ntx;
        const int X0 = tx * TX, Y0 = ty * TY;
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
        f4 acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

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
            for (int kc = sg.k0; kc < sg.k1; kc += CH) {
                const int nk = min(CH, sg.k1 - kc);
                // per-axis pixel integrals: thread (sample s, axis)
                {
                    const int s = tid & (CH - 1), axis = tid >> 7;
                    if (s < nk) {
                        const int k = kc + s;
                        double t = fma((double)k, dt, t0);
                        double x = horner<DX>(cxr, t);
                        double y = horner<DY>(cyr, t);
                        float sgx = (float)F.sigma, sgy = (float)F.sigma;
                        if (F.psf_kind == E2E_PSF_SEPARABLE)
                            sigma_at(F.sxy, F.gx, F.gy, F.gsx, F.gsy, x, y, &sgx, &sgy);
                        if (axis == 0) {
                            double axd = floor(x + 0.5);
                            axis_weights((float)(x - axd), sgx, H, 1.0f, swx[s]);
                            sax[s] = (int)axd - H;
                            sphi[s] = (float)spec_at(spec, k) * scale;
                        } else {
                            double ayd = floor(y + 0.5);
                            axis_weights((float)(y - ayd), sgy, H, 1.0f, swy[s]);
                            say[s] = (int)ayd - H;
                        }
                    } else if (axis == 0) {
                        sax[s] = -(1 << 28);
                        sphi[s] = 0.0f;
                    } else {
                        say[s] = -(1 << 28);
                    }
                }
                __syncthreads();
                // this wave's 32-sample slice: lane holds k = 8 (lane / 16) + e
                const int sb = 32 * wv + 8 * lg;
                float pmax = 0.0f;
#pragma unroll
                for (int e = 0; e < 8; ++e) pmax = fmaxf(pmax, sphi[sb + e]);
                pmax = fmaxf(pmax, __shfl_xor(pmax, 16));
                pmax = fmaxf(pmax, __shfl_xor(pmax, 32));
                pmax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(pmax)));
                if (pmax > 0.0f) {
                    int ex;
                    frexpf(pmax, &ex);
                    const float sc = ldexpf(1.0f, -ex), inv = ldexpf(1.0f, ex);
                    const int W = 2 * H;
                    V ahi[2], alo[2], bhi[4], blo[4];
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb) {
                        const int j = Y0 + 16 * rb + l16;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            int d = j - say[sb + e];
                            float v = ((unsigned)d <= (unsigned)W) ? swy[sb + e][d] : 0.0f;
                            auto h = O::hi(v);
                            ahi[rb][e] = h;
                            alo[rb][e] = O::hi(v - (float)h);
                        }
                    }
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        const int i = X0 + 16 * cb + l16;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            int d = i - sax[sb + e];
                            float v = ((unsigned)d <= (unsigned)W)
                                          ? swx[sb + e][d] * (sphi[sb + e] * sc)
                                          : 0.0f;
                            auto h = O::hi(v);
                            bhi[cb][e] = h;
                            blo[cb][e] = O::hi(v - (float)h);
                        }
                    }
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                        for (int cb = 0; cb < 4; ++cb) {
                            f4 c = f4{0.f, 0.f, 0.f, 0.f};
                            c = O::mfma(ahi[rb], bhi[cb], c);
                            c = O::mfma(ahi[rb], blo[cb], c);
                            c = O::mfma(alo[rb], bhi[cb], c);
#pragma unroll
                            for (int e = 0; e < 4; ++e) acc[rb][cb][e] = fmaf(c[e], inv, acc[rb][cb][e]);
                        }
                }
                __syncthreads();
            }
        }
        // fixed-order sum of the four waves' partial tiles
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int e = 0; e < 4; ++e) red[wv][rb * 4 + cb][e][lane] = acc[rb][cb][e];
        __syncthreads();
        for (int q = tid; q < 8 * 4 * 64; q += 256) {
            const int blk = q / 256, e = (q / 64) % 4, ln = q % 64;
            const float v = ((red[0][blk][e][ln] + red[1][blk][e][ln]) + red[2][blk][e][ln]) +
                            red[3][blk][e][ln];
            const int rb = blk / 4, cb = blk % 4;
            const int gy = Y0 + 16 * rb + 4 * (ln >> 4) + e;
            const int gx = X0 + 16 * cb + (ln & 15);
            if (gx < F.nx && gy < F.ny) {
                size_t o = (size_t)gy * F.nx + gx;
                if (F.out_f64) ((double *)F.out)[o] = (double)v;
                else ((float *)F.out)[o] = v;
            }
        }
        __syncthreads();
    }
}

template <int DX, int DY, typename ST>
hipError_t launch_st(const FrameDev *frames_dev, bool bf16, const int2 *work, int n_work,
                     int *counter, int *err, int nb, hipStream_t s)
{
    if (bf16)
        hipLaunchKernelGGL((k_render_sep_mfma<DX, DY, ST, true>), dim3(nb), dim3(256), 0, s,
                           frames_dev, work, n_work, counter, err);
    else
        hipLaunchKernelGGL((k_render_sep_mfma<DX, DY, ST, false>), dim3(nb), dim3(256), 0, s,
                           frames_dev, work, n_work, counter, err);
    return hipGetLastError();
}

template <int DX, int DY>
hipError_t launch_deg(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                      int n_work, int *counter, int *err, int nb, hipStream_t s)
{
    bool bf16 = cfg.precision == E2E_PREC_BF16_HILO;
    if (cfg.spec_f64)
        return launch_st<DX, DY, double>(frames_dev, bf16, work, n_work, counter, err, nb, s);
    return launch_st<DX, DY, float>(frames_dev, bf16, work, n_work, counter, err, nb, s);
}

}  // namespace

hipError_t launch_sep_mfma(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                           int n_work, int *counter, int *err, hipStream_t s)
{
    int nb = work == nullptr ? cfg.plain_tiles : (n_work < 1024 ? n_work : 1024);
    if (nb <= 0) return hipSuccess;
    if (cfg.degx <= 4 && cfg.degy <= 3)
        return launch_deg<4, 3>(frames_dev, cfg, work, n_work, counter, err, nb, s);
    return launch_deg<7, 7>(frames_dev, cfg, work, n_work, counter, err, nb, s);
}

}  // namespace e2e
