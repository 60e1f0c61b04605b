// Render path for analytic Gaussian PSFs (Sec. 2.1: Gaussian aberration
// model), circular (GAUSS_ERF) or axis-aligned with (sigma_x, sigma_y)
// interpolated across the field (SEPARABLE).  A pixel's weight is the exact
// integral of the Gaussian over the pixel (Sec. 2.2: SFI integrated over the
// pixel area), i.e. a product of normal-CDF differences per axis, over a
// (2H+1)^2 window around floor(x + 1/2), renormalised by the window sum.
//
// Positions are FP64; the CDF differences are evaluated in FP32 on
// pixel-relative offsets (|offset| <= H + 1), each edge through one erfc on
// the side of the distribution where nothing cancels (library erfcf; the
// FP32 variant uses a fitted FP32 normal tail).  One workgroup owns a 16 x 16
// tile and stages one sample's per-axis weights per thread in LDS, aligned
// to the tile's columns and rows (zero outside each window).  Each thread
// adds the products of one or two pixels of one column in sample order (FP64
// sums of FP32 partials over four consecutive samples, or FP32 sums), so the
// result is deterministic and written once.
#include "psf_gauss.h"

namespace e2e {

namespace {

// NP pixels per thread (rows tcy + (16 / NP) j of column tcx), 256 / NP
// threads per tile, as many samples staged together, one per thread.  Large
// frames take NP = 2 (the column's weight read shared by two pixels), small
// ones NP = 1 (twice the waves per tile, half the chunks: lower latency).
// Both add every pixel's products in the same groups of four consecutive
// samples, so they give the same bits.
constexpr int kSepSmallTiles = 16384;

template <int DX, int DY, typename ST, bool SEP, bool ACC64, int NP>
__global__ __launch_bounds__(256 / NP) void k_render_sep(const FrameDev *__restrict__ frames,
                                                         const int2 *__restrict__ work,
                                                         int n_work, int *__restrict__ counter,
                                                         int *__restrict__ err)
{
    constexpr int TS = kSepTile;
    static_assert(TS == 16, "tile-aligned weights are 16 wide");
    static_assert(NP == 1 || NP == 2, "one or two pixels per thread");
    constexpr int kChunk = 256 / NP;
    // per staged sample, its weights on the tile's 16 columns / 16 rows
    // (zero outside its window), stored column-major ([pixel][sample]) so a
    // thread reads four consecutive samples' weights in one 16-byte load
    // (rows padded by 4 floats: the 16 rows read together start on
    // different banks)
    constexpr int RS = kChunk + 4;
    __shared__ __align__(16) float swx[TS][RS];
    __shared__ __align__(16) float swy[TS][RS];
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
        const int ntr = F.ntr, H = F.H;
        const int tx = tile_id % F.ntx, ty = tile_id / F.ntx;
        const int X0 = tx * TS, Y0 = ty * TS;
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
        const int tcx = tid % TS, tcy = tid / TS;
        const int pi = X0 + tcx, pj = Y0 + tcy;
        double acc64[NP];
        float acc32[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            acc64[j] = 0.0;
            acc32[j] = 0.0f;
        }

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
            for (int kc = sg.k0; kc < sg.k1; kc += kChunk) {
                const int nk = min(kChunk, sg.k1 - kc);
                if (tid < nk) {
                    const int k = kc + tid;
                    double t = fma((double)k, dt, t0);
                    double x = horner<DX>(cxr, t);
                    double y = horner<DY>(cyr, t);
                    double axd = floor(x + 0.5), ayd = floor(y + 0.5);
                    float sgx, sgy;
                    if (SEP) {
                        sigma_at(F.sxy, F.gx, F.gy, F.gsx, F.gsy, x, y, &sgx, &sgy);
                    } else {
                        sgx = sgy = (float)F.sigma;
                    }
                    float phi = (float)spec_at(spec, k) * scale;
                    // the FP32 variant takes the FP32 fitted normal tail
                    axis_weights_tile<TS, RS, !ACC64>((float)(x - axd), sgx, H, phi,
                                                      (int)axd - H - X0, &swx[0][tid]);
                    axis_weights_tile<TS, RS, !ACC64>((float)(y - ayd), sgy, H, 1.0f,
                                                      (int)ayd - H - Y0, &swy[0][tid]);
                } else {
#pragma unroll
                    for (int c = 0; c < TS; ++c) {
                        swx[c][tid] = 0.0f;
                        swy[c][tid] = 0.0f;
                    }
                }
                __syncthreads();
                // every staged sample in order (four per 16-byte read); outside
                // its window both weights' product is 0 and leaves the sum
                // unchanged
                const float4 *px = reinterpret_cast<const float4 *>(swx[tcx]);
                for (int q = 0; q < (nk + 3) / 4; ++q) {
                    const float4 a = px[q];
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        const float4 b =
                            reinterpret_cast<const float4 *>(swy[tcy + (TS / NP) * j])[q];
                        const float v0 = a.x * b.x, v1 = a.y * b.y, v2 = a.z * b.z,
                                    v3 = a.w * b.w;
                        if (ACC64) {
                            // four non-negative products summed in FP32 (relative
                            // error <= 3 ulp of the partial), the partials in FP64
                            acc64[j] += (double)(((v0 + v1) + v2) + v3);
                        } else {
                            acc32[j] += v0;
                            acc32[j] += v1;
                            acc32[j] += v2;
                            acc32[j] += v3;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (pi < F.nx) {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const int row = pj + (TS / NP) * j;
                if (row >= F.ny) continue;
                double v = ACC64 ? acc64[j] : (double)acc32[j];
                size_t o = (size_t)row * F.nx + pi;
                if (F.out_f64) ((double *)F.out)[o] = v;
                else ((float *)F.out)[o] = (float)v;
            }
        }
        __syncthreads();
    }
}

template <int DX, int DY, typename ST, int NP>
hipError_t launch_np(const FrameDev *frames_dev, bool acc64, bool sep, const int2 *work,
                     int n_work, int *counter, int *err, hipStream_t s)
{
    // plain: one workgroup per tile; persistent: 4096 waves, 16 per CU
    constexpr int NT = 256 / NP;
    const int cap = 2048 * 256 / (NT * 2);
    const int nb = work == nullptr ? n_work : (n_work < cap ? n_work : cap);
    if (sep) {
        if (acc64)
            hipLaunchKernelGGL((k_render_sep<DX, DY, ST, true, true, NP>), dim3(nb), dim3(NT), 0,
                               s, frames_dev, work, n_work, counter, err);
        else
            hipLaunchKernelGGL((k_render_sep<DX, DY, ST, true, false, NP>), dim3(nb), dim3(NT),
                               0, s, frames_dev, work, n_work, counter, err);
    } else {
        if (acc64)
            hipLaunchKernelGGL((k_render_sep<DX, DY, ST, false, true, NP>), dim3(nb), dim3(NT),
                               0, s, frames_dev, work, n_work, counter, err);
        else
            hipLaunchKernelGGL((k_render_sep<DX, DY, ST, false, false, NP>), dim3(nb), dim3(NT),
                               0, s, frames_dev, work, n_work, counter, err);
    }
    return hipGetLastError();
}

template <int DX, int DY, typename ST>
hipError_t launch_st(const FrameDev *frames_dev, const KernelCfg &cfg, bool sep,
                     const int2 *work, int n_items, int *counter, int *err, hipStream_t s)
{
    const bool acc64 = cfg.precision != E2E_PREC_F32;
    if (n_items < kSepSmallTiles)
        return launch_np<DX, DY, ST, 1>(frames_dev, acc64, sep, work, n_items, counter, err, s);
    return launch_np<DX, DY, ST, 2>(frames_dev, acc64, sep, work, n_items, counter, err, s);
}

template <int DX, int DY>
hipError_t launch_deg(const FrameDev *frames_dev, const KernelCfg &cfg, bool sep,
                      const int2 *work, int n_items, int *counter, int *err, hipStream_t s)
{
    if (cfg.spec_f64)
        return launch_st<DX, DY, double>(frames_dev, cfg, sep, work, n_items, counter, err, s);
    return launch_st<DX, DY, float>(frames_dev, cfg, sep, work, n_items, counter, err, s);
}

}  // namespace

// sep is read from the first frame's PSF kind on the host side and passed
// through cfg.kw: 1 = SEPARABLE, 0 = GAUSS_ERF.
hipError_t launch_sep(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                      int n_work, int *counter, int *err, hipStream_t s)
{
    // tiles of the plain launch, or work items of the persistent one
    const int n_items = work == nullptr ? cfg.plain_tiles : n_work;
    if (n_items <= 0) return hipSuccess;
    bool sep = cfg.kw != 0;
    if (cfg.degx <= 3 && cfg.degy <= 2)
        return launch_deg<3, 2>(frames_dev, cfg, sep, work, n_items, counter, err, s);
    if (cfg.degx <= 4 && cfg.degy <= 3)
        return launch_deg<4, 3>(frames_dev, cfg, sep, work, n_items, counter, err, s);
    return launch_deg<7, 7>(frames_dev, cfg, sep, work, n_items, counter, err, s);
}

}  // namespace e2e
