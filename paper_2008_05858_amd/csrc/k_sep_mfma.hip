// Separable-PSF render path on the matrix cores (Sec. 2.1's axis-aligned
// Gaussian aberration model with field-dependent (sigma_x, sigma_y)).
//
// With a separable PSF the samples reaching a TY x TX tile contribute
//   F[j][i] = sum_k gy_k[j] phi_k gx_k[i],   i.e.  F = Gy diag(phi) Gx^T,
// a dense contraction over the samples, which is what MFMA computes.
//
// Per chunk of 128 samples (four k-steps of 32) one thread per (sample,
// axis) evaluates the sample's pixel integrals on the tile's columns (times
// phi) or rows and stores them in LDS already in operand layout: one line
// of 128 samples per tile column / row, so an operand fragment (8
// consecutive samples of one pixel line) is one 16-byte read.  The normal
// CDF at the pixel edges comes from fitted FP32 forms good to about one ulp
// of 1/2 (phi_lower_f32).  Each value is split into hi + lo halves (hi = round(v), lo = round(v - hi)) in two
// planes.  Entries outside a sample's window are zero: a thread clears what
// its sample slot held in the previous chunk and the new window does not
// cover (128 samples move a window by about a pixel, so one or two lines).
// Wave w then multiplies k-step w, hi*hi + hi*lo + lo*hi with
// v_mfma_f32_16x16x32_{f16,bf16} and FP32 accumulation, and skips the 16 x 16
// blocks that no sample of the k-step reaches (a chunk covers a pixel or
// two of trace, so about half of them).  phi is scaled per k-step by an
// exact power of two so every operand lies in [0, 1].  The four waves'
// partial tiles are summed in a fixed order: the result is deterministic.
#include "psf_gauss.h"

namespace e2e {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TX = kMfmaTW;   // 64 columns = 4 blocks of 16
constexpr int TY = kMfmaTH;   // 32 rows = 2 blocks of 16
constexpr int CH = 128;       // samples per chunk: 4 waves x 32
constexpr int NG = CH / 8;    // 16-byte groups of a pixel line

template <bool BF16>
struct Op;
template <>
struct Op<false> {
    using V = h8;
    using E = _Float16;
    __device__ static f4 mfma(const V &a, const V &b, const f4 &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Op<true> {
    using V = b8;
    using E = __bf16;
    __device__ static f4 mfma(const V &a, const V &b, const f4 &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// Half index of (pixel line p, sample s) in a plane: the 16-byte groups of a
// line are permuted by p, so the 16 lines one fragment read touches start on
// different banks.
__device__ __forceinline__ int lds_at(int p, int s)
{
    return p * CH + ((((s >> 3) ^ p) & (NG - 1)) << 3) + (s & 7);
}

// One sample's pixel integrals on NL consecutive pixel lines: window pixel m
// (0 .. 2H, at line off + m) gets (Phi(e_{m+1}) - Phi(e_m)) / norm * scale,
// e_m = (m - H - 1/2 - d) / sg, norm = Phi(e_{2H+1}) - Phi(e_0).  Each edge
// is one c_m = Phi(-|e_m|) (phi_lower_f32), and each difference is taken
// on the side of the centre where it does not cancel.  Writes the in-tile
// entries of both planes and returns the written line range.
template <int NL, typename E>
__device__ __forceinline__ void stage_axis(float d, float sg, int H, float scale, int off, int s,
                                           unsigned short *hi, unsigned short *lo, int *plo,
                                           int *phi_)
{
    const float inv = 1.0f / sg;
    const float c0 = phi_lower_f32(((float)(0 - H) - 0.5f - d) * inv);
    const float clast = phi_lower_f32(((float)(H + 1) - 0.5f - d) * inv);
    const float f = scale / ((1.0f - c0) - clast);
    const int m0 = max(0, -off), m1 = min(2 * H, NL - 1 - off);
    *plo = off + m0;
    *phi_ = off + m1;
    if (m0 > m1) return;
    float eprev = ((float)(m0 - H) - 0.5f - d) * inv;
    float cprev = m0 == 0 ? c0 : phi_lower_f32(eprev);
    for (int m = m0; m <= m1; ++m) {
        const float e = ((float)(m + 1 - H) - 0.5f - d) * inv;
        const float c = phi_lower_f32(e);
        // both edges right of the centre: c_m - c_{m+1}; both left:
        // c_{m+1} - c_m; one on each side: (1 - c_m) - c_{m+1}
        const bool right = eprev >= 0.0f, left = e < 0.0f;
        const float pa = right ? cprev : (left ? c : 1.0f - cprev);
        const float pb = right || !left ? c : cprev;
        const float v = pa - pb;
        const float w = v * f;
        const E h = (E)w;
        const E l = (E)(w - (float)h);
        const int a = lds_at(off + m, s);
        hi[a] = __builtin_bit_cast(unsigned short, h);
        lo[a] = __builtin_bit_cast(unsigned short, l);
        cprev = c;
        eprev = e;
    }
}

// zero lines [zlo, zhi] of both planes except [nlo, nhi]
__device__ __forceinline__ void clear_lines(int zlo, int zhi, int nlo, int nhi, int s,
                                            unsigned short *hi, unsigned short *lo)
{
    const bool none = nlo > nhi;
    const int e1 = none ? zhi : min(zhi, nlo - 1);
    for (int p = zlo; p <= e1; ++p) {
        hi[lds_at(p, s)] = 0;
        lo[lds_at(p, s)] = 0;
    }
    if (!none)
        for (int p = max(zlo, nhi + 1); p <= zhi; ++p) {
            hi[lds_at(p, s)] = 0;
            lo[lds_at(p, s)] = 0;
        }
}

// 16-line blocks covered by lines [lo, hi]
__device__ __forceinline__ unsigned block_bits(int lo, int hi)
{
    if (lo > hi) return 0u;
    const int b0 = lo >> 4, b1 = hi >> 4;
    return ((2u << b1) - 1u) & ~((1u << b0) - 1u);
}

template <int DX, int DY, typename ST, bool BF16>
__global__ __launch_bounds__(256, 3) void k_render_sep_mfma(const FrameDev *__restrict__ frames,
                                                            const int2 *__restrict__ work,
                                                            int n_work, int *__restrict__ counter,
                                                            int *__restrict__ err)
{
    using O = Op<BF16>;
    using V = typename O::V;
    using E = typename O::E;
    constexpr int PX = TX * CH, PY = TY * CH;          // halfs per plane
    constexpr int STAGEB = 2 * (2 * PX + 2 * PY);      // bytes: x hi, x lo, y hi, y lo
    constexpr int REDB = 4 * 8 * 4 * 64 * 4;           // bytes: [wave][block][e][lane] FP32
    constexpr int BUFB = STAGEB > REDB ? STAGEB : REDB;
    static_assert(TX % 16 == 0 && TY % 16 == 0 && CH == 128, "block geometry");
    __shared__ __attribute__((aligned(16))) unsigned char buf[BUFB];
    __shared__ int tlist[kMaxTileTraces];
    __shared__ int sh_count, sh_item;
    __shared__ float sinv[4];
    __shared__ unsigned smask[4][2];
    unsigned short *const xhi = reinterpret_cast<unsigned short *>(buf);
    unsigned short *const xlo = xhi + PX;
    unsigned short *const yhi = xlo + PX;
    unsigned short *const ylo = yhi + PY;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, lg = lane >> 4;
    // staging role: sample slot s of the chunk, axis (x: waves 0-1, y: 2-3)
    const int s = tid & (CH - 1);
    const bool xaxis = tid < CH;

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
                    SegDev sv = segs[tr];
                    ok = sv.k0 < sv.k1 && sv.ty0 <= ty && ty <= sv.ty1;
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
        // the staging planes start at zero
        {
            const uint4 z = {0u, 0u, 0u, 0u};
            uint4 *b4 = reinterpret_cast<uint4 *>(buf);
            for (int q = tid; q < STAGEB / 16; q += 256) b4[q] = z;
        }
        __syncthreads();
        const int count = uniform_i(sh_count);
        int zlo = 1, zhi = 0;  // lines this thread's sample slot holds (none)
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
                // ---- staging: this thread's sample and axis
                {
                    int nlo = 1, nhi = 0;
                    float phi = 0.0f;
                    double x = 0.0, y = 0.0;
                    float sgx = (float)F.sigma, sgy = (float)F.sigma;
                    if (s < nk) {
                        const int k = kc + s;
                        const double t = fma((double)k, dt, t0);
                        x = horner<DX>(cxr, t);
                        y = horner<DY>(cyr, t);
                        if (F.psf_kind == E2E_PSF_SEPARABLE)
                            sigma_at(F.sxy, F.gx, F.gy, F.gsx, F.gsy, x, y, &sgx, &sgy);
                        if (xaxis) phi = (float)spec_at(spec, k) * scale;
                    }
                    // the k-step's largest phi sets its power-of-two scale
                    float pmax = phi;
#pragma unroll
                    for (int o = 1; o < 32; o <<= 1) pmax = fmaxf(pmax, __shfl_xor(pmax, o));
                    int ex = 0;
                    if (pmax > 0.0f) frexpf(pmax, &ex);
                    if (s < nk) {
                        if (xaxis) {
                            const double axd = floor(x + 0.5);
                            stage_axis<TX, E>((float)(x - axd), sgx, H, phi * ldexpf(1.0f, -ex),
                                              (int)axd - H - X0, s, xhi, xlo, &nlo, &nhi);
                        } else {
                            const double ayd = floor(y + 0.5);
                            stage_axis<TY, E>((float)(y - ayd), sgy, H, 1.0f, (int)ayd - H - Y0,
                                              s, yhi, ylo, &nlo, &nhi);
                        }
                    }
                    if (nlo > nhi) nlo = 1, nhi = 0;
                    if (xaxis) clear_lines(zlo, zhi, nlo, nhi, s, xhi, xlo);
                    else clear_lines(zlo, zhi, nlo, nhi, s, yhi, ylo);
                    zlo = nlo;
                    zhi = nhi;
                    // blocks the k-step reaches (none where its photons are all 0)
                    unsigned bits = block_bits(nlo, nhi);
#pragma unroll
                    for (int o = 1; o < 32; o <<= 1) bits |= __shfl_xor(bits, o);
                    if ((s & 31) == 0) {
                        const int j = s >> 5;
                        if (xaxis) {
                            smask[j][0] = pmax > 0.0f ? bits : 0u;
                            sinv[j] = ldexpf(1.0f, ex);
                        } else {
                            smask[j][1] = bits;
                        }
                    }
                }
                __syncthreads();
                // ---- products: wave wv takes k-step wv (samples 32 wv .. 32 wv + 31)
                {
                    const unsigned mx = (unsigned)uniform_i((int)smask[wv][0]);
                    const unsigned my = (unsigned)uniform_i((int)smask[wv][1]);
                    if (mx != 0u && my != 0u) {
                        const float inv = sinv[wv];
                        const int g = 4 * wv + lg;  // this lane's group of 8 samples
                        V ah[2], al[2], bh[4], bl[4];
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb) {
                            if (!((my >> rb) & 1u)) continue;
                            const int p = 16 * rb + l16;
                            const int a = p * CH + (((g ^ p) & (NG - 1)) << 3);
                            ah[rb] = *reinterpret_cast<const V *>(yhi + a);
                            al[rb] = *reinterpret_cast<const V *>(ylo + a);
                        }
#pragma unroll
                        for (int cb = 0; cb < 4; ++cb) {
                            if (!((mx >> cb) & 1u)) continue;
                            const int p = 16 * cb + l16;
                            const int a = p * CH + (((g ^ p) & (NG - 1)) << 3);
                            bh[cb] = *reinterpret_cast<const V *>(xhi + a);
                            bl[cb] = *reinterpret_cast<const V *>(xlo + a);
                        }
#pragma unroll
                        for (int rb = 0; rb < 2; ++rb) {
                            if (!((my >> rb) & 1u)) continue;
#pragma unroll
                            for (int cb = 0; cb < 4; ++cb) {
                                if (!((mx >> cb) & 1u)) continue;
                                f4 c = f4{0.f, 0.f, 0.f, 0.f};
                                c = O::mfma(ah[rb], bh[cb], c);
                                c = O::mfma(ah[rb], bl[cb], c);
                                c = O::mfma(al[rb], bh[cb], c);
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    acc[rb][cb][e] = fmaf(c[e], inv, acc[rb][cb][e]);
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        // fixed-order sum of the four waves' partial tiles (the staging
        // planes are free: every wave has passed the last chunk's barrier)
        float (*red)[8][4][64] = reinterpret_cast<float (*)[8][4][64]>(buf);
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
    // plain: one workgroup per tile; persistent: three per CU
    int nb = work == nullptr ? cfg.plain_tiles : (n_work < 768 ? n_work : 768);
    if (nb <= 0) return hipSuccess;
    if (cfg.degx <= 4 && cfg.degy <= 3)
        return launch_deg<4, 3>(frames_dev, cfg, work, n_work, counter, err, nb, s);
    return launch_deg<7, 7>(frames_dev, cfg, work, n_work, counter, err, nb, s);
}

}  // namespace e2e
