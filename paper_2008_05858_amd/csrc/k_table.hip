// Render path for tabulated, field-dependent PSF maps (Sec. 2.1 maps of
// cell integrals, interpolated bilinearly across the field).
//
// Exact reformulation used here.  With os cells per pixel, a kernel placed at
// x has its cells on a grid offset by the sub-cell phase rho of
// u = os x + (os - kw)/2: cell a covers (1 - rho) of slot floor(u) + a and
// rho of the next slot, and a slot lies wholly inside one pixel.  So the
// pixel weights of a sample are the CIC split (1 - rho, rho) x (1 - rho_y,
// rho_y) of four slot-aligned placements, and an aligned placement's pixel
// weights are box sums of the table over os x os cells (the "taps").  The
// bilinear field interpolation is linear in the node tables, so a sample's
// contribution is 16 deposits (2 x-slots x 2 y-rows x 4 nodes) followed by a
// fixed stencil per node: nothing is approximated.
//
// One workgroup owns one detector tile (TW x 32 pixels) and writes each of
// its pixels exactly once; no global atomics.  For every trace reaching the
// tile (ascending trace order, then node cell) it
//   1. gives each thread one slot column and finds that column's samples
//      (an interpolated guess, secant steps, an exact test on the FP64
//      format polynomial);
//   2. walks those samples in order (spectrum values read four at a time,
//      FP64 positions, FP64 moment sums per row run) into the column's
//      private 4-row deposit window held in registers;
//   3. for each band of 4 consecutive deposit rows, stores the deposits of
//      every slot column in LDS as fp16 hi + lo parts (scaled by a power of
//      two), and applies the stencils as one dense product per node layer:
//          out[i][j] = sum over (slot offset s, band row r) of
//                      D[r][4 i + s] * T[s][phase(r)][j - offset(r)],
//      i = pixel column, j = output row of the band.  Each wave owns one
//      node layer and runs v_mfma_f32_16x16x32_f16 over 16-column blocks
//      (hi*hi + hi*lo + lo*hi, FP32 accumulation); the tap fragments come
//      pre-split from the table built at load time.  The four layer
//      partials are added in FP64, in a fixed order, into the FP64 LDS tile.
// The summation order is fixed, so reruns are bitwise identical.
#include <type_traits>

#include "dev_common.h"

namespace e2e {

namespace {

constexpr int kNone = 0x3fffffff;  // "no row yet"; far from any real row
constexpr int kUnf = 64;           // traces one tile can hand on to the next

// k! S(i, k), S the Stirling numbers of the second kind: the k-th forward
// difference at 0 of j^i (unit step), for i, k <= 7
__device__ constexpr double kFwd[8][8] = {
    {1, 0, 0, 0, 0, 0, 0, 0},
    {0, 1, 0, 0, 0, 0, 0, 0},
    {0, 1, 2, 0, 0, 0, 0, 0},
    {0, 1, 6, 6, 0, 0, 0, 0},
    {0, 1, 14, 36, 24, 0, 0, 0},
    {0, 1, 30, 150, 240, 120, 0, 0},
    {0, 1, 62, 540, 1560, 1800, 720, 0},
    {0, 1, 126, 1806, 8400, 16800, 15120, 5040},
};

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u4s __attribute__((ext_vector_type(4)));
// four spectrum values (two for FP64), read at any 4-byte-aligned index
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
// four FP64 tile pixels, moved through LDS as two 16-byte halves
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ d4 ld4(const double *p)
{
    const d2 a = *reinterpret_cast<const d2 *>(p), b = *reinterpret_cast<const d2 *>(p + 2);
    return d4{a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ void st4(double *p, d4 v)
{
    *reinterpret_cast<d2 *>(p) = d2{v.x, v.y};
    *reinterpret_cast<d2 *>(p + 2) = d2{v.z, v.w};
}

template <typename ST>
struct SpecVec;
template <>
struct SpecVec<float> {
    static constexpr int G = 4;
    __device__ static void load(gptr<float> p, int k, int n, float v[4])
    {
        if (__builtin_expect(k + 4 <= n, 1)) {
            const f4u q = *(const __attribute__((address_space(1))) f4u *)(p + k);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = k + e < n ? p[k + e] : 0.0f;
        }
    }
};
template <>
struct SpecVec<double> {
    static constexpr int G = 2;
    __device__ static void load(gptr<double> p, int k, int n, double v[2])
    {
        if (__builtin_expect(k + 2 <= n, 1)) {
            const d2u q = *(const __attribute__((address_space(1))) d2u *)(p + k);
            v[0] = q.x; v[1] = q.y;
        } else {
            v[0] = k < n ? p[k] : 0.0;
            v[1] = k + 1 < n ? p[k + 1] : 0.0;
        }
    }
};

// Reduction over the 64 lanes of a wave by DPP row operations (exchange
// within quads, mirrors within half-rows and rows, then row broadcasts into
// the last row), read back from lane 63 as a uniform value.  Every lane of
// the wave must be active.
template <typename Op>
__device__ int wave_reduce(int v, int ident, Op op)
{
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

template <int KW, int DX, int DY, typename ST>
__global__ __launch_bounds__(kTableThreads, 3) void k_render_table(
    const FrameDev *__restrict__ frames, const int2 *__restrict__ work, int n_work,
    int *__restrict__ counter, int *__restrict__ err)
{
    constexpr int OS = kOS;
    constexpr int NCOL = kTableThreads;        // slot columns per tile
    constexpr int TW = (NCOL - KW) / OS;       // tile width in pixels
    constexpr int TH = kTableTH;
    constexpr int DD = (KW + OS - 2) / OS + 1; // pixel rows per deposit row
    constexpr int NJ = DD + 1;                 // output rows a band reaches
    constexpr int NKS = table_ksteps(KW);      // k-steps of 32 per node layer
    constexpr int RL = table_band_slots(KW);   // slots of a band row in LDS
    constexpr int NFR = NJ + 1;                // tap-fragment rows per phase
    constexpr int FRS = table_frag_row(KW);    // halfs per tap-fragment row
    constexpr int KC = KW <= 32 ? 128 : 256;   // trace segments one run of tiles can hold
    constexpr double UC = 0.5 * (OS - KW);
    static_assert(OS * TW + KW == NCOL, "tile geometry");
    static_assert(TW <= 64 && NJ <= 16, "one MFMA block of output rows, four of columns");
    static_assert(4 * 63 + 2 * (4 * NKS - 1) + 2 <= RL, "band row covers the reads");

    constexpr int CR = 16;                     // carried rows below a tile
    constexpr int XS = 17;                     // floats per column in the left-half exchange
    constexpr int BANDB = 2 * 4 * RL * 8;      // bytes: [plane][layer][slot][4 rows] fp16
    constexpr int PARTB = 4 * 4 * 64 * 16;     // bytes: [layer][m-block][lane] float4
    constexpr int BUFB = BANDB > PARTB ? BANDB : PARTB;
    static_assert(NCOL * XS * 4 <= BUFB, "the left-half exchange fits the band buffer");

    // The band (fp16 hi and lo planes of the 4 layers' deposits) and, once
    // the products have read it, the four layers' FP32 partial outputs.
    __shared__ __attribute__((aligned(16))) unsigned char bandbuf[BUFB];
    __shared__ __attribute__((aligned(16))) double tile[TH][TW];
    __shared__ __attribute__((aligned(16))) double carry[CR][TW];  // rows of the next tile
    static_assert(TW % 4 == 0, "tile rows move as groups of four pixels");
    constexpr int TQ = TW / 4;                   // four-pixel groups per tile row
    __shared__ int unf[2][kUnf];                 // traces with rows beyond the carry
    __shared__ int sh_nunf[2];
    __shared__ unsigned char tcont[KC];          // item continues from the tile above
    __shared__ int kst[NCOL + 1];
    __shared__ int ctr[KC];                      // the run's trace segments: trace,
    __shared__ SegDev cseg[KC];                  // segment record,
    // per-frame constants of the run's segments (kept in LDS for 32-cell
    // tables; 48-cell tables read them from memory, so 3 workgroups fit a CU)
    constexpr bool kMetaLds = KW <= 32;
    __shared__ TraceFrameDev cmeta[kMetaLds ? KC : 1];
    __shared__ unsigned char tlist[KC];          // this tile's items (candidate index)
    __shared__ int sh_wsum[4], sh_item;
    __shared__ int sh_tsum[2][4];                // tile item counts per wave, by tile parity
    // per node-cell pass reductions, double-buffered by pass parity so a
    // pass's reset cannot meet a slow wave's read of the previous pass
    __shared__ int sh_qmin[2], sh_qmax[2];
    __shared__ unsigned sh_dmax[2];

    // The thread index is re-read through an empty asm statement (which the
    // compiler cannot see through) at the top of each loop level, so the
    // addresses, masks and conversions derived from it are recomputed where
    // they are used instead of being hoisted to the kernel entry and held, or
    // spilled, across the whole kernel; the same for the segment's sample range
    // in each node-cell pass.  (This removed every VGPR spill at 3 workgroups
    // per CU.)
    const int tid_in = threadIdx.x;
    auto fresh_tid = [&]() {
        int t = tid_in;
        asm volatile("" : "+v"(t));
        return t;
    };
    const int tid = fresh_tid();
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    int cpar = 0;  // parity of the node-cell pass

    for (int iter = 0;; ++iter) {
        const int tid = fresh_tid();
        const int lane = tid & 63;
        int fi, unit;
        if (work == nullptr) {
            if (iter > 0) break;
            fi = 0;
            unit = xcd_remap(blockIdx.x, gridDim.x);
        } else {
            if (tid == 0) sh_item = atomicAdd(counter, 1);
            __syncthreads();
            int w = uniform_i(sh_item);
            if (w >= n_work) break;
            int2 wk = work[w];
            fi = uniform_i(wk.x);
            unit = uniform_i(wk.y);
        }
        cptr<FrameDev> Fp = as_const(frames) + fi;
        const int ntr = Fp->ntr;
        // A unit is a run of `chunk` tiles down one column, walked top to
        // bottom.  A trace segment is processed at the first tile of the run
        // it reaches, for every output row up to CR rows into the next tile
        // (the carry); only a segment with rows beyond that is taken up again
        // by the next tile.
        const int chunk = Fp->chunk;
        const int nchunk = (Fp->nty + chunk - 1) / chunk;
        const int tx = unit / nchunk, ty_a = (unit % nchunk) * chunk;
        const int ty_b = min(ty_a + chunk, Fp->nty);
        const int X0 = tx * TW;
        const SegDev *segs = Fp->segs + (size_t)tx * ntr;
        // four consecutive pixels of the frame from (gy, gx), rounded once to
        // FP32 (one 16-byte store when the rows are a multiple of four pixels
        // on a 16-byte boundary: gx is a multiple of four), or kept in FP64
        auto put4 = [&](int gy, int gx, d4 v) {
            const int nx = Fp->nx;
            if (gy >= Fp->ny || gx >= nx) return;
            const size_t o = (size_t)gy * nx + gx;
            if (Fp->out_f64) {
                double *d = (double *)Fp->out + o;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (gx + e < nx) d[e] = v[e];
            } else if (((nx & 3) | ((unsigned)(size_t)Fp->out & 15u)) == 0) {
                *reinterpret_cast<f4 *>((float *)Fp->out + o) =
                    f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            } else {
                float *d = (float *)Fp->out + o;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (gx + e < nx) d[e] = (float)v[e];
            }
        };
        for (int e = tid; e < CR * TW; e += kTableThreads) carry[e / TW][e % TW] = 0.0;
        if (tid < 2) sh_nunf[tid] = 0;

        // ---- the column's trace segments that reach any tile of the run,
        // ascending: each thread tests a run of eight traces (one round of
        // loads), a block-wide prefix sum places them
        int ncand = 0;
        for (int pb = 0; pb < ntr; pb += 8 * NCOL) {
            const int mb = pb + 8 * tid;
            unsigned bits = 0;
            SegDev sgv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sgv[j] = segs[min(mb + j, ntr - 1)];
                const bool ok = mb + j < ntr && sgv[j].k0 < sgv[j].k1 && sgv[j].ty0 < ty_b &&
                                sgv[j].ty1 >= ty_a;
                bits |= ok ? 1u << j : 0u;
            }
            const int cnt = __popc(bits);
            int x = cnt;  // inclusive scan over the wave
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) sh_wsum[wv] = x;
            __syncthreads();
            int pos = ncand + x - cnt, tot = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int v = sh_wsum[w];
                pos += w < wv ? v : 0;
                tot += v;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (!((bits >> j) & 1)) continue;
                if (pos < KC) {
                    ctr[pos] = mb + j;
                    cseg[pos] = sgv[j];
                    if constexpr (kMetaLds) cmeta[pos] = Fp->tf[mb + j];
                } else {
                    atomicOr(err, kErrTileTraces);
                }
                ++pos;
            }
            ncand = min(ncand + uniform_i(tot), KC);
            __syncthreads();
        }

        for (int ty = ty_a; ty < ty_b; ++ty) {
        const int tid = fresh_tid();
        const int lane = tid & 63;
        const int Y0 = ty * TH;
        const int up = (ty - ty_a) & 1;  // unfinished list of the tile above
        const int nup = uniform_i(sh_nunf[up]);
        // this tile's own list starts empty.  Reset here, before the count
        // barrier: the list was last read in the previous tile's selection,
        // which every wave has left, and the reset is visible to all after
        // the barrier, including to the next tile when this one has no item.
        if (tid == 0) sh_nunf[up ^ 1] = 0;

        // ---- this tile's items, ascending: thread c tests candidate c.  A
        // segment is taken at the first tile of the run it reaches, and again
        // only if the tile above listed it as reaching past its carry.
        int count;
        {
            const int c = tid;
            bool ok = false, cnt_c = false;
            if (c < ncand) {
                const SegDev sc = cseg[c];
                const bool reach = sc.ty0 <= ty && ty <= sc.ty1;
                const bool fresh = sc.ty0 >= ty || ty == ty_a;
                bool more = nup > kUnf;  // the list overflowed: take every one up
                if (reach && !fresh && !more) {
                    const int t = ctr[c];
                    int lo = 0, hi = nup;  // unf[up] is ascending
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (unf[up][mid] < t) lo = mid + 1; else hi = mid;
                    }
                    more = lo < nup && unf[up][lo] == t;
                }
                ok = reach && (fresh || more);
                cnt_c = ok && !fresh;
            }
            // (the counts alternate between two buffers: a wave may reach the
            // next tile's count while another still reads this one's)
            const unsigned long long m = __ballot(ok);
            if (lane == 0) sh_tsum[up][wv] = __popcll(m);
            __syncthreads();
            int pos = __popcll(m & ((1ull << lane) - 1ull)), tot = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int v = sh_tsum[up][w];
                pos += w < wv ? v : 0;
                tot += v;
            }
            if (ok) {
                tlist[pos] = (unsigned char)c;
                tcont[pos] = cnt_c;
            }
            count = uniform_i(tot);
        }
        if (count == 0) {
            // no item: the tile is the rows carried down from the tile above,
            // written at once (each thread clears the carry entries it reads)
            for (int e = tid; e < TH * TQ; e += kTableThreads) {
                const int r = e / TQ, c = 4 * (e % TQ);
                d4 v = {0.0, 0.0, 0.0, 0.0};
                if (r < CR) {
                    v = ld4(&carry[r][c]);
                    st4(&carry[r][c], d4{0.0, 0.0, 0.0, 0.0});
                }
                put4(Y0 + r, X0 + c, v);
            }
            continue;
        }
        // the tile starts from the rows carried down from the tile above
        for (int e = tid; e < TH * TQ; e += kTableThreads) {
            const int r = e / TQ, c = 4 * (e % TQ);
            d4 v = {0.0, 0.0, 0.0, 0.0};
            if (r < CR) {
                v = ld4(&carry[r][c]);
                st4(&carry[r][c], d4{0.0, 0.0, 0.0, 0.0});
            }
            st4(&tile[r][c], v);
        }
        __syncthreads();
        const bool last_tile = ty + 1 >= ty_b;

        for (int li = 0; li < count; ++li) {
            const int ci = uniform_i(tlist[li]);
            const int tr = uniform_i(ctr[ci]);
            SegDev sg;
            {
                int4 raw = *reinterpret_cast<const int4 *>(&cseg[ci]);
                raw.x = uniform_i(raw.x);
                raw.y = uniform_i(raw.y);
                raw.z = uniform_i(raw.z);
                raw.w = uniform_i(raw.w);
                __builtin_memcpy(&sg, &raw, sizeof(sg));
            }
            const bool multi = (sg.cx0 != sg.cx1) | (sg.cy0 != sg.cy1);
            // output rows this pass owns: from the tile top (or below the rows
            // the tile above already carried) to the end of the carry
            const int out_lo = uniform_i(tcont[li]) ? Y0 + CR : Y0;
            const int out_hi = last_tile ? Y0 + TH - 1 : Y0 + TH + CR - 1;

            for (int cyc = sg.cy0; cyc <= sg.cy1; ++cyc)
            for (int cxc = sg.cx0; cxc <= sg.cx1; ++cxc) {
                const int tid = fresh_tid();
                const int lane = tid & 63;
                int k0 = sg.k0, k1 = sg.k1;
                asm volatile("" : "+s"(k0), "+s"(k1));
                cpar ^= 1;
                cptr<TraceDev> Tp = as_const(Fp->tr) + tr;
                double cxr[DX + 1], cyr[DY + 1];
#pragma unroll
                for (int j = 0; j <= DX; ++j) cxr[j] = Tp->cx[j];
#pragma unroll
                for (int j = 0; j <= DY; ++j) cyr[j] = Tp->cy[j];
                const int nspec = Tp->n;
                double t0, dt, scale;
                gptr<ST> spec;
                if constexpr (kMetaLds) {
                    t0 = uniform_d(cmeta[ci].t0);
                    dt = uniform_d(cmeta[ci].dt);
                    scale = uniform_d(cmeta[ci].scale);
                    spec = as_global(uniform_ptr<ST>(cmeta[ci].spec));
                } else {
                    cptr<TraceFrameDev> Mp = as_const(Fp->tf) + tr;
                    t0 = Mp->t0;
                    dt = Mp->dt;
                    scale = Mp->scale;
                    spec = as_global(reinterpret_cast<const ST *>(Mp->spec));
                }
                const double gsx = Fp->gsx, gsy = Fp->gsy;
                const int gxn = Fp->gx, gyn = Fp->gy;
                // ---- 1. samples of each slot column: first k with u(k) >= q
                const int q = OS * X0 - KW + tid;
                auto u_of = [&](int k) {
                    double x = horner<DX>(cxr, fma((double)k, dt, t0));
                    return fma(x, (double)OS, UC);
                };
                // The sample index as a function of the slot coordinate,
                // interpolated (Newton form) through the segment's first,
                // middle and last samples: a guess within a small fraction of
                // a sample on moderately sampled segments (hundreds of samples
                // off on densely sampled ones), which the secant steps and the
                // exact test below settle.
                const int km = k0 + ((k1 - 1 - k0) >> 1);
                const double ua = u_of(k0), um = u_of(km), ub = u_of(k1 - 1);
                double d1 = 0.0, d2 = 0.0;
                if (km > k0 && km < k1 - 1) {  // three distinct samples (u grows with k)
                    d1 = (double)(km - k0) / (um - ua);
                    d2 = ((double)(k1 - 1 - km) / (ub - um) - d1) / (ub - ua);
                }
                auto search = [&](int qq) -> int {
                    const double uq = (double)qq;
                    if (uq <= ua) return k0;
                    if (uq > ub) return k1;
                    // here u(k0) < qq <= u(k1 - 1): the answer lies in [k0 + 1, k1 - 1]
                    auto first_at = [&](double kk) {  // ceil, kept in [k0 + 1, k1 - 1]
                        const int k = (int)ceil(fmin(fmax(kk, (double)k0), (double)(k1 - 1)));
                        return min(max(k, k0 + 1), k1 - 1);
                    };
                    int k = first_at(fma((uq - ua), fma(uq - um, d2, d1), (double)k0));
                    // the guess and its left neighbour tested together
                    double uk = u_of(k), ul = u_of(k - 1);
                    // A guess more than a sample off (densely sampled segments
                    // whose format bends over the segment): secant steps on the
                    // slope between the two evaluated samples.
                    for (int it = 0; it < 8 && (uk < uq || ul >= uq); ++it) {
                        const double du = uk - ul;
                        if (!(du > 0.0)) break;
                        int kn = first_at((double)k + (uq - uk) / du);
                        if (kn == k) kn = uk < uq ? min(k + 1, k1 - 1) : max(k - 1, k0 + 1);
                        if (kn == k) break;
                        k = kn;
                        uk = u_of(k);
                        ul = u_of(k - 1);
                    }
                    // a remaining miss walks on (u(k0) < qq <= u(k1 - 1) ends
                    // either walk)
                    int guard = 0;
                    if (uk < uq) {
                        ++k;
                        while (k < k1 - 1 && u_of(k) < uq && guard < 256) { ++k; ++guard; }
                    } else if (ul >= uq) {
                        --k;
                        while (k > k0 + 1 && u_of(k - 1) >= uq && guard < 256) { --k; ++guard; }
                    }
                    if (guard >= 256) atomicOr(err, kErrSearch);
                    return k;
                };
                const int ks_own = search(q);
                kst[tid] = ks_own;
                // the last column ends where the planner's range ends (the
                // first sample at or past the tile's right edge, or past the frame's)
                if (tid == NCOL - 1) kst[NCOL] = k1;
                if (tid == 0) {
                    sh_qmin[cpar] = 0x7fffffff;
                    sh_qmax[cpar] = -0x7fffffff;
                    sh_dmax[cpar] = 0u;
                }
                // the column's first spectrum values, loaded before the barrier
                // so that their latency overlaps it
                constexpr int G = SpecVec<ST>::G;
                ST v0[G];
                SpecVec<ST>::load(spec, ks_own, nspec, v0);
                __syncthreads();

                // ---- 2. this column's samples, in order.  Within one row run the
                // 16 deposits (2 x-slots x 2 rows x 4 nodes) are polynomials of
                // degree <= 2 in the sub-slot phases (rx, ry), because the CIC
                // weights and the node weights are both affine in them; so the
                // run keeps the 9 moments sum phi rx^a ry^b (FP64) and turns
                // them into deposits when the row changes.  Deposits go to the
                // column's 4-row window wr[layer][x-slot][row] (rows rb..rb+3).
                const int ks = kst[tid];
                int ke = kst[tid + 1];
                int nbx, nby;
                double ax0, ax1, ay0, ay1;
                cell_line(cxc, gsx, gxn, &nbx, &ax0, &ax1);
                cell_line(cyc, gsy, gyn, &nby, &ay0, &ay1);
                // fx = ax0 + ax1 * x with x = (q + rx - UC) / OS
                const double fxa = fma(ax1, ((double)q - UC) / OS, ax0), fxb = ax1 / OS;
                const double fyb = ay1 / OS;
                float wr[4][2][4];
#pragma unroll
                for (int l = 0; l < 4; ++l)
#pragma unroll
                    for (int lr = 0; lr < 2; ++lr)
#pragma unroll
                        for (int r = 0; r < 4; ++r) wr[l][lr][r] = 0.0f;
                double m[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) m[a][b] = 0.0;
                int runQy = kNone, rb = kNone;
                bool run_in = false;
                int qmin = 0x7fffffff, qmax = -0x7fffffff;
                double csum = 0.0;  // photons of the column (bounds its deposits)
                // the x factor (CIC x node weight) of each deposit is a0 + a1 rx +
                // a2 rx^2 with these coefficients, times the flux scale
                const double xs = scale, xa = fxa * scale, xb = fxb * scale;

                auto flush = [&]() {
                    const int o = runQy - rb;
                    if (__builtin_expect(o < 0 || o > 2, 0)) {
                        atomicOr(err, kErrRowWindow);
                        return;
                    }
                    if (run_in) {
                        qmin = min(qmin, runQy);
                        qmax = max(qmax, runQy);
                    }
                    csum += m[0][0];
                    const double fya = fma(ay1, ((double)runQy - UC) / OS, ay0);
                    // y factor (CIC x node weight) of row half r, node ny:
                    // Y[r][ny][0] + Y[r][ny][1] ry + Y[r][ny][2] ry^2
                    double Y[2][2][3];
                    Y[0][1][0] = fya;       Y[0][1][1] = fyb - fya;       Y[0][1][2] = -fyb;
                    Y[0][0][0] = 1.0 - fya; Y[0][0][1] = fya - 1.0 - fyb; Y[0][0][2] = fyb;
                    Y[1][1][0] = 0.0;       Y[1][1][1] = fya;             Y[1][1][2] = fyb;
                    Y[1][0][0] = 0.0;       Y[1][0][1] = 1.0 - fya;       Y[1][0][2] = -fyb;
                    double X[2][2][3];
                    X[0][1][0] = xa;      X[0][1][1] = xb - xa;      X[0][1][2] = -xb;
                    X[0][0][0] = xs - xa; X[0][0][1] = xa - xs - xb; X[0][0][2] = xb;
                    X[1][1][0] = 0.0;     X[1][1][1] = xa;           X[1][1][2] = xb;
                    X[1][0][0] = 0.0;     X[1][0][1] = xs - xa;      X[1][0][2] = -xb;
                    double Tm[2][2][3];
#pragma unroll
                    for (int r = 0; r < 2; ++r)
#pragma unroll
                        for (int ny = 0; ny < 2; ++ny)
#pragma unroll
                            for (int a = 0; a < 3; ++a)
                                Tm[r][ny][a] = fma(Y[r][ny][2], m[a][2],
                                                   fma(Y[r][ny][1], m[a][1], Y[r][ny][0] * m[a][0]));
                    float dv[4][2][2];
#pragma unroll
                    for (int l = 0; l < 4; ++l)
#pragma unroll
                        for (int lr = 0; lr < 2; ++lr)
#pragma unroll
                            for (int r = 0; r < 2; ++r) {
                                const int nx = l & 1, ny = l >> 1;
                                dv[l][lr][r] = (float)fma(X[lr][nx][2], Tm[r][ny][2],
                                                          fma(X[lr][nx][1], Tm[r][ny][1],
                                                              X[lr][nx][0] * Tm[r][ny][0]));
                            }
                    // rows runQy, runQy + 1 are window rows o, o + 1: fixed rows 1, 2
                    // for a column's first run (the usual case), selects otherwise
                    // (a dynamic index would move the window out of registers)
                    if (__builtin_expect(o == 1, 1)) {
#pragma unroll
                        for (int l = 0; l < 4; ++l)
#pragma unroll
                            for (int lr = 0; lr < 2; ++lr) {
                                wr[l][lr][1] += dv[l][lr][0];
                                wr[l][lr][2] += dv[l][lr][1];
                            }
                    } else {
                        const bool o0 = o == 0, o2 = o == 2;
#pragma unroll
                        for (int l = 0; l < 4; ++l)
#pragma unroll
                            for (int lr = 0; lr < 2; ++lr) {
                                const float d0 = dv[l][lr][0], d1 = dv[l][lr][1];
                                wr[l][lr][0] += o0 ? d0 : 0.0f;
                                wr[l][lr][1] += o0 ? d1 : 0.0f;
                                wr[l][lr][2] += o2 ? d0 : 0.0f;
                                wr[l][lr][3] += o2 ? d1 : 0.0f;
                            }
                    }
                };
                // Positions of the column's samples ks + j by forward differences
                // of the FP64 format polynomials (exact up to rounding): px is
                // u - q = OS x + UC - q (the slot phase rx), py is OS y + UC - runQy
                // (the row phase ry of the current run).
                double px[DX + 1], py[DY + 1];
                auto setup = [&]() {
                    const double ts = fma((double)ks, dt, t0);
                    // Taylor coefficients at ts (synthetic division), in powers of
                    // j dt, scaled to slots
                    double bx[DX + 1], by[DY + 1];
#pragma unroll
                    for (int i = 0; i <= DX; ++i) bx[i] = cxr[i];
#pragma unroll
                    for (int i = 0; i <= DY; ++i) by[i] = cyr[i];
#pragma unroll
                    for (int i = 0; i < DX; ++i)
#pragma unroll
                        for (int k = DX - 1; k >= i; --k) bx[k] = fma(ts, bx[k + 1], bx[k]);
#pragma unroll
                    for (int i = 0; i < DY; ++i)
#pragma unroll
                        for (int k = DY - 1; k >= i; --k) by[k] = fma(ts, by[k + 1], by[k]);
                    double h = (double)OS;
#pragma unroll
                    for (int i = 0; i <= (DX > DY ? DX : DY); ++i) {
                        if (i <= DX) bx[i] *= h;
                        if (i <= DY) by[i] *= h;
                        h *= dt;
                    }
                    // forward differences at j = 0: d^k P = sum_i p_i k! S(i, k)
#pragma unroll
                    for (int k = 1; k <= DX; ++k) {
                        double d = 0.0;
#pragma unroll
                        for (int i = DX; i >= k; --i) d = fma(bx[i], kFwd[i][k], d);
                        px[k] = d;
                    }
#pragma unroll
                    for (int k = 1; k <= DY; ++k) {
                        double d = 0.0;
#pragma unroll
                        for (int i = DY; i >= k; --i) d = fma(by[i], kFwd[i][k], d);
                        py[k] = d;
                    }
                    px[0] = bx[0] + (UC - (double)q);
                    const double vy = by[0] + UC, fl = floor(vy);
                    runQy = (int)fl;
                    rb = runQy - 1;
                    py[0] = vy - fl;
                };
                auto sample = [&](double sv, auto mc) {
                    double rx = px[0];
                    double ry = py[0];
                    // the row changes (rare) unless 0 <= ry < 1: one unsigned
                    // compare of the high word (negative values have the sign bit)
                    if (__builtin_expect((unsigned)(__double_as_longlong(ry) >> 32) >= 0x3ff00000u, 0)) {
                        flush();
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b) m[a][b] = 0.0;
                        const double f = floor(ry);
                        runQy += (int)f;
                        ry -= f;
                        py[0] = ry;
                        run_in = false;
                    }
                    bool in = true;
                    if constexpr (decltype(mc)::value) {
                        const double x = (rx + ((double)q - UC)) / OS;
                        const double y = (ry + ((double)runQy - UC)) / OS;
                        in = (ext_cell(x, gsx, gxn) == cxc) & (ext_cell(y, gsy, gyn) == cyc);
                    }
                    const double phi = in ? sv : 0.0;
                    run_in |= in;
                    const double e1 = phi * ry, e2 = e1 * ry, rx2 = rx * rx;
                    m[0][0] += phi;
                    m[0][1] += e1;
                    m[0][2] += e2;
                    m[1][0] = fma(phi, rx, m[1][0]);
                    m[1][1] = fma(e1, rx, m[1][1]);
                    m[1][2] = fma(e2, rx, m[1][2]);
                    m[2][0] = fma(phi, rx2, m[2][0]);
                    m[2][1] = fma(e1, rx2, m[2][1]);
                    m[2][2] = fma(e2, rx2, m[2][2]);
                    // next sample
#pragma unroll
                    for (int k = 0; k < DX; ++k) px[k] += px[k + 1];
#pragma unroll
                    for (int k = 0; k < DY; ++k) py[k] += py[k + 1];
                };
                // a trace segment that stays in one node cell (the usual case)
                // needs no per-sample cell test: two instances of the loop
                auto walk = [&](auto mc) {
                    if (ks >= ke) return;
                    setup();
                    // spectrum values G at a time (one 16-byte load per lane),
                    // the next group's load issued before this group's samples
                    ST v[G], nv[G];
#pragma unroll
                    for (int e = 0; e < G; ++e) v[e] = v0[e];
                    int kb = ks;
                    for (; kb + G <= ke; kb += G) {  // whole groups: no per-sample test
                        SpecVec<ST>::load(spec, min(kb + G, ke - 1), nspec, nv);
#pragma unroll
                        for (int e = 0; e < G; ++e) sample((double)v[e], mc);
#pragma unroll
                        for (int e = 0; e < G; ++e) v[e] = nv[e];
                    }
#pragma unroll
                    for (int e = 0; e < G - 1; ++e)
                        if (kb + e < ke) sample((double)v[e], mc);
                    flush();
                };
                // A segment that spans several node cells is walked once per
                // cell.  A column whose x range lies wholly outside this cell
                // (with a margin far above rounding) has no sample in it and is
                // skipped; one wholly inside it, on a segment within one y cell,
                // needs no per-sample test.  Only the columns at a cell boundary
                // take the tested walk, and a wave takes it only if one of its
                // columns needs it.
                bool tested = multi;
                if (multi) {
                    const double xl = ((double)q - UC) / OS - 1e-6;
                    const double xh = ((double)q + 1.0 - UC) / OS + 1e-6;
                    const int ca = ext_cell(xl, gsx, gxn), cb = ext_cell(xh, gsx, gxn);
                    if (ca > cxc || cb < cxc) ke = ks;
                    const bool inside = ca == cxc && cb == cxc && sg.cy0 == sg.cy1;
                    tested = !__all(inside || ke <= ks);
                }
                if (tested) walk(std::true_type());
                else walk(std::false_type());
                // the left-slot halves belong to slot c - 1: hand them (and the
                // window's first row) to the column on the left through LDS
                float *xw = reinterpret_cast<float *>(bandbuf);
#pragma unroll
                for (int l = 0; l < 4; ++l)
#pragma unroll
                    for (int r = 0; r < 4; ++r) xw[tid * XS + l * 4 + r] = wr[l][0][r];
                xw[tid * XS + 16] = __int_as_float(rb);
                // column bound on any one deposit: all its photons
                const float cmax = (float)(csum * scale) * 1.0001f;  // >= 0
                const int wqmin = wave_reduce(qmin, 0x7fffffff, [](int a, int b) { return min(a, b); });
                const int wqmax = wave_reduce(qmax, -0x7fffffff, [](int a, int b) { return max(a, b); });
                const unsigned wcmax = (unsigned)wave_reduce(
                    __float_as_int(cmax), 0,
                    [](int a, int b) { return (int)max((unsigned)a, (unsigned)b); });
                if (lane == 0 && wqmin <= wqmax) {
                    atomicMin(&sh_qmin[cpar], wqmin);
                    atomicMax(&sh_qmax[cpar], wqmax);
                    atomicMax(&sh_dmax[cpar], wcmax);
                }
                __syncthreads();

                // ---- 3. stencils over bands of 4 consecutive deposit rows (any
                // start).  Deposit row 4n + p reaches output rows n .. n + DD - 1;
                // a band starting at A spans output rows A/4 .. A/4 + NJ - 1.
                const int qlo = uniform_i(sh_qmin[cpar]), qhi = uniform_i(sh_qmax[cpar]) + 1;
                if (qlo > qhi) continue;  // no sample of this cell here (uniform)
                // rows reaching below this pass: the next tile takes the trace up
                if (!last_tile && (qhi >> 2) + DD - 1 > out_hi && tid == 0) {
                    const int n = sh_nunf[up ^ 1];
                    if (n == 0 || unf[up ^ 1][min(n, kUnf) - 1] != tr) {
                        if (n < kUnf) unf[up ^ 1][n] = tr;
                        sh_nunf[up ^ 1] = n + 1;
                    }
                }
                const int rlo = max(qlo, OS * (out_lo - (DD - 1)));
                const int rhi = min(qhi, OS * out_hi + OS - 1);
                if (rlo > rhi) continue;
                // deposits are non-negative and at most 2 column totals: scale
                // them into [0, 2^14) for fp16 (an exact power of two)
                const float dmax = 2.0f * __uint_as_float(uniform_i((int)sh_dmax[cpar]));
                if (!(dmax > 0.0f)) continue;
                int dex;
                frexpf(dmax, &dex);
                const float dsc = ldexpf(1.0f, 14 - dex);
                const double unsc = ldexp(1.0, dex - 14 - kTapShift);
                // slot c's deposits: its right-slot halves and column c + 1's
                // left-slot halves.  Adjacent columns' first rows differ by at
                // most one (|dy/dx| <= 1/2 over a quarter pixel), so slot c's
                // rows fit a 5-row window from mrb.  Each layer's window is kept
                // scaled, as fp16 hi and lo parts packed four rows to a 64-bit
                // word: rows 1..4 in w1[l], row 0 in the top half of w0[l].
                unsigned long long w1h[4], w1l[4];
                unsigned w0h[4], w0l[4];
                int mrb;
                {
                    const int nrb = tid + 1 < NCOL ? __float_as_int(xw[(tid + 1) * XS + 16]) : kNone;
                    mrb = rb == kNone ? nrb : (nrb == kNone ? rb : min(rb, nrb));
                    const int da = rb == kNone ? 8 : rb - mrb, dn = nrb == kNone ? 8 : nrb - mrb;
                    if (da > 1 && da != 8) atomicOr(err, kErrRowWindow);
                    if (dn > 1 && dn != 8) atomicOr(err, kErrRowWindow);
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        float nl[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            nl[r] = tid + 1 < NCOL ? xw[(tid + 1) * XS + l * 4 + r] : 0.0f;
                        unsigned hh[5], ll[5];
#pragma unroll
                        for (int u = 0; u < 5; ++u) {
                            float a = 0.0f, b = 0.0f;
                            if (u < 4) a = da == 0 ? wr[l][1][u] : a;
                            if (u >= 1) a = da == 1 ? wr[l][1][u - 1] : a;
                            if (u < 4) b = dn == 0 ? nl[u] : b;
                            if (u >= 1) b = dn == 1 ? nl[u - 1] : b;
                            const float v = (a + b) * dsc;
                            const _Float16 h = (_Float16)v;
                            const _Float16 lo = (_Float16)(v - (float)h);
                            hh[u] = __builtin_bit_cast(unsigned short, h);
                            ll[u] = __builtin_bit_cast(unsigned short, lo);
                        }
                        w0h[l] = hh[0] << 16;
                        w0l[l] = ll[0] << 16;
                        w1h[l] = (unsigned long long)(hh[1] | (hh[2] << 16)) |
                                 ((unsigned long long)(hh[3] | (hh[4] << 16)) << 32);
                        w1l[l] = (unsigned long long)(ll[1] | (ll[2] << 16)) |
                                 ((unsigned long long)(ll[3] | (ll[4] << 16)) << 32);
                    }
                }
                __syncthreads();  // the exchange area becomes the band
                // rows A - mrb .. A - mrb + 3 of the packed window (zero outside):
                // with o = A - mrb + 3, halfs o..o+3 of [0, 0, 0, row 0 .. row 4, 0 ...]
                // (a 128-bit funnel shift, without branches: the columns of a wave
                // have different o)
                auto band4 = [](unsigned w0, unsigned long long w1, int o) -> unsigned long long {
                    const unsigned long long lo = (unsigned long long)w0 << 32;
                    const unsigned sh = 16u * (unsigned)o;
                    const unsigned long long a = lo >> (sh & 63u);
                    const unsigned long long b = w1 << ((64u - sh) & 63u);
                    const unsigned long long c = w1 >> ((sh - 64u) & 63u);
                    const unsigned long long r = sh >= 64u ? c : (sh == 0u ? a : (a | b));
                    return (o < 0 || o > 7) ? 0ull : r;
                };
                // this wave's node layer: fragments of its taps (both planes)
                const int mx = min(nbx + (wv & 1), gxn - 1);
                const int my = min(nby + (wv >> 1), gyn - 1);
                gptr<h8> tfr = as_global(reinterpret_cast<const h8 *>(Fp->tfrag)) +
                               (size_t)(my * gxn + mx) * (2 * 4 * NFR * FRS / 8);
                for (int A = rlo; A <= rhi; A += 4) {
                    const int tid = fresh_tid();
                    const int lane = tid & 63;
                    const int l16 = lane & 15, lg = lane >> 4;
                    const int C = A & 3;
                    // this wave's first tap fragments (both planes) of the band's
                    // phase, issued before the band is written and the barrier
                    const int row = min(l16, NJ);
                    gptr<h8> fh = tfr + ((size_t)(0 * 4 + C) * NFR + row) * (FRS / 8) + lg;
                    gptr<h8> fl = tfr + ((size_t)(1 * 4 + C) * NFR + row) * (FRS / 8) + lg;
                    h8 bh = fh[0], bl = fl[0];
                    // 3a. slot c's deposits in band rows A..A+3, scaled, as fp16
                    // hi + lo parts
                    {
                        const int o = mrb == kNone ? -8 : A - mrb + 3;
                        unsigned short *bs = reinterpret_cast<unsigned short *>(bandbuf);
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            *reinterpret_cast<unsigned long long *>(bs + ((0 * 4 + l) * RL + tid) * 4) =
                                band4(w0h[l], w1h[l], o);
                            *reinterpret_cast<unsigned long long *>(bs + ((1 * 4 + l) * RL + tid) * 4) =
                                band4(w0l[l], w1l[l], o);
                        }
                        // slots past the last column read as zeros
                        if (tid < RL - NCOL) {
                            const u4s z = {0, 0, 0, 0};
#pragma unroll
                            for (int pl = 0; pl < 8; ++pl)
                                *reinterpret_cast<u4s *>(bs + (pl * RL + NCOL + tid) * 4) = z;
                        }
                    }
                    __syncthreads();
                    // 3c. this wave's layer: out[i][j] for 4 blocks of 16 pixel
                    // columns.  Lane (lg, l16) reads k = (slot pair 4t + lg, rows
                    // 0..3): of block row i = l16 from the band (slots 4 i + 2 (4t
                    // + lg) .. +1), of output row j = l16 from the tap fragments
                    // of the band phase (loaded one k-step ahead).
                    f4 acc[4];
                    {
                        // this lane's band row: slot 4 l16 + 2 lg of layer wv, plane 0
                        const h8 *ap = reinterpret_cast<const h8 *>(bandbuf) +
                                       ((wv * RL + 4 * l16 + 2 * lg) >> 1);
#pragma unroll
                        for (int mb = 0; mb < 4; ++mb) acc[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int t = 0; t < NKS; ++t) {
                            h8 nh = bh, nl = bl;
                            if (t + 1 < NKS) {
                                nh = fh[4 * (t + 1)];
                                nl = fl[4 * (t + 1)];
                            }
#pragma unroll
                            for (int mb = 0; mb < 4; ++mb) {
                                // slots 64 mb + 8 t further on; plane 1 is 4 rows of RL later
                                const h8 ah = ap[32 * mb + 4 * t];
                                const h8 al = ap[32 * mb + 4 * t + 2 * RL];
                                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc[mb], 0, 0, 0);
                                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc[mb], 0, 0, 0);
                                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc[mb], 0, 0, 0);
                            }
                            bh = nh;
                            bl = nl;
                        }
                    }
                    __syncthreads();
                    // 3d. the layer partials, then a fixed-order FP64 sum per
                    // pixel into the tile (wave w adds column block w)
                    f4 *part = reinterpret_cast<f4 *>(bandbuf);
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb) part[(wv * 4 + mb) * 64 + lane] = acc[mb];
                    __syncthreads();
                    {
                        const f4 p0 = part[(0 * 4 + wv) * 64 + lane];
                        const f4 p1 = part[(1 * 4 + wv) * 64 + lane];
                        const f4 p2 = part[(2 * 4 + wv) * 64 + lane];
                        const f4 p3 = part[(3 * 4 + wv) * 64 + lane];
                        const int o = (A >> 2) + l16;  // output row
                        const int i0 = 16 * wv + 4 * lg;  // first of the lane's 4 pixel columns
                        if (l16 < NJ && o >= out_lo && o <= out_hi && i0 < TW) {
                            double *row = o < Y0 + TH ? &tile[o - Y0][i0] : &carry[o - Y0 - TH][i0];
                            d4 t = ld4(row);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                t[e] += ((((double)p0[e] + (double)p1[e]) + (double)p2[e]) +
                                         (double)p3[e]) * unsc;
                            st4(row, t);
                        }
                    }
                    // the next band is written over the partials: every wave must
                    // have read its own first (after the last band, the next write
                    // to this buffer follows the next pass's search barrier)
                    if (A + 4 <= rhi) __syncthreads();
                }
            }
        }
        __syncthreads();

        // ---- write the tile once
        for (int e = tid; e < TH * TQ; e += kTableThreads) {
            const int r = e / TQ, c = 4 * (e % TQ);
            put4(Y0 + r, X0 + c, ld4(&tile[r][c]));
        }
        // (no barrier: the next tile writes the tile array only after its
        // count barrier, which every wave reaches after this write-out)
        }  // tiles of the unit
    }
}

template <int KW, int DX, int DY>
hipError_t launch_kw(const FrameDev *frames_dev, int spec_f64, const int2 *work, int n_work,
                     int *counter, int *err, int nblocks, hipStream_t s)
{
    if (spec_f64)
        hipLaunchKernelGGL((k_render_table<KW, DX, DY, double>), dim3(nblocks),
                           dim3(kTableThreads), 0, s, frames_dev, work, n_work, counter, err);
    else
        hipLaunchKernelGGL((k_render_table<KW, DX, DY, float>), dim3(nblocks),
                           dim3(kTableThreads), 0, s, frames_dev, work, n_work, counter, err);
    return hipGetLastError();
}

template <int KW>
hipError_t launch_deg(const FrameDev *frames_dev, int degx, int degy, int spec_f64,
                      const int2 *work, int n_work, int *counter, int *err, int nblocks,
                      hipStream_t s)
{
    if (degx <= 4 && degy <= 3)
        return launch_kw<KW, 4, 3>(frames_dev, spec_f64, work, n_work, counter, err, nblocks, s);
    return launch_kw<KW, 7, 7>(frames_dev, spec_f64, work, n_work, counter, err, nblocks, s);
}

}  // namespace

hipError_t launch_table(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                        int n_work, int *counter, int *err, hipStream_t s)
{
    const int fit = 3;  // workgroups per CU the kernel's resources allow
    const int resident = cfg.resident > 0 && cfg.resident < fit ? cfg.resident : fit;
    const int cap = 256 * resident;
    int nblocks = work == nullptr ? cfg.plain_tiles : (n_work < cap ? n_work : cap);
    if (nblocks <= 0) return hipSuccess;
    if (cfg.kw == 32)
        return launch_deg<32>(frames_dev, cfg.degx, cfg.degy, cfg.spec_f64, work, n_work,
                              counter, err, nblocks, s);
    if (cfg.kw == 48)
        return launch_deg<48>(frames_dev, cfg.degx, cfg.degy, cfg.spec_f64, work, n_work,
                              counter, err, nblocks, s);
    return hipErrorInvalidValue;
}

}  // namespace e2e
