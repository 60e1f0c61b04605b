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
//   1. gives each thread one slot column and finds that column's samples by
//      a Newton search on the FP64 format polynomial;
//   2. walks those samples in order (FP64 positions, FP64 register sums of
//      the 16 deposits, flushed to the column's private 4-row LDS window);
//   3. per deposit row, densifies the slots and applies the node stencils,
//      one wave per node, taps read through the scalar cache, FP64 sums in a
//      rolling register window, then adds the four node partials into the
//      FP64 LDS tile in node order.
// The summation order is fixed, so reruns are bitwise identical.
#include "dev_common.h"

namespace e2e {

namespace {

constexpr int kNone = 0x3fffffff;  // "no row yet"; far from any real row

template <int KW, int DX, int DY, typename ST>
__global__ __launch_bounds__(kTableThreads, 2) void k_render_table(
    const FrameDev *__restrict__ frames, const int2 *__restrict__ work, int n_work,
    int *__restrict__ counter, int *__restrict__ err)
{
    constexpr int OS = kOS;
    constexpr int NCOL = kTableThreads;        // slot columns per tile
    constexpr int TW = (NCOL - KW) / OS;       // tile width in pixels
    constexpr int TH = kTableTH;
    constexpr int NSLOT = NCOL - 1;            // slots that reach the tile
    constexpr int NS = KW + OS - 1;            // slots per pixel column
    constexpr int DD = (KW + OS - 2) / OS + 1; // pixel rows per deposit row
    constexpr int NODE = OS * NS * DD;         // taps per node
    constexpr int SU = (NS % 5 == 0) ? 5 : ((NS % 3 == 0) ? 3 : 1);  // stencil unroll
    constexpr double UC = 0.5 * (OS - KW);
    static_assert(OS * TW + KW == NCOL, "tile geometry");
    static_assert(TW <= 64, "one wave spans the tile width");

    constexpr int NN = KW <= 32 ? 4 : 2;       // deposit rows per stencil chunk
    constexpr int NJ = NN + DD - 1;            // output rows a chunk reaches
    constexpr int SQ = (NS + 3) / 4;           // stencil columns per wave
    static_assert(NN * OS <= 16, "flag bits");

    __shared__ float W[4][2][4][NCOL];          // per-column deposit windows
    __shared__ int rbase[NCOL];                 // window base row per column
    __shared__ float D[NN][OS][OS][64];         // one layer, NN deposit rows, phase split
    __shared__ double tile[TH][TW];
    __shared__ double P[2][NJ][64];
    __shared__ int kst[NCOL + 1];
    __shared__ int tlist[kMaxTileTraces];
    __shared__ int flagw[2];
    __shared__ int sh_count, sh_item, sh_qmin, sh_qmax;
    __shared__ float sh_touch[kTableThreads];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int clane = lane < TW ? lane : TW - 1;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

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
        cptr<FrameDev> Fp = as_const(frames) + fi;
        const int ntr = Fp->ntr;
        const int tx = tile_id % Fp->ntx, ty = tile_id / Fp->ntx;
        const int X0 = tx * TW, Y0 = ty * TH;
        const SegDev *segs = Fp->segs + (size_t)tx * ntr;
        const double beta = Fp->beta, flux_scale = Fp->flux_scale, gsx = Fp->gsx, gsy = Fp->gsy;
        const int gxn = Fp->gx, gyn = Fp->gy;

        // ---- traces reaching this tile, ascending
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
        for (int e = tid; e < TH * TW; e += kTableThreads) tile[e / TW][e % TW] = 0.0;
        __syncthreads();
        const int count = uniform_i(sh_count);

        for (int li = 0; li < count; ++li) {
            const int tr = uniform_i(tlist[li]);
            cptr<TraceDev> Tp = as_const(Fp->tr) + tr;
            const SegDev sg = segs[tr];
            double cxr[DX + 1], cyr[DY + 1];
#pragma unroll
            for (int j = 0; j <= DX; ++j) cxr[j] = Tp->cx[j];
#pragma unroll
            for (int j = 0; j <= DY; ++j) cyr[j] = Tp->cy[j];
            TraceDev Tl;
            Tl.lmin = Tp->lmin;
            Tl.lmax = Tp->lmax;
            Tl.n = Tp->n;
            double t0, dt;
            trace_affine(Tl, beta, &t0, &dt);
            const double scale = Tp->thr * flux_scale;
            gptr<ST> spec = as_global((const ST *)as_const(Fp->spec)[Tp->slot]);
            const int k0 = sg.k0, k1 = sg.k1;
            const double ua = fma(horner<DX>(cxr, fma((double)k0, dt, t0)), (double)OS, UC);
            const double ub = fma(horner<DX>(cxr, fma((double)(k1 - 1), dt, t0)), (double)OS, UC);
            const double kspan = (double)(k1 - 1 - k0);
            const double inv_slope = ub > ua ? kspan / (ub - ua) : 0.0;  // samples per slot
            const bool multi = (sg.cx0 != sg.cx1) | (sg.cy0 != sg.cy1);
            // pull this item's spectrum into L2 while the column search runs
            float touch = 0.0f;
            for (int kk = k0 + 32 * tid; kk < k1; kk += 32 * kTableThreads)
                touch += (float)spec_at(spec, kk);

            for (int cyc = sg.cy0; cyc <= sg.cy1; ++cyc)
            for (int cxc = sg.cx0; cxc <= sg.cx1; ++cxc) {
                // ---- 1. samples of each slot column: first k with u(k) >= q
                const int q = OS * X0 - KW + tid;
                auto u_of = [&](int k) {
                    double x = horner<DX>(cxr, fma((double)k, dt, t0));
                    return fma(x, (double)OS, UC);
                };
                auto search = [&](int qq) -> int {
                    if ((double)qq <= ua) return k0;
                    if ((double)qq > ub) return k1;
                    // secant steps on the (nearly linear) slot index, then exact fix-up
                    double kk = (double)k0 + ((double)qq - ua) * inv_slope;
                    for (int it = 0; it < 2; ++it) {
                        kk = fmin(fmax(kk, (double)k0), (double)(k1 - 1));
                        kk -= (u_of((int)kk) - (double)qq) * inv_slope;
                    }
                    int k = (int)ceil(fmin(fmax(kk, (double)k0), (double)(k1 - 1)));
                    k = min(max(k, k0 + 1), k1 - 1);
                    int guard = 0;
                    while (k < k1 && u_of(k) < (double)qq && guard < 256) { ++k; ++guard; }
                    while (k > k0 && u_of(k - 1) >= (double)qq && guard < 256) { --k; ++guard; }
                    if (guard >= 256) atomicOr(err, kErrSearch);
                    return k;
                };
                kst[tid] = search(q);
                if (tid == NCOL - 1) kst[NCOL] = search(q + 1);
                if (tid == 0) { sh_qmin = 0x7fffffff; sh_qmax = -0x7fffffff; }
#pragma unroll
                for (int l = 0; l < 4; ++l)
#pragma unroll
                    for (int lr = 0; lr < 2; ++lr)
#pragma unroll
                        for (int r = 0; r < 4; ++r) W[l][lr][r][tid] = 0.0f;
                if (tid < 2) flagw[tid] = 0;
                __syncthreads();

                // ---- 2. this column's samples, in order.  Within one row run the
                // 16 deposits (2 x-slots x 2 rows x 4 nodes) are polynomials of
                // degree <= 2 in the sub-slot phases (rx, ry), because the CIC
                // weights and the node weights are both affine in them; so the
                // run keeps the 9 moments sum phi rx^a ry^b (FP64) and turns
                // them into deposits when the row changes.
                const int ks = kst[tid], ke = kst[tid + 1];
                int nbx, nby;
                double ax0, ax1, ay0, ay1;
                cell_line(cxc, gsx, gxn, &nbx, &ax0, &ax1);
                cell_line(cyc, gsy, gyn, &nby, &ay0, &ay1);
                // fx = ax0 + ax1 * x with x = (q + rx - UC) / OS
                const double fxa = fma(ax1, ((double)q - UC) / OS, ax0), fxb = ax1 / OS;
                const double fyb = ay1 / OS;
                double m[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) m[a][b] = 0.0;
                int runQy = kNone, rb = kNone;
                bool run_in = false;
                int qmin = 0x7fffffff, qmax = -0x7fffffff;
                auto flush = [&]() {
                    int o = runQy - rb;
                    if (o < 0 || o > 2) {
                        atomicOr(err, kErrRowWindow);
                        return;
                    }
                    if (run_in) {
                        qmin = min(qmin, runQy);
                        qmax = max(qmax, runQy);
                    }
                    const double fya = fma(ay1, ((double)runQy - UC) / OS, ay0);
                    // polynomial coefficients (in rho) of cic x node weight
                    double X[2][2][3], Y[2][2][3];
                    auto coef = [](double a, double b, double c[2][2][3]) {
                        c[0][1][0] = a;       c[0][1][1] = b - a;       c[0][1][2] = -b;
                        c[0][0][0] = 1.0 - a; c[0][0][1] = a - 1.0 - b; c[0][0][2] = b;
                        c[1][1][0] = 0.0;     c[1][1][1] = a;           c[1][1][2] = b;
                        c[1][0][0] = 0.0;     c[1][0][1] = 1.0 - a;     c[1][0][2] = -b;
                    };
                    coef(fxa, fxb, X);
                    coef(fya, fyb, Y);
                    double Tm[2][2][3];
#pragma unroll
                    for (int r = 0; r < 2; ++r)
#pragma unroll
                        for (int ny = 0; ny < 2; ++ny)
#pragma unroll
                            for (int a = 0; a < 3; ++a)
                                Tm[r][ny][a] = fma(Y[r][ny][2], m[a][2],
                                                   fma(Y[r][ny][1], m[a][1], Y[r][ny][0] * m[a][0]));
#pragma unroll
                    for (int l = 0; l < 4; ++l)
#pragma unroll
                        for (int lr = 0; lr < 2; ++lr)
#pragma unroll
                            for (int r = 0; r < 2; ++r) {
                                const int nx = l & 1, ny = l >> 1;
                                double d = fma(X[lr][nx][2], Tm[r][ny][2],
                                               fma(X[lr][nx][1], Tm[r][ny][1],
                                                   X[lr][nx][0] * Tm[r][ny][0]));
                                W[l][lr][o + r][tid] += (float)(d * scale);
                            }
                };
                double sv_next = ks < ke ? spec_at(spec, ks) : 0.0;
                const double UCq = UC - (double)q;
                for (int k = ks; k < ke; ++k) {
                    double sv = sv_next;
                    if (k + 1 < ke) sv_next = spec_at(spec, k + 1);
                    double t = fma((double)k, dt, t0);
                    double x = horner<DX>(cxr, t);
                    double y = horner<DY>(cyr, t);
                    double rx = fma(x, (double)OS, UCq);
                    double vy = fma(y, (double)OS, UC);
                    double fly = floor(vy);
                    int Qy = (int)fly;
                    double ry = vy - fly;
                    bool in = true;
                    if (multi) in = (ext_cell(x, gsx, gxn) == cxc) & (ext_cell(y, gsy, gyn) == cyc);
                    double phi = in ? sv : 0.0;
                    if (Qy != runQy) {
                        if (runQy != kNone) {
                            flush();
#pragma unroll
                            for (int a = 0; a < 3; ++a)
#pragma unroll
                                for (int b = 0; b < 3; ++b) m[a][b] = 0.0;
                        }
                        if (rb == kNone) rb = Qy - 1;
                        runQy = Qy;
                        run_in = false;
                    }
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
                }
                if (runQy != kNone) flush();
                rbase[tid] = rb;
                sh_touch[tid] = touch;
                if (qmin <= qmax) {
                    atomicMin(&sh_qmin, qmin);
                    atomicMax(&sh_qmax, qmax);
                }
                __syncthreads();

                // ---- 3. stencils: chunks of NN deposit rows; per node layer the
                // slots are densified, then each wave applies the taps of its
                // quarter of the slot offsets to all NN rows (one scalar tap
                // load feeds NN x DD FMAs); the four partial sums are added
                // into the FP64 tile in a fixed order.
                const int qlo = uniform_i(sh_qmin), qhi = uniform_i(sh_qmax) + 1;
                if (qlo > qhi) continue;  // no sample of this cell here (uniform)
                const int nlo = floordiv(qlo, OS), nhi = floordiv(qhi, OS);
                const int nb = max(nlo, Y0 - (DD - 1));
                const int ne = min(nhi, Y0 + TH - 1);
                if (nb > ne) continue;
                for (int nc = nb; nc <= ne; nc += NN) {
                    double acc[NJ];
#pragma unroll
                    for (int d = 0; d < NJ; ++d) acc[d] = 0.0;
                    for (int L = 0; L < 4; ++L) {
                        if (tid < NSLOT) {
                            const int sgm = tid;
                            const int rL = rbase[sgm + 1], rR = rbase[sgm];
                            int bits = 0;
#pragma unroll
                            for (int nn = 0; nn < NN; ++nn)
#pragma unroll
                                for (int p = 0; p < OS; ++p) {
                                    const int r = OS * (nc + nn) + p;
                                    const int oL = r - rL, oR = r - rR;
                                    float vL = (unsigned)oL < 4u ? W[L][0][oL & 3][sgm + 1] : 0.0f;
                                    float vR = (unsigned)oR < 4u ? W[L][1][oR & 3][sgm] : 0.0f;
                                    float d = vL + vR;
                                    D[nn][p][sgm & 3][sgm >> 2] = d;
                                    bits |= (d != 0.0f) ? (1 << (nn * OS + p)) : 0;
                                }
                            if (bits) atomicOr(&flagw[L & 1], bits);
                        }
                        __syncthreads();
                        const int fw = uniform_i(flagw[L & 1]);
                        if (tid == 0) flagw[(L + 1) & 1] = 0;
                        if (fw) {
                            const int mx = min(nbx + (L & 1), gxn - 1);
                            const int my = min(nby + (L >> 1), gyn - 1);
                            cptr<double> taps = as_const(Fp->tb) + (size_t)(my * gxn + mx) * NODE;
#pragma unroll
                            for (int p = 0; p < OS; ++p) {
                                int pm = 0;
#pragma unroll
                                for (int nn = 0; nn < NN; ++nn) pm |= (fw >> (nn * OS + p)) & 1;
                                if (!pm) continue;
                                for (int ss = 0; ss < SQ; ++ss) {
                                    const int s = wv * SQ + ss;
                                    if (s >= NS) break;
                                    cptr<double> tp = taps + (p * NS + s) * DD;
                                    double tv[DD];
#pragma unroll
                                    for (int dd = 0; dd < DD; ++dd) tv[dd] = tp[dd];
#pragma unroll
                                    for (int nn = 0; nn < NN; ++nn) {
                                        if (!((fw >> (nn * OS + p)) & 1)) continue;
                                        double d = (double)D[nn][p][s & 3][clane + (s >> 2)];
#pragma unroll
                                        for (int dd = 0; dd < DD; ++dd) {
                                            if (p == 0 && dd == DD - 1) continue;  // zero tap row
                                            acc[nn + dd] = fma(d, tv[dd], acc[nn + dd]);
                                        }
                                    }
                                }
                            }
                        }
                        __syncthreads();
                    }
                    // fixed-order sum of the four partials: (w0 + w2) + (w1 + w3)
                    if (wv >= 2) {
#pragma unroll
                        for (int d = 0; d < NJ; ++d) P[wv - 2][d][lane] = acc[d];
                    }
                    __syncthreads();
                    if (wv < 2) {
#pragma unroll
                        for (int d = 0; d < NJ; ++d) acc[d] += P[wv][d][lane];
                    }
                    __syncthreads();
                    if (wv == 1) {
#pragma unroll
                        for (int d = 0; d < NJ; ++d) P[0][d][lane] = acc[d];
                    }
                    __syncthreads();
                    if (wv == 0 && lane < TW) {
#pragma unroll
                        for (int d = 0; d < NJ; ++d) {
                            const int j = nc + d - Y0;
                            if (j >= 0 && j < TH) tile[j][lane] += acc[d] + P[0][d][lane];
                        }
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();

        // ---- write the tile once
        for (int e = tid; e < TH * TW; e += kTableThreads) {
            int r = e / TW, c = e % TW;
            int gx = X0 + c, gy = Y0 + r;
            if (gx < Fp->nx && gy < Fp->ny) {
                size_t o = (size_t)gy * Fp->nx + gx;
                if (Fp->out_f64) ((double *)Fp->out)[o] = tile[r][c];
                else ((float *)Fp->out)[o] = (float)tile[r][c];
            }
        }
        __syncthreads();
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
    int nblocks = work == nullptr ? cfg.plain_tiles : (n_work < 512 ? n_work : 512);
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
