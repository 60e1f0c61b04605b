// Host runtime of the C ABI declared in include/e2e.h: context, validation
// of the spectral-format / PSF database (Genoni et al. 2020, Sec. 2.1),
// device-resident tables, render and batch dispatch, kernel timing.  The
// serve loop lives in serve.cpp.
#include "api_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace e2e;

static thread_local std::string g_err;

e2e_status e2e::fail(e2e_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

e2e_status e2e::hip_fail(hipError_t e, const char *what)
{
    return fail(E2E_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *e2e_last_error(void) { return g_err.c_str(); }
extern "C" const char *e2e_version(void) { return "e2e-mi355x 0.1 (gfx950)"; }

double e2e::now_us(const e2e_ctx *ctx)
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - ctx->t0)
        .count();
}

// ------------------------------------------------------------------ context

// The allocation-free render's device memory (e2e_render_noalloc): each
// device holds its own copy for the life of the process.  Host code must use
// the address hipGetSymbolAddress returns on that device, never this name.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

extern "C" e2e_status e2e_create(e2e_ctx **out, int32_t dev, uint64_t budget)
{
    if (!out) return fail(E2E_EINVAL, "e2e_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (dev < 0 || dev >= ndev)
        return fail(E2E_EINVAL, "e2e_create: device %d not in [0, %d)", dev, ndev);
    if ((e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    size_t freeb = 0, totb = 0;
    if ((e = hipMemGetInfo(&freeb, &totb)) != hipSuccess) return hip_fail(e, "hipMemGetInfo");
    auto *c = new e2e_ctx();
    c->dev = dev;
    c->budget = budget ? budget : (uint64_t)(0.9 * (double)freeb);
    c->t0 = std::chrono::steady_clock::now();
    const char *g = getenv("E2E_GRAPHS");
    c->graphs = !(g && g[0] == '0');
    if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipStreamCreate");
    }
    // this device's copy of the allocation-free render's array (dev is current)
    if ((e = hipGetSymbolAddress((void **)&c->noalloc.base, HIP_SYMBOL(scratch))) != hipSuccess) {
        hipStreamDestroy(c->stream);
        delete c;
        return hip_fail(e, "hipGetSymbolAddress(scratch)");
    }
    *out = c;
    return E2E_OK;
}

static void free_scratch(Scratch *s)
{
    if (!s) return;
    hipFree(s->frames_dev);
    hipFree(s->segs);
    hipFree(s->work);
    hipFree(s->specptrs);
    hipFree(s->err);
    hipFree(s->counter);
    if (s->err_host) hipHostFree(s->err_host);
    if (s->stage) hipHostFree(s->stage);
    if (s->staged) hipEventDestroy(s->staged);
    for (void *p : s->temps) hipFree(p);
    for (auto &g : s->graphs) {
        hipGraphExecDestroy(g.second.exec);
        hipGraphDestroy(g.second.graph);
    }
    delete s;
}

extern "C" void e2e_destroy(e2e_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->dev);
    e2e_serve_stop(ctx);
    hipDeviceSynchronize();
    for (auto &kv : ctx->fmts) {
        hipFree(kv.second->dev);
        delete kv.second;
    }
    for (auto &kv : ctx->psfs) {
        hipFree(kv.second->tfrag);
        hipFree(kv.second->sxy);
        delete kv.second;
    }
    for (auto &kv : ctx->scratch) free_scratch(kv.second);
    for (auto &p : ctx->prof_pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    hipStreamDestroy(ctx->stream);
    delete ctx;
}

// ------------------------------------------------------------ format load

static double poly(const double *c, int deg, double t)
{
    double v = c[deg];
    for (int j = deg - 1; j >= 0; --j) v = v * t + c[j];
    return v;
}

static double dpoly(const double *c, int deg, double t, int order)
{
    // derivative of given order, evaluated directly
    double v = 0.0;
    for (int j = deg; j >= order; --j) {
        double f = 1.0;
        for (int q = 0; q < order; ++q) f *= (double)(j - q);
        v = v * t + c[j] * f;
    }
    return v;
}

extern "C" e2e_status e2e_format_load(e2e_ctx *ctx, const e2e_trace_desc *tr, int32_t n,
                                      int32_t nx, int32_t ny, e2e_format_id *out)
{
    if (!ctx || !tr || !out) return fail(E2E_EINVAL, "e2e_format_load: NULL argument");
    if (n < 1 || n > (1 << 20)) return fail(E2E_EINVAL, "e2e_format_load: n_traces=%d", n);
    if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536)
        return fail(E2E_EINVAL, "e2e_format_load: detector %dx%d", nx, ny);
    std::vector<TraceDev> h(n);
    int dxm = 0, dym = 0, nslots = 0;
    const int NG = 4097;
    for (int i = 0; i < n; ++i) {
        const e2e_trace_desc &d = tr[i];
        if (d.deg_x < 1 || d.deg_x > 7 || d.deg_y < 0 || d.deg_y > 7)
            return fail(E2E_EFORMAT, "trace %d: degrees (%d, %d) outside x 1..7, y 0..7", i,
                        d.deg_x, d.deg_y);
        if (!d.cx || !d.cy) return fail(E2E_EINVAL, "trace %d: NULL coefficients", i);
        if (!(std::isfinite(d.lambda_min_nm) && std::isfinite(d.lambda_max_nm) &&
              d.lambda_min_nm > 0 && d.lambda_min_nm < d.lambda_max_nm))
            return fail(E2E_EFORMAT, "trace %d: need 0 < lambda_min < lambda_max", i);
        if (d.n_samples < 1 || d.n_samples > 0x7ffffffe)
            return fail(E2E_EINVAL, "trace %d: n_samples=%lld", i, (long long)d.n_samples);
        if (!(std::isfinite(d.throughput) && d.throughput >= 0))
            return fail(E2E_EINVAL, "trace %d: throughput must be finite and >= 0", i);
        if (d.spectrum_slot < 0 || d.spectrum_slot >= (1 << 20))
            return fail(E2E_EINVAL, "trace %d: spectrum_slot=%d", i, d.spectrum_slot);
        TraceDev &T = h[i];
        memset(&T, 0, sizeof T);
        for (int j = 0; j <= d.deg_x; ++j) {
            if (!std::isfinite(d.cx[j])) return fail(E2E_EFORMAT, "trace %d: cx not finite", i);
            T.cx[j] = d.cx[j];
        }
        for (int j = 0; j <= d.deg_y; ++j) {
            if (!std::isfinite(d.cy[j])) return fail(E2E_EFORMAT, "trace %d: cy not finite", i);
            T.cy[j] = d.cy[j];
        }
        T.lmin = d.lambda_min_nm;
        T.lmax = d.lambda_max_nm;
        T.thr = d.throughput;
        T.n = (int32_t)d.n_samples;
        T.degx = d.deg_x;
        T.degy = d.deg_y;
        T.slot = d.spectrum_slot;
        // x strictly increasing and |dy/dx| <= 0.5 over t in [-1.001, 1.001]
        // (the Doppler range); grid minima corrected by the second derivative
        double h_t = 2.002 / (NG - 1), minx1 = 1e300, maxx2 = 0, maxslope = 0, maxy2 = 0,
               maxy1 = 0;
        for (int g = 0; g < NG; ++g) {
            double t = -1.001 + h_t * g;
            double x1 = dpoly(T.cx, T.degx, t, 1);
            double x2 = fabs(dpoly(T.cx, T.degx, t, 2));
            double y1 = fabs(dpoly(T.cy, T.degy, t, 1));
            double y2 = fabs(dpoly(T.cy, T.degy, t, 2));
            minx1 = std::min(minx1, x1);
            maxx2 = std::max(maxx2, x2);
            maxy2 = std::max(maxy2, y2);
            maxy1 = std::max(maxy1, y1);
            if (x1 > 0) maxslope = std::max(maxslope, y1 / x1);
        }
        double xlow = minx1 - maxx2 * h_t / 2;
        if (!(xlow > 0))
            return fail(E2E_EFORMAT, "trace %d: x(lambda) is not strictly increasing", i);
        if (xlow * 2.0 / (double)T.n < 1e-9)
            return fail(E2E_EFORMAT, "trace %d: samples closer than 1e-9 px", i);
        double slope_hi = (maxy1 + maxy2 * h_t / 2) / xlow;
        if (maxslope > 0.5 || slope_hi > 0.5 + 1e-3)
            return fail(E2E_EFORMAT, "trace %d: |dy/dx| up to %.3g exceeds 0.5", i,
                        std::max(maxslope, slope_hi));
        // |y''| bound for the planner (grid max plus third-derivative slack)
        double y3 = 0;
        for (int g = 0; g < NG; ++g)
            y3 = std::max(y3, fabs(dpoly(T.cy, T.degy, -1.001 + h_t * g, 3)));
        T.y2max = maxy2 + y3 * h_t + 1e-9;
        dxm = std::max(dxm, T.degx);
        dym = std::max(dym, T.degy);
        nslots = std::max(nslots, T.slot + 1);
    }
    hipSetDevice(ctx->dev);
    size_t bytes = sizeof(TraceDev) * n;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->used + bytes > ctx->budget)
        return fail(E2E_ENOMEM, "e2e_format_load: %zu bytes exceed the HBM budget", bytes);
    auto *F = new FormatRes();
    F->nx = nx;
    F->ny = ny;
    F->ntr = n;
    F->nslots = nslots;
    F->degx = dxm;
    F->degy = dym;
    F->host = h;
    F->bytes = bytes;
    hipError_t e = hipMalloc(&F->dev, bytes);
    if (e == hipSuccess) e = hipMemcpy(F->dev, h.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(F->dev);
        delete F;
        return hip_fail(e, "e2e_format_load");
    }
    ctx->used += bytes;
    uint64_t id = ctx->next_id++;
    ctx->fmts[id] = F;
    *out = id;
    return E2E_OK;
}

// --------------------------------------------------------------- PSF load

// Taps of one node: B(vy, vx) = sum of the table over the os x os cells
// starting at (vx, vy) (cells outside the table are zero), stored as
// tb[s][p][dd] = B(os dd - p, kw - 1 - s): the taps of one slot offset s are
// contiguous, which is the order the stencil streams them in.  The sums are
// exact in FP64; the device copy is rounded once to FP32 (the pixel
// integrals of the PSF run in FP32, positions in FP64).
static void node_taps(const float *K, int kw, double *tb)
{
    const int OS = kOS, NS = kw + OS - 1, DD = (kw + OS - 2) / OS + 1;
    auto box = [&](int vy, int vx) {
        int y0 = std::max(vy, 0), y1 = std::min(vy + OS, kw);
        int x0 = std::max(vx, 0), x1 = std::min(vx + OS, kw);
        if (y0 >= y1 || x0 >= x1) return 0.0;
        // direct sum (exact in FP64 for float inputs)
        double s = 0.0;
        for (int b = y0; b < y1; ++b)
            for (int a = x0; a < x1; ++a) s += (double)K[(size_t)b * kw + a];
        return s;
    };
    for (int s = 0; s < NS; ++s)
        for (int p = 0; p < OS; ++p)
            for (int dd = 0; dd < DD; ++dd)
                tb[((size_t)s * OS + p) * DD + dd] = box(OS * dd - p, kw - 1 - s);
}

// The stencil of one node over a band of 4 deposit rows starting at phase C
// (rows C .. C + 3 of a 4-row pixel period) is the matrix
//   T_C[k = (s, r)][j] = tb[s][(C + r) mod 4][j - floor((C + r) / 4)]
// (zero outside 0 <= that row offset < DD and for padded s).  Stored per
// output row j as the fragments v_mfma_f32_16x16x32_f16 reads (eight
// consecutive k = two slot offsets x four band rows), scaled by 2^kTapShift
// and split into fp16 hi + lo parts (the FP64 tap to about 2^-22 relative).
static void node_frags(const double *tb, int kw, uint16_t *out)
{
    const int NS = kw + kOS - 1, DD = table_dd(kw), NJ = DD + 1;
    const int NFR = table_frag_rows(kw), SP = table_slots_padded(kw), FRS = table_frag_row(kw);
    for (int C = 0; C < 4; ++C)
        for (int j = 0; j < NFR; ++j)
            for (int s = 0; s < SP; ++s)
                for (int r = 0; r < 4; ++r) {
                    double v = 0.0;
                    const int w = C + r, dd = j - (w >> 2);
                    if (j < NJ && s < NS && dd >= 0 && dd < DD)
                        v = std::ldexp(tb[((size_t)s * kOS + (w & 3)) * DD + dd], kTapShift);
                    const _Float16 hi = (_Float16)v;
                    const _Float16 lo = (_Float16)(v - (double)hi);
                    const size_t o = ((size_t)C * NFR + j) * FRS + (size_t)s * 4 + r;
                    out[o] = __builtin_bit_cast(uint16_t, hi);
                    out[(size_t)4 * NFR * FRS + o] = __builtin_bit_cast(uint16_t, lo);
                }
}

// Gauss-Legendre rule of n points on [-1, 1]: Newton's method on P_n from
// the asymptotic guesses cos(pi (4i - 1) / (4n + 2)), P_n and P_n' by the
// three-term recurrence; weights 2 / ((1 - x^2) P_n'(x)^2).
static void legendre_rule(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 1; i <= n; ++i) {
        double z = std::cos(M_PI * (4.0 * i - 1.0) / (4.0 * n + 2.0)), d = 1.0;
        for (int it = 0; it < 64; ++it) {
            double pm = 1.0, pc = z;
            for (int k = 2; k <= n; ++k) {
                const double pn = ((2 * k - 1) * z * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pn;
            }
            d = n * (pm - z * pc) / (1.0 - z * z);
            const double step = pc / d;
            z -= step;
            if (std::fabs(step) <= 1e-16) break;
        }
        x[i - 1] = z;
        w[i - 1] = 2.0 / ((1.0 - z * z) * d * d);
    }
}

extern "C" e2e_status e2e_psf_load(e2e_ctx *ctx, const e2e_psf_desc *d, e2e_psf_id *out)
{
    if (!ctx || !d || !out) return fail(E2E_EINVAL, "e2e_psf_load: NULL argument");
    auto *P = new PsfRes();
    P->kind = d->kind;
    P->sigma = d->sigma;
    P->H = d->half_width;
    P->gx = d->grid_nx;
    P->gy = d->grid_ny;
    P->kw = d->kw;
    P->kh = d->kh;
    P->os = d->oversample;
    std::vector<double> tb;
    std::vector<uint16_t> frag;
    std::vector<float> sxy, sfq;
    auto bad = [&](e2e_status c, const char *m) {
        delete P;
        return fail(c, "e2e_psf_load: %s", m);
    };
    if (d->kind == E2E_PSF_GAUSS_ERF) {
        if (!(std::isfinite(d->sigma) && d->sigma > 0)) return bad(E2E_EPSF, "sigma must be > 0");
        if (d->half_width < 1 || d->half_width > 8) return bad(E2E_EPSF, "half_width outside 1..8");
        P->gx = P->gy = 1;
    } else if (d->kind == E2E_PSF_SEPARABLE) {
        if (d->half_width < 1 || d->half_width > 8) return bad(E2E_EPSF, "half_width outside 1..8");
        if (d->grid_nx < 1 || d->grid_ny < 1 || d->grid_nx > 127 || d->grid_ny > 127)
            return bad(E2E_EPSF, "grid outside 1..127");
        if (!d->sigma_xy) return bad(E2E_EINVAL, "sigma_xy is NULL");
        size_t nn = (size_t)d->grid_nx * d->grid_ny * 2;
        sxy.assign(d->sigma_xy, d->sigma_xy + nn);
        for (float v : sxy)
            if (!(std::isfinite(v) && v > 0)) return bad(E2E_EPSF, "sigma_xy must be > 0");
    } else if (d->kind == E2E_PSF_SFI) {
        if (d->half_width < 1 || d->half_width > kSfiMaxH)
            return bad(E2E_EPSF, "half_width outside 1..7");
        if (d->subpixels < 1 || d->subpixels > 16) return bad(E2E_EPSF, "subpixels outside 1..16");
        if (d->fiber_shape < E2E_FIBER_DISC || d->fiber_shape > E2E_FIBER_HALF_DOWN)
            return bad(E2E_EPSF, "unknown fiber shape");
        if (d->grid_nx < 1 || d->grid_ny < 1 || d->grid_nx > 127 || d->grid_ny > 127)
            return bad(E2E_EPSF, "grid outside 1..127");
        if (!d->sigma_xy) return bad(E2E_EINVAL, "sigma_xy is NULL");
        size_t nn = (size_t)d->grid_nx * d->grid_ny * 2;
        sxy.assign(d->sigma_xy, d->sigma_xy + nn);
        float smin = 1e30f;
        for (float v : sxy) {
            if (!(std::isfinite(v) && v > 0)) return bad(E2E_EPSF, "sigma_xy must be > 0");
            smin = std::min(smin, v);
        }
        const double rho = d->fiber_radius;
        if (!(std::isfinite(rho) && rho > 0)) return bad(E2E_EPSF, "fiber_radius must be > 0");
        const double r = rho / smin;
        if (r > 4.0) return bad(E2E_EPSF, "fiber_radius / min(sigma) exceeds 4");
        // Gauss-Legendre points over the fiber's chord angle: enough for
        // rounding-level agreement with the converged integral up to
        // rho / sigma = 4; an even count pairs th with -th, which share
        // the chord half-length, so only the positive half is kept
        int Q = 2 * (int)std::ceil((8.0 + 5.0 * r) / 2.0);
        Q = std::min(2 * kSfiMaxR, std::max(12, Q));
        std::vector<double> gx, gw;
        legendre_rule(Q, gx, gw);
        for (int q = 0; q < Q; ++q) {
            if (gx[q] <= 0.0) continue;
            const double th = 0.5 * M_PI * gx[q];
            sfq.push_back((float)(rho * std::sin(th)));
            sfq.push_back((float)(rho * std::cos(th)));
            sfq.push_back((float)(gw[q] * std::cos(th)));
        }
        P->sfi_R = (int)sfq.size() / 3;
        P->sfi_S = d->subpixels;
        P->sfi_shape = d->fiber_shape;
        P->rho = rho;
    } else if (d->kind == E2E_PSF_TABLE) {
        if (d->grid_nx < 1 || d->grid_ny < 1 || d->grid_nx > 127 || d->grid_ny > 127)
            return bad(E2E_EPSF, "grid outside 1..127");
        if (!d->tables) return bad(E2E_EINVAL, "tables is NULL");
        if (d->kw < 1 || d->kh < 1 || d->oversample < 1) return bad(E2E_EPSF, "bad table shape");
        if (d->oversample != kOS || d->kw != d->kh || (d->kw != 32 && d->kw != 48))
            return bad(E2E_EUNSUPPORTED, "GPU path needs oversample 4 and kw = kh in {32, 48}");
        size_t ksz = (size_t)d->kw * d->kh, nodes = (size_t)d->grid_nx * d->grid_ny;
        const int NS = d->kw + kOS - 1, DD = (d->kw + kOS - 2) / kOS + 1;
        size_t node = (size_t)kOS * NS * DD;
        tb.resize(node);
        frag.resize((size_t)table_frag_node(d->kw) * nodes);
        for (size_t q = 0; q < nodes; ++q) {
            const float *K = d->tables + q * ksz;
            double s = 0;
            for (size_t e = 0; e < ksz; ++e) {
                if (!std::isfinite(K[e])) return bad(E2E_EPSF, "table value not finite");
                s += K[e];
            }
            if (fabs(s - 1.0) > 1e-5) {
                delete P;
                return fail(E2E_EPSF, "e2e_psf_load: node %zu sums to %.9g, not 1", q, s);
            }
            node_taps(K, d->kw, tb.data());
            node_frags(tb.data(), d->kw, frag.data() + q * table_frag_node(d->kw));
        }
    } else {
        return bad(E2E_EINVAL, "unknown PSF kind");
    }
    hipSetDevice(ctx->dev);
    size_t bytes = frag.size() * sizeof(uint16_t) + (sxy.size() + sfq.size()) * sizeof(float);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->used + bytes > ctx->budget) return bad(E2E_ENOMEM, "tables exceed the HBM budget");
    hipError_t e = hipSuccess;
    if (!frag.empty()) {
        e = hipMalloc(&P->tfrag, frag.size() * sizeof(uint16_t));
        if (e == hipSuccess)
            e = hipMemcpy(P->tfrag, frag.data(), frag.size() * sizeof(uint16_t),
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !sxy.empty()) {
        e = hipMalloc(&P->sxy, sxy.size() * sizeof(float));
        if (e == hipSuccess)
            e = hipMemcpy(P->sxy, sxy.data(), sxy.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !sfq.empty()) {
        e = hipMalloc(&P->sfq, sfq.size() * sizeof(float));
        if (e == hipSuccess)
            e = hipMemcpy(P->sfq, sfq.data(), sfq.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        hipFree(P->tfrag);
        hipFree(P->sxy);
        hipFree(P->sfq);
        delete P;
        return hip_fail(e, "e2e_psf_load");
    }
    P->bytes = bytes;
    ctx->used += bytes;
    uint64_t id = ctx->next_id++;
    ctx->psfs[id] = P;
    *out = id;
    return E2E_OK;
}

extern "C" e2e_status e2e_format_free(e2e_ctx *ctx, e2e_format_id id)
{
    if (!ctx) return fail(E2E_EINVAL, "e2e_format_free: NULL context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->fmts.find(id);
    if (it == ctx->fmts.end()) return fail(E2E_ENOTFOUND, "format %llu not found",
                                           (unsigned long long)id);
    if (it->second->refs > 0) return fail(E2E_EBUSY, "format %llu in use", (unsigned long long)id);
    hipSetDevice(ctx->dev);
    hipDeviceSynchronize();
    hipFree(it->second->dev);
    ctx->used -= it->second->bytes;
    delete it->second;
    ctx->fmts.erase(it);
    return E2E_OK;
}

extern "C" e2e_status e2e_psf_free(e2e_ctx *ctx, e2e_psf_id id)
{
    if (!ctx) return fail(E2E_EINVAL, "e2e_psf_free: NULL context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->psfs.find(id);
    if (it == ctx->psfs.end()) return fail(E2E_ENOTFOUND, "psf %llu not found",
                                           (unsigned long long)id);
    if (it->second->refs > 0) return fail(E2E_EBUSY, "psf %llu in use", (unsigned long long)id);
    hipSetDevice(ctx->dev);
    hipDeviceSynchronize();
    hipFree(it->second->tfrag);
    hipFree(it->second->sxy);
    hipFree(it->second->sfq);
    ctx->used -= it->second->bytes;
    delete it->second;
    ctx->psfs.erase(it);
    return E2E_OK;
}

// ------------------------------------------------------------ render core

static e2e_status grow(void **p, size_t *cap, size_t need, const char *what)
{
    if (*cap >= need) return E2E_OK;
    size_t n = std::max(need, *cap * 2);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, n);
    if (e != hipSuccess) return hip_fail(e, what);
    hipFree(*p);
    *p = q;
    *cap = n;
    return E2E_OK;
}

Scratch *e2e::scratch_for(e2e_ctx *ctx, hipStream_t s)
{
    auto it = ctx->scratch.find(s);
    if (it != ctx->scratch.end()) return it->second;
    auto *sc = new Scratch();
    if (hipMalloc(&sc->err, sizeof(int)) != hipSuccess ||
        hipMalloc(&sc->counter, sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&sc->err_host, sizeof(int)) != hipSuccess ||
        launch_fill_i32(sc->err, 1, 0, s) != hipSuccess) {
        free_scratch(sc);
        return nullptr;
    }
    *sc->err_host = 0;
    ctx->scratch[s] = sc;
    return sc;
}

e2e_status e2e::validate_req(e2e_ctx *ctx, const e2e_render_req *r, FormatRes **pf,
                             PsfRes **pp)
{
    if (!r) return fail(E2E_EINVAL, "request is NULL");
    auto fi = ctx->fmts.find(r->fmt);
    if (fi == ctx->fmts.end())
        return fail(E2E_ENOTFOUND, "format %llu not found", (unsigned long long)r->fmt);
    auto pi = ctx->psfs.find(r->psf);
    if (pi == ctx->psfs.end())
        return fail(E2E_ENOTFOUND, "psf %llu not found", (unsigned long long)r->psf);
    FormatRes *F = fi->second;
    PsfRes *P = pi->second;
    if (!r->spectra) return fail(E2E_EINVAL, "spectra is NULL");
    if (r->n_spectra < F->nslots)
        return fail(E2E_EINVAL, "n_spectra=%d but the format uses %d slots", r->n_spectra,
                    F->nslots);
    for (int s = 0; s < F->nslots; ++s)
        if (!r->spectra[s]) return fail(E2E_EINVAL, "spectra[%d] is NULL", s);
    if (r->spectrum_dtype != E2E_F32 && r->spectrum_dtype != E2E_F64)
        return fail(E2E_EINVAL, "spectrum_dtype=%d", r->spectrum_dtype);
    if (r->out_dtype != E2E_F32 && r->out_dtype != E2E_F64)
        return fail(E2E_EINVAL, "out_dtype=%d", r->out_dtype);
    if (!r->out) return fail(E2E_EINVAL, "out is NULL");
    if (!(std::isfinite(r->rv_mps) && fabs(r->rv_mps) <= 1.5e5))
        return fail(E2E_EINVAL, "rv_mps must be finite with |v| <= 1.5e5 m/s");
    if (!(std::isfinite(r->flux_scale) && r->flux_scale >= 0))
        return fail(E2E_EINVAL, "flux_scale must be finite and >= 0");
    if (r->precision < E2E_PREC_F64 || r->precision > E2E_PREC_F16_HILO)
        return fail(E2E_EINVAL, "precision=%d", r->precision);
    if (r->precision != E2E_PREC_F64 && P->kind != E2E_PSF_SEPARABLE)
        return fail(E2E_EUNSUPPORTED, "reduced precisions exist on the separable path only");
    *pf = F;
    *pp = P;
    return E2E_OK;
}

static void tile_geom(const PsfRes *P, int precision, int *tw, int *th)
{
    if (P->kind == E2E_PSF_TABLE) {
        *tw = table_tw(P->kw);
        *th = kTableTH;
    } else if (P->kind == E2E_PSF_SEPARABLE &&
               (precision == E2E_PREC_BF16_HILO || precision == E2E_PREC_F16_HILO)) {
        *tw = kMfmaTW;
        *th = kMfmaTH;
    } else if (P->kind == E2E_PSF_SFI) {
        *tw = kSfiTW;
        *th = kSfiTH;
    } else {
        *tw = *th = kSepTile;
    }
}

e2e_status e2e::run_frames(e2e_ctx *ctx, const e2e_render_req *reqs, int n, bool batch,
                           bool noalloc)
{
    if (!ctx) return fail(E2E_EINVAL, "NULL context");
    if (n < 1) return fail(E2E_EINVAL, "n=%d", n);
    if (noalloc && (n != 1 || batch || !reqs[0].out_on_device || !reqs[0].spectra_on_device))
        return fail(E2E_EINVAL, "e2e_render_noalloc: one frame, device spectra and output");
    hipSetDevice(ctx->dev);
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::vector<FormatRes *> fs(n);
    std::vector<PsfRes *> ps(n);
    for (int i = 0; i < n; ++i) {
        e2e_status st = validate_req(ctx, &reqs[i], &fs[i], &ps[i]);
        if (st != E2E_OK) return st;
    }
    // one launch: a single PSF kind / table size / precision
    for (int i = 1; i < n; ++i) {
        if (ps[i]->kind != ps[0]->kind || ps[i]->kw != ps[0]->kw ||
            reqs[i].precision != reqs[0].precision ||
            reqs[i].spectrum_dtype != reqs[0].spectrum_dtype)
            return fail(E2E_EINVAL,
                        "batch frames must share PSF kind, table size, precision, spectrum type");
        if (reqs[i].hip_stream != reqs[0].hip_stream)
            return fail(E2E_EINVAL, "batch frames must share one stream");
    }
    hipStream_t s = reqs[0].hip_stream ? (hipStream_t)reqs[0].hip_stream : ctx->stream;
    // the allocation-free render uses a Scratch view of the device array
    Scratch na_sc;
    Scratch *sc = noalloc ? &na_sc : scratch_for(ctx, s);
    if (!sc) return fail(E2E_EDEVICE, "scratch allocation failed");
    if (noalloc) {
        if (!ctx->noalloc.base) return fail(E2E_EDEVICE, "no allocation-free scratch on device");
        sc->err = reinterpret_cast<int *>(ctx->noalloc.base);
        sc->counter = reinterpret_cast<int *>(ctx->noalloc.base + 64);
        sc->err_host = &ctx->noalloc.err_host;
    }
    // temporaries of the previous call on this stream are free once the
    // stream has passed it
    hipError_t e = hipSuccess;
    if (!sc->temps.empty()) {
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        for (void *p : sc->temps) hipFree(p);
        sc->temps.clear();
    }

    const int kind = ps[0]->kind, prec = reqs[0].precision;
    KernelCfg cfg{};
    cfg.kw = kind == E2E_PSF_TABLE ? ps[0]->kw : (kind == E2E_PSF_SEPARABLE ? 1 : 0);
    cfg.spec_f64 = reqs[0].spectrum_dtype == E2E_F64;
    cfg.precision = prec;
    // launch choices of each frame's workload shape (e2e_autotune), else
    // defaults (ctx->mu is held for the whole call)
    std::vector<TuneRec> tr(n);
    for (int i = 0; i < n; ++i) {
        auto it = ctx->tune.find(tune_key(fs[i], ps[i], prec, reqs[i].spectrum_dtype));
        if (it != ctx->tune.end()) tr[i] = it->second;
    }
    cfg.resident = tr[0].resident;
    size_t seg_total = 0;
    std::vector<size_t> seg_off(n);
    std::vector<int> tiles(n);
    int nslots_total = 0;
    std::vector<int> spec_off(n);
    size_t temp_bytes = 0;
    for (int i = 0; i < n; ++i) {
        int tw, th;
        tile_geom(ps[i], prec, &tw, &th);
        int ntx = (fs[i]->nx + tw - 1) / tw, nty = (fs[i]->ny + th - 1) / th;
        tiles[i] = kind == E2E_PSF_TABLE ? table_units(ntx, nty, tr[i].chunk) : ntx * nty;
        seg_off[i] = seg_total;
        seg_total += (size_t)ntx * fs[i]->ntr;
        spec_off[i] = nslots_total;
        nslots_total += fs[i]->nslots;
        cfg.degx = std::max(cfg.degx, fs[i]->degx);
        cfg.degy = std::max(cfg.degy, fs[i]->degy);
        if (!reqs[i].out_on_device)
            temp_bytes += (size_t)fs[i]->nx * fs[i]->ny * (reqs[i].out_dtype == E2E_F64 ? 8 : 4);
    }
    size_t work_n = 0;
    for (int i = 0; i < n; ++i) work_n += tiles[i];
    size_t tf_total = 0;
    std::vector<size_t> tf_off(n);
    for (int i = 0; i < n; ++i) {
        tf_off[i] = tf_total;
        tf_total += fs[i]->ntr;
    }
    const size_t seg_bytes = seg_total * sizeof(SegDev) + tf_total * sizeof(TraceFrameDev);
    size_t scratch_need = seg_bytes + n * sizeof(FrameDev) +
                          work_n * sizeof(int2) + nslots_total * sizeof(void *);
    if (ctx->used + temp_bytes + scratch_need > ctx->budget)
        return fail(E2E_ENOMEM, "render needs %zu bytes beyond the %llu-byte budget",
                    temp_bytes + scratch_need, (unsigned long long)ctx->budget);
    e2e_status st;
    if (noalloc) {
        // [err, counter | frame record | spectrum pointers | planner output]
        auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
        const size_t o_fr = 256, o_sp = o_fr + up(sizeof(FrameDev));
        const size_t o_seg = o_sp + up(kParamSlots * sizeof(void *));
        if (nslots_total > kParamSlots)
            return fail(E2E_EINVAL, "e2e_render_noalloc: %d spectrum slots, at most %d",
                        nslots_total, kParamSlots);
        if (o_seg + seg_bytes + 16 > kNoAllocBytes)
            return fail(E2E_ENOMEM,
                        "e2e_render_noalloc: needs %zu bytes of scratch, the limit is %zu",
                        o_seg + seg_bytes + 16, kNoAllocBytes);
        sc->frames_dev = reinterpret_cast<FrameDev *>(ctx->noalloc.base + o_fr);
        sc->specptrs = reinterpret_cast<const void **>(ctx->noalloc.base + o_sp);
        sc->segs = reinterpret_cast<SegDev *>(ctx->noalloc.base + o_seg);
    }
    // planner output: segments of every frame, then the per-trace constants
    if (!noalloc && (st = grow((void **)&sc->segs, &sc->segs_cap, seg_bytes + 16, "segs")) != E2E_OK)
        return st;
    if (!noalloc) {
        if ((st = grow((void **)&sc->frames_dev, &sc->frames_cap, n * sizeof(FrameDev),
                       "frames")) != E2E_OK)
            return st;
        if ((st = grow((void **)&sc->work, &sc->work_cap, work_n * sizeof(int2) + 16, "work")) !=
            E2E_OK)
            return st;
        if ((st = grow((void **)&sc->specptrs, &sc->specptrs_cap,
                       nslots_total * sizeof(void *) + 16, "spectra")) != E2E_OK)
            return st;
    }

    // spectra pointers (device), host spectra copied to temporaries
    sc->h_specptrs.assign(nslots_total, nullptr);
    for (int i = 0; i < n; ++i) {
        const e2e_render_req &r = reqs[i];
        size_t esz = r.spectrum_dtype == E2E_F64 ? 8 : 4;
        std::vector<int64_t> len(fs[i]->nslots, 0);
        for (auto &T : fs[i]->host) len[T.slot] = std::max<int64_t>(len[T.slot], T.n);
        for (int q = 0; q < fs[i]->nslots; ++q) {
            if (r.spectra_on_device || len[q] == 0) {
                sc->h_specptrs[spec_off[i] + q] = (void *)r.spectra[q];
                continue;
            }
            void *d = nullptr;
            if ((e = hipMalloc(&d, len[q] * esz)) != hipSuccess) return hip_fail(e, "spectrum");
            sc->temps.push_back(d);
            if ((e = hipMemcpyAsync(d, r.spectra[q], len[q] * esz, hipMemcpyHostToDevice, s)) !=
                hipSuccess)
                return hip_fail(e, "spectrum upload");
            sc->h_specptrs[spec_off[i] + q] = d;
        }
    }
    sc->h_frames.assign(n, FrameDev{});
    std::vector<void *> dev_out(n);
    for (int i = 0; i < n; ++i) {
        const e2e_render_req &r = reqs[i];
        FrameDev &F = sc->h_frames[i];
        FormatRes *fm = fs[i];
        PsfRes *P = ps[i];
        int tw, th;
        tile_geom(P, prec, &tw, &th);
        F.tr = fm->dev;
        F.spec = sc->specptrs + spec_off[i];
        if (r.out_on_device) {
            dev_out[i] = r.out;
        } else {
            size_t ob = (size_t)fm->nx * fm->ny * (r.out_dtype == E2E_F64 ? 8 : 4);
            if ((e = hipMalloc(&dev_out[i], ob)) != hipSuccess) return hip_fail(e, "out");
            sc->temps.push_back(dev_out[i]);
        }
        F.out = dev_out[i];
        F.tfrag = P->tfrag;
        F.sxy = P->sxy;
        F.sfq = P->sfq;
        F.sfi_R = P->sfi_R;
        F.sfi_S = P->sfi_S;
        F.sfi_shape = P->sfi_shape;
        F.segs = sc->segs + seg_off[i];
        F.tf = reinterpret_cast<TraceFrameDev *>(sc->segs + seg_total) + tf_off[i];
        F.beta = r.rv_mps / 299792458.0;
        F.flux_scale = r.flux_scale;
        F.sigma = P->sigma;
        F.gx = P->gx;
        F.gy = P->gy;
        F.gsx = P->gx > 1 ? (double)(P->gx - 1) / (double)(fm->nx - 1) : 0.0;
        F.gsy = P->gy > 1 ? (double)(P->gy - 1) / (double)(fm->ny - 1) : 0.0;
        F.ntr = fm->ntr;
        F.nx = fm->nx;
        F.ny = fm->ny;
        F.psf_kind = P->kind;
        F.H = P->H;
        F.kw = P->kw;
        F.spec_f64 = r.spectrum_dtype == E2E_F64;
        F.out_f64 = r.out_dtype == E2E_F64;
        F.precision = r.precision;
        F.tw = tw;
        F.th = th;
        F.ntx = (fm->nx + tw - 1) / tw;
        F.nty = (fm->ny + th - 1) / th;
        F.chunk = tr[i].chunk;
        F.poisson = r.poisson ? 1 : 0;
        F.frame_index = r.frame_index;
        F.seed = r.seed;
    }
    cfg.plain_tiles = tiles[0];
    // work list: frames by decreasing size, tiles in order
    sc->h_work.clear();
    if (batch) {
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return tiles[a] > tiles[b]; });
        sc->h_work.reserve(work_n);
        // frames of equal size go unit by unit, so the same unit of each (the
        // same spectrum ranges, read again under another Doppler shift) runs
        // at about the same time and its reads hit the caches
        for (size_t g = 0; g < order.size();) {
            size_t h = g;
            while (h < order.size() && tiles[order[h]] == tiles[order[g]]) ++h;
            for (int t = 0; t < tiles[order[g]]; ++t)
                for (size_t q = g; q < h; ++q) sc->h_work.push_back(make_int2(order[q], t));
            g = h;
        }
    }
    if (noalloc) {
        // parameters travel as a kernel argument: no staging buffer
        FrameParams prm{};
        prm.f = sc->h_frames[0];
        prm.nslots = nslots_total;
        for (int q = 0; q < nslots_total; ++q) prm.spec[q] = sc->h_specptrs[q];
        if ((e = launch_put_params(prm, sc->frames_dev, sc->specptrs, s)) != hipSuccess)
            return hip_fail(e, "parameter kernel");
    } else {
        // parameter upload through pinned staging (reused once its copy ran)
        size_t b_spec = nslots_total * sizeof(void *), b_fr = n * sizeof(FrameDev),
               b_work = batch ? work_n * sizeof(int2) : 0;
        size_t b_all = b_spec + b_fr + b_work + 64;
        if (sc->staged_valid) {
            if ((e = hipEventSynchronize(sc->staged)) != hipSuccess) return hip_fail(e, "staging");
        }
        if (sc->stage_cap < b_all) {
            if (sc->stage) hipHostFree(sc->stage);
            sc->stage = nullptr;
            sc->stage_cap = 0;
            if ((e = hipHostMalloc(&sc->stage, b_all * 2)) != hipSuccess) return hip_fail(e, "staging");
            sc->stage_cap = b_all * 2;
        }
        if (!sc->staged) {
            if ((e = hipEventCreateWithFlags(&sc->staged, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "event");
        }
        char *stg = (char *)sc->stage;
        memcpy(stg, sc->h_specptrs.data(), b_spec);
        memcpy(stg + b_spec, sc->h_frames.data(), b_fr);
        if (b_work) memcpy(stg + b_spec + b_fr, sc->h_work.data(), b_work);
        if ((e = hipMemcpyAsync(sc->specptrs, stg, b_spec, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(sc->frames_dev, stg + b_spec, b_fr, hipMemcpyHostToDevice, s)) !=
                hipSuccess)
            return hip_fail(e, "parameter upload");
        if (b_work && (e = hipMemcpyAsync(sc->work, stg + b_spec + b_fr, b_work,
                                          hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "work upload");
        if ((e = hipEventRecord(sc->staged, s)) != hipSuccess) return hip_fail(e, "event");
        sc->staged_valid = true;
    }

    if (noalloc && (e = launch_fill_i32(sc->err, 1, 0, s)) != hipSuccess)
        return hip_fail(e, "error word");
    bool any_noise = false;
    for (int i = 0; i < n; ++i) any_noise |= reqs[i].poisson != 0;
    const int2 *work = batch ? sc->work : nullptr;
    const int nwork = batch ? (int)work_n : 0;
    // the launch sequence: clear error word and queue counter, plan, render, noise
    auto enqueue = [&]() -> hipError_t {
        hipError_t q;
        // the error word is sticky (cleared after a synchronous read), so an
        // asynchronous launch's device error reaches the next synchronous call
        if ((q = launch_fill_i32(sc->counter, 1, 0, s)) != hipSuccess) return q;
        prof_begin(ctx, s, "plan");
        q = launch_plan(sc->frames_dev, sc->h_frames.data(), n, sc->err, s);
        prof_end(ctx, s);
        if (q != hipSuccess) return q;
        if (kind == E2E_PSF_TABLE) {
            prof_begin(ctx, s, "render_table");
            q = launch_table(sc->frames_dev, cfg, work, nwork, sc->counter, sc->err, s);
        } else if (kind == E2E_PSF_SEPARABLE &&
                   (prec == E2E_PREC_BF16_HILO || prec == E2E_PREC_F16_HILO)) {
            prof_begin(ctx, s, "render_sep_mfma");
            q = launch_sep_mfma(sc->frames_dev, cfg, work, nwork, sc->counter, sc->err, s);
        } else if (kind == E2E_PSF_SFI) {
            prof_begin(ctx, s, "render_sfi");
            q = launch_sfi(sc->frames_dev, cfg, work, nwork, sc->counter, sc->err, s);
        } else {
            prof_begin(ctx, s, "render_sep");
            q = launch_sep(sc->frames_dev, cfg, work, nwork, sc->counter, sc->err, s);
        }
        prof_end(ctx, s);
        if (q != hipSuccess) return q;
        if (any_noise) {
            prof_begin(ctx, s, "noise");
            q = launch_noise_frames(sc->frames_dev, sc->h_frames.data(), n, s);
            prof_end(ctx, s);
        }
        return q;
    };
    // A batch replays a HIP graph captured once per launch signature (the
    // graph's kernels read their parameters from the scratch buffers just
    // uploaded); no memset nodes are recorded, counters are cleared by a
    // fill kernel.  Timed runs (profiling on) launch eagerly.
    bool use_graph = batch && !ctx->prof && ctx->graphs;
    if (use_graph) {
        int maxw = 0;
        int64_t maxpix = 0;
        for (int i = 0; i < n; ++i) {
            maxw = std::max(maxw, sc->h_frames[i].ntx * sc->h_frames[i].ntr);
            maxpix = std::max(maxpix, (int64_t)sc->h_frames[i].nx * sc->h_frames[i].ny);
        }
        char key[256];
        snprintf(key, sizeof key, "%d/%d/%d/%d/%d/%d/%d/%d/%zu/%d/%lld/%d/%p/%p", kind, cfg.kw,
                 cfg.resident, cfg.degx, cfg.degy, cfg.spec_f64, prec, n, work_n, maxw,
                 any_noise ? (long long)maxpix : 0ll, (int)any_noise, (void *)sc->frames_dev,
                 (void *)sc->work);
        auto it = sc->graphs.find(key);
        if (it == sc->graphs.end()) {
            GraphRec g;
            if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "graph capture");
            hipError_t qe = enqueue();
            e = hipStreamEndCapture(s, &g.graph);
            if (qe != hipSuccess) return hip_fail(qe, "render launch (capture)");
            if (e != hipSuccess) return hip_fail(e, "graph capture");
            if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) {
                hipGraphDestroy(g.graph);
                return hip_fail(e, "graph instantiate");
            }
            it = sc->graphs.emplace(key, g).first;
        }
        if ((e = hipGraphLaunch(it->second.exec, s)) != hipSuccess)
            return hip_fail(e, "graph launch");
    } else {
        if ((e = enqueue()) != hipSuccess) return hip_fail(e, "render launch");
    }
    for (int i = 0; i < n; ++i) {
        if (reqs[i].out_on_device) continue;
        size_t ob = (size_t)fs[i]->nx * fs[i]->ny * (reqs[i].out_dtype == E2E_F64 ? 8 : 4);
        if ((e = hipMemcpyAsync(reqs[i].out, dev_out[i], ob, hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            return hip_fail(e, "out download");
    }
    if ((e = hipMemcpyAsync(sc->err_host, sc->err, sizeof(int), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return hip_fail(e, "error word");
    bool all_async = !noalloc;
    for (int i = 0; i < n; ++i)
        all_async &= (reqs[i].flags & E2E_FLAG_ASYNC) && reqs[i].out_on_device &&
                     reqs[i].spectra_on_device;
    if (all_async) return E2E_OK;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "render");
    return take_err_word(sc, s);
}

// The device error word of a stream's scratch after the stream has passed
// the copy into err_host: reported (also for the asynchronous launches since
// the last synchronous read) and cleared.
e2e_status e2e::take_err_word(Scratch *sc, hipStream_t s)
{
    const int w = *sc->err_host;
    if (w == 0) return E2E_OK;
    *sc->err_host = 0;
    launch_fill_i32(sc->err, 1, 0, s);
    return check_err_word(w);
}

extern "C" e2e_status e2e_sync(e2e_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(E2E_EINVAL, "e2e_sync: NULL context");
    hipSetDevice(ctx->dev);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->scratch.find(s);
    hipError_t e;
    if (it == ctx->scratch.end()) {
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "e2e_sync");
        return E2E_OK;
    }
    Scratch *sc = it->second;
    if ((e = hipMemcpyAsync(sc->err_host, sc->err, sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "e2e_sync");
    return take_err_word(sc, s);
}

e2e_status e2e::check_err_word(int w)
{
    if (w == 0) return E2E_OK;
    return fail(E2E_EINTERNAL,
                "device check failed (0x%x):%s%s%s%s", w,
                (w & kErrTileTraces) ? " too many traces reach one tile;" : "",
                (w & kErrRowWindow) ? " a slot column left its row window;" : "",
                (w & kErrSearch) ? " column search did not converge;" : "",
                (w & kErrCells) ? " PSF node-cell range inconsistent;" : "");
}

extern "C" e2e_status e2e_render(e2e_ctx *ctx, const e2e_render_req *req)
{
    return run_frames(ctx, req, 1, false);
}

extern "C" e2e_status e2e_render_noalloc(e2e_ctx *ctx, const e2e_render_req *req)
{
    if (!req) return fail(E2E_EINVAL, "e2e_render_noalloc: req is NULL");
    return run_frames(ctx, req, 1, false, true);
}

std::string e2e::tune_key(const FormatRes *f, const PsfRes *p, int precision, int spectrum_dtype)
{
    char k[160];
    snprintf(k, sizeof k, "%d/%d/%d/%d/%d/%d/%d/%d/%d/%d", p->kind, p->kw, p->gx, p->gy, precision,
             spectrum_dtype, f->nx, f->ny, f->ntr, f->degx * 16 + f->degy);
    return k;
}

// Candidate launch choices are rendered on the caller's own requests (a warm
// run, then the best of two timed runs) and the fastest is kept for their
// workload shapes.  The work-unit length changes only the order in which a
// pixel's contributions are summed (the result stays deterministic for a
// given choice); the persistent-grid width changes nothing in the result.
extern "C" e2e_status e2e_autotune(e2e_ctx *ctx, const e2e_render_req *reqs, int32_t n,
                                   e2e_tune_report *report)
{
    if (!ctx || !reqs || n < 1) return fail(E2E_EINVAL, "e2e_autotune: bad arguments");
    std::vector<std::string> keys(n);
    bool table = false;
    {
        // handles are looked up under the context lock; run_frames takes it
        // again for each timed run, so it is not held across them
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (int i = 0; i < n; ++i) {
            FormatRes *f = nullptr;
            PsfRes *p = nullptr;
            e2e_status st = validate_req(ctx, &reqs[i], &f, &p);
            if (st != E2E_OK) return st;
            keys[i] = tune_key(f, p, reqs[i].precision, reqs[i].spectrum_dtype);
            if (i == 0) table = p->kind == E2E_PSF_TABLE;
        }
    }
    const bool batch = n > 1;
    std::vector<int> chunks = table ? std::vector<int>{2, 4, 8, 16} : std::vector<int>{kTableChunk};
    // a single-frame tuning keeps the batch width already chosen for the shape
    int keep_resident = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->tune.find(keys[0]);
        if (it != ctx->tune.end()) keep_resident = it->second.resident;
    }
    std::vector<int> residents =
        batch ? std::vector<int>{1, 2, 3} : std::vector<int>{keep_resident};
    hipSetDevice(ctx->dev);
    hipStream_t s = reqs[0].hip_stream ? (hipStream_t)reqs[0].hip_stream : ctx->stream;
    hipEvent_t e0, e1;
    hipError_t he;
    if ((he = hipEventCreate(&e0)) != hipSuccess) return hip_fail(he, "event");
    if ((he = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(he, "event");
    }
    // synchronous runs for timing, whatever the requests' flags say
    std::vector<e2e_render_req> rq(reqs, reqs + n);
    for (auto &r : rq) r.flags &= ~(uint32_t)E2E_FLAG_ASYNC;
    e2e_tune_report rep{};
    double best = 1e300;
    TuneRec best_rec;
    e2e_status st = E2E_OK;
    for (int c : chunks) {
        for (int r : residents) {
            TuneRec t;
            t.chunk = c;
            t.resident = r;
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                for (auto &k : keys) ctx->tune[k] = t;
            }
            double ms = 1e300;
            for (int rep_i = 0; rep_i < 3 && st == E2E_OK; ++rep_i) {
                hipEventRecord(e0, s);
                st = run_frames(ctx, rq.data(), n, batch);
                hipEventRecord(e1, s);
                hipEventSynchronize(e1);
                float f = 0.f;
                hipEventElapsedTime(&f, e0, e1);
                if (rep_i > 0) ms = std::min(ms, (double)f);  // first run warms up
            }
            if (st != E2E_OK) break;
            if (rep.n_candidates < E2E_TUNE_MAX) {
                rep.cand_chunk[rep.n_candidates] = c;
                rep.cand_resident[rep.n_candidates] = r;
                rep.cand_ms[rep.n_candidates] = ms;
                rep.n_candidates++;
            }
            if (ms < best) {
                best = ms;
                best_rec = t;
            }
        }
        if (st != E2E_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &k : keys) ctx->tune[k] = best_rec;
    }
    if (st != E2E_OK) return st;
    rep.chunk = best_rec.chunk;
    rep.resident = best_rec.resident;
    rep.ms = best;
    if (report) *report = rep;
    return E2E_OK;
}

extern "C" e2e_status e2e_render_batch(e2e_ctx *ctx, const e2e_render_req *reqs, int32_t n)
{
    if (!reqs) return fail(E2E_EINVAL, "e2e_render_batch: reqs is NULL");
    return run_frames(ctx, reqs, n, true);
}

// ------------------------------------------------------------------ noise

extern "C" e2e_status e2e_noise_poisson(e2e_ctx *ctx, void *frame, int32_t dtype, int64_t n,
                                        uint64_t seed, uint32_t fidx, int32_t on_device,
                                        void *stream)
{
    if (!ctx || !frame) return fail(E2E_EINVAL, "e2e_noise_poisson: NULL argument");
    if (dtype != E2E_F32 && dtype != E2E_F64) return fail(E2E_EINVAL, "dtype=%d", dtype);
    if (n < 0) return fail(E2E_EINVAL, "n_pixels=%lld", (long long)n);
    if (n == 0) return E2E_OK;
    hipSetDevice(ctx->dev);
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    size_t bytes = (size_t)n * (dtype == E2E_F64 ? 8 : 4);
    void *d = frame;
    hipError_t e;
    if (!on_device) {
        if ((e = hipMalloc(&d, bytes)) != hipSuccess) return hip_fail(e, "noise buffer");
        if ((e = hipMemcpyAsync(d, frame, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) {
            hipFree(d);
            return hip_fail(e, "noise upload");
        }
    }
    prof_begin(ctx, s, "noise");
    e = launch_noise(d, dtype == E2E_F64, n, seed, fidx, s);
    prof_end(ctx, s);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(frame, d, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (!on_device) hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "e2e_noise_poisson");
    return E2E_OK;
}

extern "C" e2e_status e2e_detector(e2e_ctx *ctx, const e2e_detector_desc *d, const void *frame,
                                   int32_t dtype, const float *prnu, int32_t nx, int32_t ny,
                                   uint16_t *adu_out, int32_t on_device, void *stream)
{
    if (!ctx || !d || !frame || !adu_out) return fail(E2E_EINVAL, "e2e_detector: NULL argument");
    if (dtype != E2E_F32 && dtype != E2E_F64) return fail(E2E_EINVAL, "dtype=%d", dtype);
    if (nx < 0 || ny < 0 || ny > 65535 * 64)
        return fail(E2E_EINVAL, "e2e_detector: nx=%d ny=%d", nx, ny);
    if (d->bits < 1 || d->bits > 16) return fail(E2E_EINVAL, "e2e_detector: bits=%d", d->bits);
    if (!(d->gain_e_per_adu > 0.0) || !std::isfinite(d->gain_e_per_adu))
        return fail(E2E_EINVAL, "e2e_detector: gain_e_per_adu=%g", d->gain_e_per_adu);
    if (!(d->exposure_s >= 0.0) || !std::isfinite(d->exposure_s) || !(d->dark_e_per_s >= 0.0) ||
        !std::isfinite(d->dark_e_per_s) || !(d->ron_e >= 0.0) || !std::isfinite(d->ron_e) ||
        !std::isfinite(d->bias_adu))
        return fail(E2E_EINVAL, "e2e_detector: exposure, dark current, read noise or bias");
    for (int q = 0; q < 9; ++q)
        if (!std::isfinite(d->xtalk[q])) return fail(E2E_EINVAL, "e2e_detector: xtalk[%d]", q);
    const int64_t n = (int64_t)nx * ny;
    if (n == 0) return E2E_OK;
    hipSetDevice(ctx->dev);
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    const size_t fbytes = (size_t)n * (dtype == E2E_F64 ? 8 : 4);
    const size_t gbytes = prnu ? (size_t)n * 4 : 0;
    const size_t obytes = (size_t)n * 2;
    const void *fd = frame;
    const float *gd = prnu;
    uint16_t *od = adu_out;
    char *blk = nullptr;
    hipError_t e = hipSuccess;
    if (!on_device) {
        // staged copies of the caller's host buffers
        const size_t off_g = (fbytes + 255) & ~(size_t)255;
        const size_t off_o = off_g + ((gbytes + 255) & ~(size_t)255);
        if ((e = hipMalloc((void **)&blk, off_o + obytes)) != hipSuccess)
            return hip_fail(e, "detector buffers");
        fd = blk;
        gd = prnu ? (const float *)(blk + off_g) : nullptr;
        od = (uint16_t *)(blk + off_o);
        e = hipMemcpyAsync((void *)fd, frame, fbytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && prnu)
            e = hipMemcpyAsync((void *)gd, prnu, gbytes, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) {
        prof_begin(ctx, s, "detector");
        e = launch_detector(fd, dtype == E2E_F64, gd, nx, ny, d->dark_e_per_s * d->exposure_s,
                            d->shot_noise != 0, d->xtalk, d->ron_e, d->gain_e_per_adu,
                            d->bias_adu, d->bits, d->seed, d->frame_index, od, s);
        prof_end(ctx, s);
    }
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(adu_out, od, obytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (blk) hipFree(blk);
    if (e != hipSuccess) return hip_fail(e, "e2e_detector");
    return E2E_OK;
}

extern "C" e2e_status e2e_philox_blocks(e2e_ctx *ctx, uint64_t seed, uint32_t fidx,
                                        uint64_t pixel0, int64_t n, uint32_t blocks,
                                        uint32_t *out)
{
    if (!ctx || !out) return fail(E2E_EINVAL, "e2e_philox_blocks: NULL argument");
    if (n < 0 || blocks == 0 || (uint64_t)n * blocks > (1ull << 28))
        return fail(E2E_EINVAL, "e2e_philox_blocks: bad size");
    if (n == 0) return E2E_OK;
    hipSetDevice(ctx->dev);
    size_t bytes = (size_t)n * blocks * 16;
    uint32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e == hipSuccess) e = launch_philox(seed, fidx, pixel0, n, blocks, d, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "e2e_philox_blocks");
    return E2E_OK;
}

// -------------------------------------------------------------- profiling

void e2e::prof_begin(e2e_ctx *ctx, hipStream_t s, const char *name)
{
    if (!ctx->prof) return;
    ProfRec r;
    r.name = name;
    hipEventCreate(&r.a);
    hipEventCreate(&r.b);
    hipEventRecord(r.a, s);
    ctx->prof_pending.push_back(r);
}

void e2e::prof_end(e2e_ctx *ctx, hipStream_t s)
{
    if (!ctx->prof || ctx->prof_pending.empty()) return;
    hipEventRecord(ctx->prof_pending.back().b, s);
}

extern "C" e2e_status e2e_set_profiling(e2e_ctx *ctx, int32_t on)
{
    if (!ctx) return fail(E2E_EINVAL, "NULL context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->prof = on != 0;
    return E2E_OK;
}

static void prof_collect(e2e_ctx *ctx)
{
    for (auto &r : ctx->prof_pending) {
        hipEventSynchronize(r.b);
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &acc = ctx->prof_acc[r.name];
            acc.first += 1;
            acc.second += ms;
        }
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    ctx->prof_pending.clear();
}

extern "C" e2e_status e2e_kernel_time(e2e_ctx *ctx, const char *k, int64_t *launches,
                                      double *total_ms)
{
    if (!ctx || !k || !launches || !total_ms) return fail(E2E_EINVAL, "NULL argument");
    hipSetDevice(ctx->dev);
    std::lock_guard<std::mutex> lk(ctx->mu);
    prof_collect(ctx);
    auto it = ctx->prof_acc.find(k);
    *launches = it == ctx->prof_acc.end() ? 0 : it->second.first;
    *total_ms = it == ctx->prof_acc.end() ? 0.0 : it->second.second;
    return E2E_OK;
}

extern "C" e2e_status e2e_reset_kernel_time(e2e_ctx *ctx)
{
    if (!ctx) return fail(E2E_EINVAL, "NULL context");
    hipSetDevice(ctx->dev);
    std::lock_guard<std::mutex> lk(ctx->mu);
    prof_collect(ctx);
    ctx->prof_acc.clear();
    return E2E_OK;
}
