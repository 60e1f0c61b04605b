// C ABI of the closing-the-loop steps (Sec. 1, Sec. 4.2): e2e_extract and
// e2e_ccf.  Argument checks, staging of host buffers, the template
// smoothing widths, launches, and the parabola vertex of the summed CCF.
#include <cmath>
#include <cstring>
#include <vector>

#include "api_internal.h"

namespace e2e {
hipError_t launch_extract(const TraceDev *trs, int ntr, int nx, int ny, const void *frame,
                          int f64, double A, double *flux, double *edges, hipStream_t s);
hipError_t launch_smooth3(const void *lt_dev, int ntr, int64_t nmax, int wmax, int f64,
                          hipStream_t s);
int loop_max_width();
hipError_t launch_ccf(const TraceDev *trs, int tr0, int ntr, const void *lt_dev, int nx,
                      const double *flux, const double *flat, const double *edges, double v0,
                      double dv, int nv, double *C, hipStream_t s);
size_t loop_trace_bytes();
void loop_trace_fill(void *dst, const void *tmpl, double *P, double *X, int64_t n, int w);
}  // namespace e2e

using namespace e2e;

namespace {

// Device buffers of one call, released on every exit path.
struct Bufs {
    std::vector<void *> p;
    ~Bufs()
    {
        for (void *q : p) hipFree(q);
    }
    hipError_t get(void **out, size_t bytes)
    {
        *out = nullptr;
        hipError_t e = hipMalloc(out, bytes > 0 ? bytes : 16);
        if (e == hipSuccess) p.push_back(*out);
        return e;
    }
};

// Holds a reference on a format for the duration of a call, so that
// e2e_format_free reports E2E_EBUSY instead of freeing it underneath.
struct FormatRef {
    e2e_ctx *ctx;
    FormatRes *F = nullptr;
    FormatRef(e2e_ctx *c, e2e_format_id id) : ctx(c)
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->fmts.find(id);
        if (it == ctx->fmts.end()) return;
        F = it->second;
        F->refs++;
    }
    ~FormatRef()
    {
        if (!F) return;
        std::lock_guard<std::mutex> lk(ctx->mu);
        F->refs--;
    }
};

double horner_host(const double *c, int deg, double t)
{
    double v = c[deg];
    for (int j = deg - 1; j >= 0; --j) v = v * t + c[j];
    return v;
}

}  // namespace

extern "C" e2e_status e2e_extract(e2e_ctx *ctx, e2e_format_id fmt, const void *frame,
                                  int32_t dtype, double A, double *flux, double *edges,
                                  int32_t on_device, void *stream)
{
    if (!ctx || !frame || !flux || !edges) return fail(E2E_EINVAL, "e2e_extract: NULL argument");
    if (dtype != E2E_F32 && dtype != E2E_F64) return fail(E2E_EINVAL, "dtype=%d", dtype);
    if (!(std::isfinite(A) && A > 0.0 && A <= 1e6))
        return fail(E2E_EINVAL, "aperture_half_px=%g", A);
    FormatRef ref(ctx, fmt);
    FormatRes *F = ref.F;
    if (!F) return fail(E2E_ENOTFOUND, "format %llu not found", (unsigned long long)fmt);
    hipSetDevice(ctx->dev);
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    const size_t npx = (size_t)F->nx * F->ny, fb = npx * (dtype == E2E_F64 ? 8 : 4);
    const size_t eb = (size_t)F->ntr * F->nx * 8, lb = (size_t)F->ntr * (F->nx + 1) * 8;
    Bufs B;
    const void *fd = frame;
    double *ed = flux, *ld = edges;
    hipError_t e = hipSuccess;
    if (!on_device) {
        void *a, *b, *c;
        if ((e = B.get(&a, fb)) != hipSuccess || (e = B.get(&b, eb)) != hipSuccess ||
            (e = B.get(&c, lb)) != hipSuccess)
            return hip_fail(e, "extraction buffers");
        if ((e = hipMemcpyAsync(a, frame, fb, hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "frame upload");
        fd = a;
        ed = (double *)b;
        ld = (double *)c;
    }
    prof_begin(ctx, s, "extract");
    e = launch_extract(F->dev, F->ntr, F->nx, F->ny, fd, dtype == E2E_F64, A, ed, ld, s);
    prof_end(ctx, s);
    if (e == hipSuccess && !on_device) {
        e = hipMemcpyAsync(flux, ed, eb, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(edges, ld, lb, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "e2e_extract");
    return E2E_OK;
}

extern "C" e2e_status e2e_ccf(e2e_ctx *ctx, e2e_format_id fmt, const e2e_ccf_req *r,
                              double *rv_out)
{
    if (!ctx || !r || !rv_out || !r->flux || !r->edges || !r->templates)
        return fail(E2E_EINVAL, "e2e_ccf: NULL argument");
    if (r->template_dtype != E2E_F32 && r->template_dtype != E2E_F64)
        return fail(E2E_EINVAL, "template_dtype=%d", r->template_dtype);
    if (r->n_v < 3) return fail(E2E_EINVAL, "n_v=%d (needs >= 3)", r->n_v);
    if (!(std::isfinite(r->dv_mps) && r->dv_mps != 0.0) || !std::isfinite(r->v0_mps))
        return fail(E2E_EINVAL, "e2e_ccf: velocity grid");
    const double vmax = std::fmax(std::fabs(r->v0_mps), std::fabs(r->v0_mps + (r->n_v - 1) * r->dv_mps));
    if (vmax > 1.5e7) return fail(E2E_EINVAL, "e2e_ccf: |v| above 1.5e7 m/s");
    if (!(std::isfinite(r->smooth_px) && r->smooth_px > 0.0))
        return fail(E2E_EINVAL, "smooth_px=%g", r->smooth_px);
    FormatRef ref(ctx, fmt);
    FormatRes *F = ref.F;
    if (!F) return fail(E2E_ENOTFOUND, "format %llu not found", (unsigned long long)fmt);
    if (r->n_templates < F->nslots)
        return fail(E2E_EINVAL, "n_templates=%d, the format uses %d", r->n_templates, F->nslots);
    hipSetDevice(ctx->dev);
    hipStream_t s = r->hip_stream ? (hipStream_t)r->hip_stream : ctx->stream;
    const int ntr = F->ntr, nx = F->nx, nv = r->n_v;
    const size_t esz = r->template_dtype == E2E_F64 ? 8 : 4;
    const size_t eb = (size_t)ntr * nx * 8, lb = (size_t)ntr * (nx + 1) * 8;
    Bufs B;
    hipError_t e = hipSuccess;
    const double *fd = r->flux, *fl = r->flat, *ld = r->edges;
    std::vector<const void *> tmpl(F->nslots, nullptr);
    for (auto &T : F->host) {
        if (!r->templates[T.slot]) return fail(E2E_EINVAL, "template of slot %d is NULL", T.slot);
        tmpl[T.slot] = r->templates[T.slot];
    }
    if (!r->on_device) {
        void *a, *b, *c = nullptr;
        if ((e = B.get(&a, eb)) != hipSuccess || (e = B.get(&b, lb)) != hipSuccess ||
            (r->flat && (e = B.get(&c, eb)) != hipSuccess))
            return hip_fail(e, "ccf buffers");
        if ((e = hipMemcpyAsync(a, r->flux, eb, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(b, r->edges, lb, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (r->flat && (e = hipMemcpyAsync(c, r->flat, eb, hipMemcpyHostToDevice, s)) !=
                            hipSuccess))
            return hip_fail(e, "ccf upload");
        fd = (const double *)a;
        ld = (const double *)b;
        fl = (const double *)c;
        std::vector<int64_t> len(F->nslots, 0);
        for (auto &T : F->host) len[T.slot] = std::max<int64_t>(len[T.slot], T.n);
        for (int q = 0; q < F->nslots; ++q) {
            if (!tmpl[q]) continue;
            void *d;
            if ((e = B.get(&d, (size_t)len[q] * esz)) != hipSuccess) return hip_fail(e, "template");
            if ((e = hipMemcpyAsync(d, tmpl[q], (size_t)len[q] * esz, hipMemcpyHostToDevice,
                                    s)) != hipSuccess)
                return hip_fail(e, "template upload");
            tmpl[q] = d;
        }
    }
    // moving-mean width of each trace: the odd integer nearest sqrt(4 s^2 + 1),
    // s = smooth_px samples-per-pixel
    std::vector<int> w(ntr);
    int64_t nmax = 0;
    for (int t = 0; t < ntr; ++t) {
        const TraceDev &T = F->host[t];
        const double span = horner_host(T.cx, kNCoef - 1, 1.0) - horner_host(T.cx, kNCoef - 1, -1.0);
        const double sg = r->smooth_px * (double)T.n / span;
        int wi = (int)std::floor(std::sqrt(4.0 * sg * sg + 1.0) + 0.5);
        if (wi % 2 == 0) wi += 1;
        w[t] = std::max(1, wi);
        if (w[t] > loop_max_width())
            return fail(E2E_EINVAL, "e2e_ccf: smoothing window of trace %d is %d samples (max %d)",
                        t, w[t], loop_max_width());
        nmax = std::max<int64_t>(nmax, T.n);
    }
    double *Cd;
    {
        void *c;
        if ((e = B.get(&c, (size_t)ntr * nv * 8)) != hipSuccess) return hip_fail(e, "ccf out");
        Cd = (double *)c;
    }
    // traces in groups: smoothed templates (X) and prefix sums (P) per trace
    const int G = 64;
    void *work, *ltd;
    if ((e = B.get(&work, (size_t)std::min(G, ntr) * (2 * nmax + 2) * 8)) != hipSuccess)
        return hip_fail(e, "template scratch");
    const size_t ltb = loop_trace_bytes();
    if ((e = B.get(&ltd, (size_t)G * ltb)) != hipSuccess) return hip_fail(e, "trace table");
    void *stage = nullptr;
    if ((e = hipHostMalloc(&stage, (size_t)G * ltb)) != hipSuccess) return hip_fail(e, "staging");
    for (int t0 = 0; t0 < ntr && e == hipSuccess; t0 += G) {
        const int g = std::min(G, ntr - t0);
        // the previous group's table copy must have been consumed
        if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
        for (int q = 0; q < g; ++q) {
            const TraceDev &T = F->host[t0 + q];
            double *base = (double *)work + (size_t)q * (2 * nmax + 2);
            loop_trace_fill((char *)stage + q * ltb, tmpl[T.slot], base, base + nmax + 1, T.n,
                            w[t0 + q]);
        }
        if ((e = hipMemcpyAsync(ltd, stage, g * ltb, hipMemcpyHostToDevice, s)) != hipSuccess)
            break;
        prof_begin(ctx, s, "template_smooth");
        int64_t ng = 0;
        int wg = 1;
        for (int q = 0; q < g; ++q) {
            ng = std::max<int64_t>(ng, F->host[t0 + q].n);
            wg = std::max(wg, w[t0 + q]);
        }
        e = launch_smooth3(ltd, g, ng, wg, r->template_dtype == E2E_F64, s);
        prof_end(ctx, s);
        if (e != hipSuccess) break;
        prof_begin(ctx, s, "ccf");
        e = launch_ccf(F->dev, t0, g, ltd, nx, fd, fl, ld, r->v0_mps, r->dv_mps, nv, Cd, s);
        prof_end(ctx, s);
    }
    std::vector<double> C((size_t)ntr * nv);
    if (e == hipSuccess) e = hipMemcpyAsync(C.data(), Cd, C.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && r->ccf_out)
        e = hipMemcpyAsync(r->ccf_out, Cd, C.size() * 8,
                           r->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipHostFree(stage);
    if (e != hipSuccess) return hip_fail(e, "e2e_ccf");
    // parabola vertex of the summed CCF (traces added in order)
    std::vector<double> tot(nv, 0.0);
    for (int t = 0; t < ntr; ++t)
        for (int k = 0; k < nv; ++k) tot[k] += C[(size_t)t * nv + k];
    int kb = 1;
    for (int k = 1; k < nv - 1; ++k)
        if (tot[k] > tot[kb]) kb = k;
    const double ym = tot[kb - 1], y0 = tot[kb], yp = tot[kb + 1];
    const double den = ym - 2.0 * y0 + yp;
    const double off = den != 0.0 ? 0.5 * (ym - yp) / den : 0.0;
    *rv_out = r->v0_mps + r->dv_mps * ((double)kb + off);
    return E2E_OK;
}
