// Planner: for every (tile column, trace) of a frame, the range of samples
// whose PSF footprint can reach the column, the tile rows they can reach and
// the PSF node cells they fall in.  x grows strictly along a trace (checked
// at format load), so each range is found by bisection on the same FP64
// positions the render kernels evaluate.
#include "dev_common.h"

namespace e2e {

namespace {

// The coefficients are held in registers, padded with zeros to degree 7
// (the format loader zeroes them; a zero leading coefficient leaves Horner's
// value bit-identical), so the bisection steps do not reload them.
__device__ double x_at(const double *cx, double t0, double dt, int k)
{
    return horner<kNCoef - 1>(cx, fma((double)k, dt, t0));
}

// first k in [lo, hi] with u(k) = fma(x(k), os, uc) >= qv (hi if none): the
// table path's slot coordinate, compared exactly as its render kernel does
__device__ int first_slot_at_or_above(const double *cx, double t0, double dt, double os,
                                      double uc, double qv, int lo, int hi)
{
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (fma(x_at(cx, t0, dt, mid), os, uc) >= qv) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// first k in [lo, hi] with x(k) >= xv (hi if none)
__device__ int first_at_or_above(const double *cx, double t0, double dt, double xv, int lo,
                                 int hi)
{
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (x_at(cx, t0, dt, mid) >= xv) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__global__ void k_plan(const FrameDev *__restrict__ frames, int *__restrict__ err)
{
    const FrameDev &F = frames[blockIdx.y];
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= F.ntx * F.ntr) return;
    int c = idx / F.ntr, tr = idx % F.ntr;
    const TraceDev &T = F.tr[tr];
    SegDev S;
    S.k0 = 0; S.k1 = 0; S.ty0 = 1; S.ty1 = 0;
    S.cx0 = S.cx1 = S.cy0 = S.cy1 = 0;

    double t0, dt;
    trace_affine(T, F.beta, &t0, &dt);
    double cx[kNCoef], cy[kNCoef];
#pragma unroll
    for (int j = 0; j < kNCoef; ++j) {
        cx[j] = T.cx[j];
        cy[j] = T.cy[j];
    }
    if (c == 0) {
        TraceFrameDev tfd;
        tfd.t0 = t0;
        tfd.dt = dt;
        tfd.scale = T.thr * F.flux_scale;
        tfd.spec = F.spec[T.slot];
        F.tf[tr] = tfd;
    }
    int X0 = c * F.tw, X1 = min(X0 + F.tw, F.nx);
    const bool table = F.psf_kind == E2E_PSF_TABLE;
    double hw = table ? (double)F.kw / (2.0 * kOS) : 0.0;
    double xlo, xhi;
    if (table) {
        xlo = X0 - 0.5 - hw;
        xhi = X1 - 0.5 + hw;
    } else {
        xlo = X0 - F.H - 0.5;
        xhi = X1 + F.H - 0.5;
    }
    int k0, k1;
    if (table) {
        // The render kernel's slot columns start at slot os X0 - kw (its left
        // halo) and the tile's pixels end at slot os X1; its samples are those
        // with u = os x + (os - kw)/2 in that range, found here with the
        // kernel's own comparison (the format polynomial is zero-padded to
        // degree 7, which leaves its value bit-identical), so the kernel takes
        // the range's ends from here without searching for them.
        const double os = (double)kOS, uc = 0.5 * (double)(kOS - F.kw);
        k0 = first_slot_at_or_above(cx, t0, dt, os, uc, (double)(kOS * X0 - F.kw), 0, T.n);
        k1 = first_slot_at_or_above(cx, t0, dt, os, uc, (double)(kOS * X1), k0, T.n);
    } else {
        xlo -= 1e-3;
        xhi += 1e-3;
        k0 = first_at_or_above(cx, t0, dt, xlo, 0, T.n);
        k1 = first_at_or_above(cx, t0, dt, xhi, k0, T.n);
    }
    if (k0 < k1) {
        // y range over [k0, k1): 9 nodes plus the curvature bound between them
        const int NP = 9;
        double ta = fma((double)k0, dt, t0), tb = fma((double)(k1 - 1), dt, t0);
        double ymin = 1e300, ymax = -1e300;
        for (int q = 0; q < NP; ++q) {
            double t = (q == NP - 1) ? tb : ta + (tb - ta) * (double)q / (NP - 1);
            double y = horner<kNCoef - 1>(cy, t);
            ymin = fmin(ymin, y);
            ymax = fmax(ymax, y);
        }
        double h = fabs(tb - ta) / (NP - 1);
        double m = T.y2max * h * h / 8.0 + 1e-6;
        ymin -= m;
        ymax += m;
        int jlo, jhi;
        if (table) {
            jlo = (int)floor(ymin - hw - 0.5) - 1;
            jhi = (int)ceil(ymax + hw + 0.5) + 1;
        } else {
            jlo = (int)floor(ymin + 0.5) - F.H - 1;
            jhi = (int)floor(ymax + 0.5) + F.H + 1;
        }
        int ty0 = max(floordiv(jlo, F.th), 0);
        int ty1 = min(floordiv(jhi, F.th), F.nty - 1);
        if (ty0 <= ty1) {
            S.k0 = k0;
            S.k1 = k1;
            S.ty0 = (int16_t)ty0;
            S.ty1 = (int16_t)ty1;
            if (table) {
                int ca = ext_cell(x_at(cx, t0, dt, k0), F.gsx, F.gx);
                int cb = ext_cell(x_at(cx, t0, dt, k1 - 1), F.gsx, F.gx);
                int ra = ext_cell(ymin, F.gsy, F.gy);
                int rb = ext_cell(ymax, F.gsy, F.gy);
                S.cx0 = (int8_t)ca;
                S.cx1 = (int8_t)cb;
                S.cy0 = (int8_t)ra;
                S.cy1 = (int8_t)rb;
            }
        }
    }
    F.segs[(size_t)c * F.ntr + tr] = S;
}

__global__ void k_fill_i32(int *p, int n, int v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Copies the frame record and spectrum pointers carried in the argument.
__global__ void k_put_params(FrameParams p, FrameDev *frame_dst, const void **spec_dst)
{
    const int t = threadIdx.x;
    if (t < p.nslots) spec_dst[t] = p.spec[t];
    if (t == 0) *frame_dst = p.f;
}

}  // namespace

hipError_t launch_put_params(const FrameParams &p, FrameDev *frame_dst, const void **spec_dst,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_put_params, dim3(1), dim3(kParamSlots), 0, s, p, frame_dst, spec_dst);
    return hipGetLastError();
}

hipError_t launch_plan(const FrameDev *frames_dev, const FrameDev *frames_host, int n_frames,
                       int *err, hipStream_t s)
{
    int maxw = 0;
    for (int f = 0; f < n_frames; ++f) maxw = max(maxw, frames_host[f].ntx * frames_host[f].ntr);
    if (maxw == 0) return hipSuccess;
    dim3 grid((maxw + 255) / 256, n_frames);
    hipLaunchKernelGGL(k_plan, grid, dim3(256), 0, s, frames_dev, err);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int n, int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace e2e
