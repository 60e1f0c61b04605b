// Closing the loop from the frame back to a radial velocity (Sec. 1: the
// simulated frames feed a data-reduction pipeline; Sec. 4.2: 1-D spectra
// extracted along the traced orders, the wavelength scale from the
// dispersion, the RV recovered by cross-correlation).
//
//  * k_extract: one thread per (trace, pixel column edge): the format
//    coordinate of the edge and of the column centre by safeguarded Newton
//    on x(t) (FP64), the edge wavelength, and the column's box extraction
//    over the rows within +-A of the trace centre (fractional end rows).
//    Neighbouring lanes read neighbouring pixels of each row.
//  * k_smooth3_fused / k_box_pass: the three passes of a clipped moving
//    mean over the template (the input spectrum of the trace); one
//    workgroup per 2048 outputs of a trace stages its inputs and the
//    windows around them in LDS, scans them (FP64) and takes window
//    differences -- all three passes in one launch when the window is
//    narrow (the template read once, the result written once), else one
//    launch per pass.
//  * k_ccf: one workgroup per (trace, 8 trial velocities): the mean of the
//    flat-divided flux over the usable columns, then per column and
//    velocity the template read at the Doppler-shifted column centre by
//    linear interpolation; fixed-order block sums.
#include "dev_common.h"

namespace e2e {

namespace {

// Format coordinate t in [-1, 1] with x(t) = xe, x increasing on [-1, 1]
// (xa = x(-1) <= xe <= xb = x(1)): Newton steps from the linear guess,
// kept inside the shrinking bracket (bisection when a step would leave it).
__device__ double t_at_x(const double *cx, double xe, double xa, double xb)
{
    double lo = -1.0, hi = 1.0;
    double t = xb > xa ? fma(2.0, (xe - xa) / (xb - xa), -1.0) : 0.0;
    t = fmin(fmax(t, lo), hi);
    for (int it = 0; it < 64; ++it) {
        double d;
        const double f = horner_d<kNCoef - 1>(cx, t, &d) - xe;
        if (f == 0.0) break;
        if (f < 0.0) lo = t;
        else hi = t;
        double tn = d > 0.0 ? t - f / d : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == t || hi - lo <= 0.0) break;
        t = tn;
    }
    return t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_extract(const TraceDev *__restrict__ trs, int nx, int ny,
                                                 const T *__restrict__ frame, double A,
                                                 double *__restrict__ flux,
                                                 double *__restrict__ edges)
{
    const int e = blockIdx.x * 256 + threadIdx.x, tr = blockIdx.y;
    if (e > nx) return;
    const TraceDev &Tr = trs[tr];
    const double xa = horner<kNCoef - 1>(Tr.cx, -1.0), xb = horner<kNCoef - 1>(Tr.cx, 1.0);
    const double span = Tr.lmax - Tr.lmin;
    const double xe = (double)e - 0.5;
    double lam = __builtin_nan("");
    if (xe >= xa && xe <= xb) {
        const double t = t_at_x(Tr.cx, xe, xa, xb);
        lam = 0.5 * fma(t, span, Tr.lmin + Tr.lmax);
    }
    edges[(size_t)tr * (nx + 1) + e] = lam;
    if (e == nx) return;
    const int i = e;
    double acc = 0.0;
    if ((double)i - 0.5 >= xa && (double)i + 0.5 <= xb) {
        const double yc = horner<kNCoef - 1>(Tr.cy, t_at_x(Tr.cx, (double)i, xa, xb));
        const double lo = yc - A, hi = yc + A;
        const int j0 = max(0, (int)floor(lo + 0.5)), j1 = min(ny - 1, (int)floor(hi + 0.5));
        for (int j = j0; j <= j1; ++j) {
            const double ov = fmin((double)j + 0.5, hi) - fmax((double)j - 0.5, lo);
            if (ov > 0.0) acc = fma(ov, (double)frame[(size_t)j * nx + i], acc);
        }
    }
    flux[(size_t)tr * nx + i] = acc;
}

// Per-trace parameters of the template smoothing and the CCF.
struct LoopTrace {
    const void *tmpl;   // template (spectrum slot), FP32 or FP64
    double *P;          // prefix sums, n + 1
    double *X;          // smoothed template, n
    int64_t n;
    int32_t w;          // moving-mean width (odd)
    int32_t pad;
};

constexpr int SMT = 2048;        // smoothed samples per workgroup
constexpr int SMW = 4095;        // widest moving mean

__device__ void lds_scan(double *q, int len, double *tsum)
{
    // q[1 .. len] -> inclusive prefix sums in place (q[0] = 0): each thread
    // sums a run of consecutive values, the run totals are scanned with wave
    // shuffles and the four wave totals (fixed order), then each thread
    // rewrites its run
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = (len + 255) / 256;
    const int a = 1 + tid * r, b = min(len + 1, a + r);
    double run = 0.0;
    for (int k = a; k < b; ++k) run += q[k];
    double x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) tsum[wv] = x;
    __syncthreads();
    double off = x - run;
    for (int u = 0; u < wv; ++u) off += tsum[u];
    for (int k = a; k < b; ++k) {
        off += q[k];
        q[k] = off;
    }
    __syncthreads();
}

// One moving-mean pass over a tile of SMT outputs of one trace: the tile's
// inputs with a half-window on each side are staged in LDS, scanned (FP64),
// and each output is the window sum (the
// window clipped to the array) over its count.  Pass 0 reads the template
// into X, pass 1 X into P, pass 2 P into X.
template <typename TT>
__global__ __launch_bounds__(256) void k_box_pass(const LoopTrace *__restrict__ lt, int pass)
{
    __shared__ double q[SMT + SMW + 1];
    __shared__ double tsum[4];
    const LoopTrace L = lt[blockIdx.y];
    const int64_t n = L.n, h = L.w / 2;
    const int64_t t0 = (int64_t)blockIdx.x * SMT;
    if (t0 >= n) return;
    const int64_t t1 = t0 + SMT < n ? t0 + SMT : n;
    const int64_t base = t0 - h > 0 ? t0 - h : 0, end = t1 + h < n ? t1 + h : n;
    const int len = (int)(end - base);
    const double *src = pass == 1 ? L.X : L.P;
    double *dst = pass == 1 ? L.P : L.X;
    const int tid = threadIdx.x;
    for (int k = tid; k < len; k += 256)
        q[k + 1] = pass == 0 ? (double)((const TT *)L.tmpl)[base + k] : src[base + k];
    if (tid == 0) q[0] = 0.0;
    __syncthreads();
    lds_scan(q, len, tsum);
    for (int64_t i = t0 + tid; i < t1; i += 256) {
        const int64_t lo = i - h > 0 ? i - h : 0, hi = i + h + 1 < n ? i + h + 1 : n;
        dst[i] = (q[hi - base] - q[lo - base]) / (double)(hi - lo);
    }
}

// All three passes in one launch when the windows are narrow (6h <= SMT):
// a workgroup loads its SMT outputs with 3h on each side, and pass k
// (k = 1, 2, 3) produces the range widened by (3 - k) h from the previous
// one in LDS (scan, window differences).  The template is read once and the
// smoothed template written once; the halo is recomputed by the neighbours.
constexpr int SFH = SMT / 6;     // widest half-window of the fused form

template <typename TT>
__global__ __launch_bounds__(256) void k_smooth3_fused(const LoopTrace *__restrict__ lt)
{
    __shared__ double qa[SMT + 6 * SFH + 2], qb[SMT + 6 * SFH + 2];
    __shared__ double tsum[4];
    const LoopTrace L = lt[blockIdx.y];
    const int64_t n = L.n, h = L.w / 2;
    const int64_t t0 = (int64_t)blockIdx.x * SMT;
    if (t0 >= n) return;
    const int64_t t1 = t0 + SMT < n ? t0 + SMT : n;
    const int tid = threadIdx.x;
    int64_t b = t0 - 3 * h > 0 ? t0 - 3 * h : 0, e = t1 + 3 * h < n ? t1 + 3 * h : n;
    int len = (int)(e - b);
    for (int k = tid; k < len; k += 256) qa[k + 1] = (double)((const TT *)L.tmpl)[b + k];
    if (tid == 0) qa[0] = 0.0;
    __syncthreads();
    double *src = qa, *dst = qb;
    for (int pass = 1; pass <= 3; ++pass) {
        lds_scan(src, len, tsum);
        const int64_t wb = (int64_t)(3 - pass) * h;
        const int64_t nb = t0 - wb > 0 ? t0 - wb : 0, ne = t1 + wb < n ? t1 + wb : n;
        const int nlen = (int)(ne - nb);
        for (int k = tid; k < nlen; k += 256) {
            const int64_t i = nb + k;
            const int64_t lo = i - h > 0 ? i - h : 0, hi = i + h + 1 < n ? i + h + 1 : n;
            const double v = (src[hi - b] - src[lo - b]) / (double)(hi - lo);
            if (pass < 3) dst[k + 1] = v;
            else L.X[i] = v;
        }
        if (tid == 0) dst[0] = 0.0;
        __syncthreads();
        double *t = src;
        src = dst;
        dst = t;
        b = nb;
        len = nlen;
    }
}

constexpr int KV = 8;   // trial velocities per workgroup

__global__ __launch_bounds__(256) void k_ccf(const TraceDev *__restrict__ trs, int tr0,
                                             const LoopTrace *__restrict__ lt, int nx,
                                             const double *__restrict__ flux,
                                             const double *__restrict__ flat,
                                             const double *__restrict__ edges, double v0,
                                             double dv, int nv, double *__restrict__ C)
{
    __shared__ double red[KV][256];
    __shared__ double sh_mean;
    const int tid = threadIdx.x, g = blockIdx.y, tr = tr0 + g, k0 = blockIdx.x * KV;
    const TraceDev &Tr = trs[tr];
    const LoopTrace L = lt[g];
    const double c = 299792458.0;
    const double vlo = fmin(v0, v0 + (nv - 1) * dv), vhi = fmax(v0, v0 + (nv - 1) * dv);
    const double bmin = vlo / c, bmax = vhi / c;
    const double dl = (Tr.lmax - Tr.lmin) / (double)L.n;
    const int h = L.w / 2;
    const double ulo = 6.0 * h, uhi = (double)(L.n - 2 - 6 * h);
    const double *Ft = flux + (size_t)tr * nx, *Lt = edges + (size_t)tr * (nx + 1);
    const double *Ff = flat ? flat + (size_t)tr * nx : nullptr;
    auto usable = [&](int i, double *lc) {
        const double a = Lt[i], b = Lt[i + 1];
        if (isnan(a) || isnan(b)) return false;
        if (Ff && !(Ff[i] > 0.0)) return false;
        *lc = 0.5 * (a + b);
        return (*lc / (1.0 + bmax) - Tr.lmin) / dl - 0.5 >= ulo &&
               (*lc / (1.0 + bmin) - Tr.lmin) / dl - 0.5 <= uhi;
    };
    // mean of e over the usable columns
    double s = 0.0, cnt = 0.0;
    for (int i = tid; i < nx; i += 256) {
        double lc;
        if (usable(i, &lc)) {
            s += Ff ? Ft[i] / Ff[i] : Ft[i];
            cnt += 1.0;
        }
    }
    red[0][tid] = s;
    red[1][tid] = cnt;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            red[0][tid] += red[0][tid + o];
            red[1][tid] += red[1][tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) sh_mean = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;
    __syncthreads();
    const double mean = sh_mean;
    double acc[KV];
#pragma unroll
    for (int q = 0; q < KV; ++q) acc[q] = 0.0;
    for (int i = tid; i < nx; i += 256) {
        double lc;
        if (!usable(i, &lc)) continue;
        const double e = (Ff ? Ft[i] / Ff[i] : Ft[i]) - mean;
#pragma unroll
        for (int q = 0; q < KV; ++q) {
            const int k = k0 + q;
            if (k >= nv) break;
            const double beta = (v0 + k * dv) / c;
            const double u = (lc / (1.0 + beta) - Tr.lmin) / dl - 0.5;
            const int64_t m = (int64_t)floor(u);
            const double f = u - (double)m;
            acc[q] = fma(e, fma(L.X[m + 1] - L.X[m], f, L.X[m]), acc[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KV; ++q) red[q][tid] = acc[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o)
#pragma unroll
            for (int q = 0; q < KV; ++q) red[q][tid] += red[q][tid + o];
        __syncthreads();
    }
    if (tid < KV && k0 + tid < nv) C[(size_t)tr * nv + k0 + tid] = red[tid][0];
}

}  // namespace

hipError_t launch_extract(const TraceDev *trs, int ntr, int nx, int ny, const void *frame,
                          int f64, double A, double *flux, double *edges, hipStream_t s)
{
    if (ntr <= 0 || nx <= 0) return hipSuccess;
    const dim3 grid((nx + 1 + 255) / 256, ntr);
    if (f64)
        hipLaunchKernelGGL(k_extract<double>, grid, dim3(256), 0, s, trs, nx, ny,
                           (const double *)frame, A, flux, edges);
    else
        hipLaunchKernelGGL(k_extract<float>, grid, dim3(256), 0, s, trs, nx, ny,
                           (const float *)frame, A, flux, edges);
    return hipGetLastError();
}

hipError_t launch_smooth3(const void *lt_dev, int ntr, int64_t nmax, int wmax, int f64,
                          hipStream_t s)
{
    if (ntr <= 0 || nmax <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nmax + SMT - 1) / SMT), ntr);
    if (wmax / 2 <= SFH) {
        if (f64)
            hipLaunchKernelGGL(k_smooth3_fused<double>, grid, dim3(256), 0, s,
                               (const LoopTrace *)lt_dev);
        else
            hipLaunchKernelGGL(k_smooth3_fused<float>, grid, dim3(256), 0, s,
                               (const LoopTrace *)lt_dev);
        return hipGetLastError();
    }
    for (int pass = 0; pass < 3; ++pass) {
        if (f64)
            hipLaunchKernelGGL(k_box_pass<double>, grid, dim3(256), 0, s,
                               (const LoopTrace *)lt_dev, pass);
        else
            hipLaunchKernelGGL(k_box_pass<float>, grid, dim3(256), 0, s,
                               (const LoopTrace *)lt_dev, pass);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int loop_max_width() { return SMW; }

hipError_t launch_ccf(const TraceDev *trs, int tr0, int ntr, const void *lt_dev, int nx,
                      const double *flux, const double *flat, const double *edges, double v0,
                      double dv, int nv, double *C, hipStream_t s)
{
    if (ntr <= 0) return hipSuccess;
    const dim3 grid((nv + KV - 1) / KV, ntr);
    hipLaunchKernelGGL(k_ccf, grid, dim3(256), 0, s, trs, tr0, (const LoopTrace *)lt_dev, nx,
                       flux, flat, edges, v0, dv, nv, C);
    return hipGetLastError();
}

size_t loop_trace_bytes() { return sizeof(LoopTrace); }

void loop_trace_fill(void *dst, const void *tmpl, double *P, double *X, int64_t n, int w)
{
    LoopTrace L;
    L.tmpl = tmpl;
    L.P = P;
    L.X = X;
    L.n = n;
    L.w = w;
    L.pad = 0;
    *(LoopTrace *)dst = L;
}

}  // namespace e2e
