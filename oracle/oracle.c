/*
 * FP64 CPU oracle of the echellogram renderer -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library.  The GPU library never calls it and
 * shares no code, header or table with it.
 *
 * What it computes is the plain definition of the paper's frame (Genoni et
 * al. 2020, Sec. 2 and Sec. 2.2): the synthetic echellogram is the
 * superposition, over every wavelength sample of every spectral trace, of
 * that sample's photons spread by the PSF and integrated over the area of
 * each detector pixel.  One sample at a time, in FP64, traces in ascending
 * order and samples in ascending order within a trace; nothing is blocked,
 * fused or reordered.
 *
 * Readings of points the paper leaves open (each one listed in the design
 * notes with its justification):
 *   - pixel (i, j) covers [i-1/2, i+1/2) x [j-1/2, j+1/2), frame [y][x];
 *   - sample k of a trace sits at lmin + (k+1/2)(lmax-lmin)/n (cell-centred
 *     uniform grid; Sec. 2.1 only says the step is a fraction of the
 *     resolution element);
 *   - the Doppler shift moves each sample to lambda (1 + v/c);
 *   - the spectral format (Sec. 2.1's per-SFI centroid) is a polynomial in
 *     t = (2 lambda' - lmin - lmax) / (lmax - lmin);
 *   - the analytic PSF (Sec. 2.1: a Gaussian) is integrated exactly over
 *     each pixel by differences of the normal CDF, truncated to a
 *     (2H+1)^2 window around floor(x+1/2) and renormalised by the window sum;
 *   - a tabulated PSF map holds cell integrals (piecewise-constant density)
 *     centred on the table centre; its value at a field point is the
 *     bilinear interpolation of the node maps at that sample's (x, y); the
 *     pixel weight is the exact box overlap of every cell with the pixel;
 *   - a separable PSF interpolates (sigma_x, sigma_y) bilinearly and then
 *     integrates each axis like the analytic case;
 *   - an explicit SFI (Sec. 2.2: the surface integral of the fiber's spatial
 *     profile convolved with the PSF, on a sub-pixel grid) takes the fiber
 *     image as a uniform disc of radius rho (or the half of it on one side
 *     of the trace's y) centred on the sample position, the PSF as the
 *     separable case's Gaussian, and the pixel value as the mean of the
 *     convolution at the centres of S x S sub-pixels (S = 10 in the paper:
 *     0.1-px sampling), over the (2H+1)^2 window, renormalised by the
 *     window sum;
 *   - flux of pixels off the detector is dropped, never renormalised;
 *   - photon noise (Sec. 2.2: added on the final frame) is Poisson with the
 *     expected count as mean, drawn from Philox-4x32-10 (Salmon et al.,
 *     SC'11) uniforms; small means use Knuth's multiplication method
 *     (TAOCP vol. 2, 3.4.1), large means Hormann's PTRS transformed
 *     rejection (Insurance: Math. & Econ. 12, 1993).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXDEG 7
#define ORC_NCOEF 8

typedef struct {
    int n_traces;
    const int *deg_x, *deg_y;   /* [n_traces] */
    const double *cx, *cy;      /* [n_traces][8], ascending powers of t */
    const double *lmin, *lmax;  /* [n_traces] nm */
    const int64_t *n;           /* [n_traces] samples */
    const double *thr;          /* [n_traces] throughput */
    const int *slot;            /* [n_traces] spectrum slot */
    const double *spec;         /* all slots concatenated, photons / sample */
    const int64_t *spec_off;    /* [n_slots] offset of each slot in spec */
    int nx, ny;
} orc_scene;

typedef struct {
    int kind;            /* 0 erf Gaussian, 1 table, 2 separable */
    double sigma;        /* erf */
    int half_width;      /* erf / separable footprint radius H */
    int gx, gy;          /* field node grid */
    int kw, kh, os;      /* table cells and cells per pixel */
    const float *tables; /* [gy][gx][kh][kw] */
    const float *sigma_xy; /* [gy][gx][2] */
    double fiber_radius; /* sfi: radius of the fiber image (px)            */
    int fiber_shape;     /* sfi: 0 disc, 1 half b >= 0, 2 half b <= 0      */
    int subpix;          /* sfi: sub-pixels per pixel side                  */
} orc_psf;

static const double C_LIGHT = 299792458.0;

/* ---------------------------------------------------------------- format */

static double horner(const double *c, int deg, double t)
{
    double v = c[deg];
    for (int j = deg - 1; j >= 0; --j) v = v * t + c[j];
    return v;
}

/* Sample k of trace tr, Doppler factor (1 + beta): detector position. */
static void position(const orc_scene *s, int tr, int64_t k, double beta,
                     double *x, double *y)
{
    double lmin = s->lmin[tr], lmax = s->lmax[tr];
    double dl = (lmax - lmin) / (double)s->n[tr];
    double lam = lmin + ((double)k + 0.5) * dl;
    double lam2 = lam * (1.0 + beta);
    double t = (2.0 * lam2 - lmin - lmax) / (lmax - lmin);
    *x = horner(s->cx + ORC_NCOEF * tr, s->deg_x[tr], t);
    *y = horner(s->cy + ORC_NCOEF * tr, s->deg_y[tr], t);
}

/* ------------------------------------------------------------ PSF pieces */

/* Phi(b) - Phi(a) for the standard normal CDF, evaluated on the side of the
 * distribution where it does not cancel. */
static double dphi(double a, double b)
{
    const double r = 0.70710678118654752440; /* 1/sqrt(2) */
    if (a >= 0.0) return 0.5 * (erfc(a * r) - erfc(b * r));
    if (b <= 0.0) return 0.5 * (erfc(-b * r) - erfc(-a * r));
    return 0.5 * (erf(b * r) - erf(a * r));
}

/* Bilinear node weights at (x, y) over a g x g grid spanning the detector
 * edge to edge (node m at m (n-1)/(g-1)); returns the lower node index and
 * the fraction towards the next node, clamped at the edges. */
static void node_frac(double p, int npix, int g, int *c, double *f)
{
    if (g < 2) { *c = 0; *f = 0.0; return; }
    double sp = p * (double)(g - 1) / (double)(npix - 1);
    if (sp < 0.0) sp = 0.0;
    if (sp > (double)(g - 1)) sp = (double)(g - 1);
    int ci = (int)floor(sp);
    if (ci > g - 2) ci = g - 2;
    *c = ci;
    *f = sp - (double)ci;
}

/* Per-axis normalised pixel integrals of a Gaussian centred at p with sigma
 * sg over the window [a-H, a+H], a = floor(p + 1/2). */
static int erf_axis(double p, double sg, int H, double *e)
{
    int a = (int)floor(p + 0.5);
    double norm = dphi(((double)(a - H) - 0.5 - p) / sg,
                       ((double)(a + H) + 0.5 - p) / sg);
    for (int d = -H; d <= H; ++d) {
        double lo = ((double)(a + d) - 0.5 - p) / sg;
        double hi = ((double)(a + d) + 0.5 - p) / sg;
        e[d + H] = dphi(lo, hi) / norm;
    }
    return a - H;
}

static double overlap(double lo1, double hi1, double lo2, double hi2)
{
    double lo = lo1 > lo2 ? lo1 : lo2;
    double hi = hi1 < hi2 ? hi1 : hi2;
    return hi > lo ? hi - lo : 0.0;
}

/* Gauss-Legendre nodes and weights on [-1, 1] (n <= 128): Newton's
 * iteration on the three-term recurrence of the Legendre polynomials from
 * the Chebyshev-like first guesses cos(pi (i + 3/4) / (n + 1/2)). */
static void gauss_legendre(int n, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(pi * ((double)i + 0.75) / ((double)n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

#define ORC_SFI_NQ 48

/*
 * Fiber image (uniform disc of radius rho, area A; or one half of it, area
 * A/2) convolved with the axis-aligned Gaussian of (sx, sy): the photon
 * density at offset (u, v) from the disc centre,
 *   C(u, v) = (1/A_D) int_D N(u - a; sx) N(v - b; sy) da db.
 * With a = rho sin(th) the chord of the disc at a is b in [-h, h],
 * h = rho cos(th) ([0, h] or [-h, 0] for the halves); the b integral is a
 * normal-CDF difference and the th integral, over [-pi/2, pi/2], has a
 * smooth integrand and is taken with ORC_SFI_NQ Gauss-Legendre points
 * (converged to rounding for rho / sigma <= 4).
 */
static double sfi_density(double u, double v, double rho, int shape, double sx, double sy,
                          const double *qx, const double *qw)
{
    const double pi = 3.14159265358979323846;
    double area = pi * rho * rho * (shape ? 0.5 : 1.0);
    double acc = 0.0;
    for (int q = 0; q < ORC_SFI_NQ; ++q) {
        double th = 0.5 * pi * qx[q];
        double a = rho * sin(th), h = rho * cos(th);
        double lo = shape == 1 ? 0.0 : -h, hi = shape == 2 ? 0.0 : h;
        double ga = exp(-0.5 * ((u - a) / sx) * ((u - a) / sx)) / (sqrt(2.0 * pi) * sx);
        double gb = dphi((v - hi) / sy, (v - lo) / sy);
        acc += 0.5 * pi * qw[q] * h * ga * gb;   /* da = rho cos(th) dth = h dth */
    }
    return acc / area;
}

/* Pixel weights of an explicit SFI centred at (x, y) over the window
 * [a-H, a+H] x [b-H, b+H], a = floor(x+1/2), b = floor(y+1/2): the mean of
 * sfi_density over the S x S sub-pixel centres of each pixel, renormalised
 * by the window sum. */
static void sfi_window(double x, double y, double rho, int shape, int S, double sx, double sy,
                       int H, int *i0, int *j0, double *wt)
{
    double qx[ORC_SFI_NQ], qw[ORC_SFI_NQ];
    gauss_legendre(ORC_SFI_NQ, qx, qw);
    int a = (int)floor(x + 0.5), b = (int)floor(y + 0.5), n = 2 * H + 1;
    double tot = 0.0;
    for (int jj = 0; jj < n; ++jj)
        for (int ii = 0; ii < n; ++ii) {
            double acc = 0.0;
            for (int t = 0; t < S; ++t) {
                double v = (double)(b - H + jj) - 0.5 + ((double)t + 0.5) / S - y;
                for (int s2 = 0; s2 < S; ++s2) {
                    double u = (double)(a - H + ii) - 0.5 + ((double)s2 + 0.5) / S - x;
                    acc += sfi_density(u, v, rho, shape, sx, sy, qx, qw);
                }
            }
            wt[jj * n + ii] = acc / ((double)S * S);
            tot += wt[jj * n + ii];
        }
    for (int q = 0; q < n * n; ++q) wt[q] /= tot;
    *i0 = a - H;
    *j0 = b - H;
}

/*
 * Footprint of one sample at (x, y): the weight of every pixel of a
 * (*w) x (*h) box whose lower-left pixel is (*i0, *j0).  Off-detector pixels
 * are included here; callers drop them.  `wt` needs room for the largest
 * footprint (orc_footprint_cap).  Returns 0 on success.
 */
int orc_sample_weights(const orc_psf *p, int nx, int ny, double x, double y,
                       int *i0, int *j0, int *w, int *h, double *wt)
{
    if (p->kind == 0 || p->kind == 2 || p->kind == 3) {
        double sx = p->sigma, sy = p->sigma;
        if (p->kind == 2 || p->kind == 3) {
            int cx, cy; double fx, fy;
            node_frac(x, nx, p->gx, &cx, &fx);
            node_frac(y, ny, p->gy, &cy, &fy);
            int cx1 = cx + (p->gx > 1), cy1 = cy + (p->gy > 1);
            const float *s = p->sigma_xy;
#define SXY(l, m, c) ((double)s[(((size_t)(l) * p->gx + (m)) * 2) + (c)])
            sx = (1 - fx) * (1 - fy) * SXY(cy, cx, 0) + fx * (1 - fy) * SXY(cy, cx1, 0)
               + (1 - fx) * fy * SXY(cy1, cx, 0) + fx * fy * SXY(cy1, cx1, 0);
            sy = (1 - fx) * (1 - fy) * SXY(cy, cx, 1) + fx * (1 - fy) * SXY(cy, cx1, 1)
               + (1 - fx) * fy * SXY(cy1, cx, 1) + fx * fy * SXY(cy1, cx1, 1);
#undef SXY
        }
        int H = p->half_width, n = 2 * H + 1;
        double ex[2 * 64 + 1], ey[2 * 64 + 1];
        if (H > 64) return -1;
        if (p->kind == 3) {
            if (!(p->fiber_radius > 0.0) || p->subpix < 1 || p->fiber_shape < 0 ||
                p->fiber_shape > 2)
                return -1;
            sfi_window(x, y, p->fiber_radius, p->fiber_shape, p->subpix, sx, sy, H, i0, j0, wt);
            *w = n; *h = n;
            return 0;
        }
        *i0 = erf_axis(x, sx, H, ex);
        *j0 = erf_axis(y, sy, H, ey);
        *w = n; *h = n;
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) wt[b * n + a] = ey[b] * ex[a];
        return 0;
    }
    if (p->kind != 1) return -1;

    /* interpolated kernel K = sum_n w_n K_n at this field point */
    int kw = p->kw, kh = p->kh, os = p->os;
    int cx, cy; double fx, fy;
    node_frac(x, nx, p->gx, &cx, &fx);
    node_frac(y, ny, p->gy, &cy, &fy);
    int cx1 = cx + (p->gx > 1), cy1 = cy + (p->gy > 1);
    size_t ksz = (size_t)kw * kh;
    const float *K00 = p->tables + ((size_t)cy * p->gx + cx) * ksz;
    const float *K10 = p->tables + ((size_t)cy * p->gx + cx1) * ksz;
    const float *K01 = p->tables + ((size_t)cy1 * p->gx + cx) * ksz;
    const float *K11 = p->tables + ((size_t)cy1 * p->gx + cx1) * ksz;
    double *K = (double *)malloc(sizeof(double) * ksz);
    for (size_t q = 0; q < ksz; ++q)
        K[q] = (1 - fx) * (1 - fy) * (double)K00[q] + fx * (1 - fy) * (double)K10[q]
             + (1 - fx) * fy * (double)K01[q] + fx * fy * (double)K11[q];

    /* cell a spans [L + a/os, L + (a+1)/os) with L = x - kw/(2 os) */
    double Lx = x - (double)kw / (2.0 * os), Ly = y - (double)kh / (2.0 * os);
    int ia = (int)floor(Lx + 0.5) - 1, ib = (int)floor(Lx + (double)kw / os + 0.5) + 1;
    int ja = (int)floor(Ly + 0.5) - 1, jb = (int)floor(Ly + (double)kh / os + 0.5) + 1;
    int W = ib - ia + 1, Hh = jb - ja + 1;
    /* box overlaps of every cell with every pixel, per axis (x os); a cell
     * is os^-1 px wide so it meets at most two pixels: keep those pairs */
    int *pxa = (int *)malloc(sizeof(int) * 2 * kw), *pya = (int *)malloc(sizeof(int) * 2 * kh);
    double *ovx = (double *)malloc(sizeof(double) * 2 * kw);
    double *ovy = (double *)malloc(sizeof(double) * 2 * kh);
    for (int a = 0; a < kw; ++a) {
        int m = 0;
        pxa[2 * a] = pxa[2 * a + 1] = 0;
        ovx[2 * a] = ovx[2 * a + 1] = 0.0;
        for (int i = ia; i <= ib && m < 2; ++i) {
            double ov = overlap(Lx + (double)a / os, Lx + (double)(a + 1) / os, i - 0.5, i + 0.5) * os;
            if (ov != 0.0) { pxa[2 * a + m] = i - ia; ovx[2 * a + m] = ov; ++m; }
        }
    }
    for (int b = 0; b < kh; ++b) {
        int m = 0;
        pya[2 * b] = pya[2 * b + 1] = 0;
        ovy[2 * b] = ovy[2 * b + 1] = 0.0;
        for (int j = ja; j <= jb && m < 2; ++j) {
            double ov = overlap(Ly + (double)b / os, Ly + (double)(b + 1) / os, j - 0.5, j + 0.5) * os;
            if (ov != 0.0) { pya[2 * b + m] = j - ja; ovy[2 * b + m] = ov; ++m; }
        }
    }
    /* w_ij = sum_b sum_a K[b][a] ovx[a][i] ovy[b][j]
     *      = sum_b ovy[b][j] T[b][i],  T[b][i] = sum_a K[b][a] ovx[a][i] */
    double *T = (double *)calloc((size_t)kh * W, sizeof(double));
    for (int b = 0; b < kh; ++b)
        for (int a = 0; a < kw; ++a)
            for (int e = 0; e < 2; ++e)
                T[(size_t)b * W + pxa[2 * a + e]] += K[(size_t)b * kw + a] * ovx[2 * a + e];
    for (size_t q = 0; q < (size_t)W * Hh; ++q) wt[q] = 0.0;
    for (int b = 0; b < kh; ++b)
        for (int e = 0; e < 2; ++e) {
            double ov = ovy[2 * b + e];
            if (ov == 0.0) continue;
            int j = pya[2 * b + e];
            for (int i = 0; i < W; ++i) wt[(size_t)j * W + i] += ov * T[(size_t)b * W + i];
        }
    free(pxa);
    free(pya);
    free(ovx);
    free(ovy);
    free(T);
    free(K);
    *i0 = ia; *j0 = ja; *w = W; *h = Hh;
    return 0;
}

/* C(u, v) of sfi_density, for the pins. */
double orc_sfi_density(double u, double v, double rho, int shape, double sx, double sy)
{
    double qx[ORC_SFI_NQ], qw[ORC_SFI_NQ];
    gauss_legendre(ORC_SFI_NQ, qx, qw);
    return sfi_density(u, v, rho, shape, sx, sy, qx, qw);
}

/* Gauss-Legendre rule of n points, for the pins. */
void orc_gauss_legendre(int n, double *x, double *w)
{
    if (n >= 1 && n <= 128) gauss_legendre(n, x, w);
}

int orc_footprint_cap(const orc_psf *p)
{
    if (p->kind == 1) {
        int W = p->kw / p->os + 4, H = p->kh / p->os + 4;
        return W * H;
    }
    return (2 * p->half_width + 1) * (2 * p->half_width + 1);
}

/* ----------------------------------------------------------------- frames */

/* Accumulate traces [tr_lo, tr_hi) into frame[ny][nx] (caller zeroes it). */
int orc_render(const orc_scene *s, const orc_psf *p, double rv_mps,
               double flux_scale, int tr_lo, int tr_hi, double *frame)
{
    double beta = rv_mps / C_LIGHT;
    double *wt = (double *)malloc(sizeof(double) * orc_footprint_cap(p));
    if (!wt) return -1;
    for (int tr = tr_lo; tr < tr_hi; ++tr) {
        const double *S = s->spec + s->spec_off[s->slot[tr]];
        double scale = s->thr[tr] * flux_scale;
        for (int64_t k = 0; k < s->n[tr]; ++k) {
            double x, y;
            position(s, tr, k, beta, &x, &y);
            double phi = S[k] * scale;
            int i0, j0, w, h;
            if (orc_sample_weights(p, s->nx, s->ny, x, y, &i0, &j0, &w, &h, wt)) {
                free(wt);
                return -1;
            }
            for (int b = 0; b < h; ++b) {
                int j = j0 + b;
                if (j < 0 || j >= s->ny) continue;
                for (int a = 0; a < w; ++a) {
                    int i = i0 + a;
                    if (i < 0 || i >= s->nx) continue;
                    frame[(size_t)j * s->nx + i] += phi * wt[b * w + a];
                }
            }
        }
    }
    free(wt);
    return 0;
}

/* First k in [lo, hi] with x(k) >= xv (x increasing in k). */
static int64_t first_k_at_or_above(const orc_scene *s, int tr, double beta,
                                   double xv, int64_t lo, int64_t hi)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        double x, y;
        position(s, tr, mid, beta, &x, &y);
        if (x >= xv) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/*
 * The same frame evaluated at chosen pixels only.  For each pixel, every
 * trace contributes the samples whose footprint can reach that pixel; x is
 * increasing along a trace, so those samples form one index range found by
 * bisection.  Samples outside it have zero weight on the pixel.
 */
int orc_render_pixels(const orc_scene *s, const orc_psf *p, double rv_mps,
                      double flux_scale, int npix, const int *px,
                      const int *py, double *out)
{
    double beta = rv_mps / C_LIGHT;
    double reach;
    if (p->kind == 1) {
        int kmax = p->kw > p->kh ? p->kw : p->kh;
        reach = 0.5 * ((double)kmax / p->os) + 2.0;
    } else {
        reach = (double)p->half_width + 2.0;
    }
    double *wt = (double *)malloc(sizeof(double) * orc_footprint_cap(p));
    if (!wt) return -1;
    for (int q = 0; q < npix; ++q) {
        int i = px[q], j = py[q];
        double acc = 0.0;
        for (int tr = 0; tr < s->n_traces; ++tr) {
            int64_t n = s->n[tr];
            int64_t ka = first_k_at_or_above(s, tr, beta, i - reach, 0, n);
            int64_t kb = first_k_at_or_above(s, tr, beta, i + reach, ka, n);
            const double *S = s->spec + s->spec_off[s->slot[tr]];
            double scale = s->thr[tr] * flux_scale;
            for (int64_t k = ka; k < kb; ++k) {
                double x, y;
                position(s, tr, k, beta, &x, &y);
                if (fabs(y - j) > reach) continue;
                int i0, j0, w, h;
                if (orc_sample_weights(p, s->nx, s->ny, x, y, &i0, &j0, &w, &h, wt)) {
                    free(wt);
                    return -1;
                }
                if (i < i0 || i >= i0 + w || j < j0 || j >= j0 + h) continue;
                acc += S[k] * scale * wt[(j - j0) * w + (i - i0)];
            }
        }
        out[q] = acc;
    }
    free(wt);
    return 0;
}

/* Detector positions of samples k0 .. k0+count-1 of one trace. */
void orc_positions(const orc_scene *s, int tr, double rv_mps, int64_t k0,
                   int64_t count, double *x, double *y)
{
    double beta = rv_mps / C_LIGHT;
    for (int64_t q = 0; q < count; ++q) position(s, tr, k0 + q, beta, x + q, y + q);
}

/* ------------------------------------------------------------ photon noise */

/* Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
        x0 = n0; x1 = lo1; x2 = n2; x3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Raw stream: block b of pixel p is Philox(ctr = (p lo, p hi, frame, b)). */
void orc_philox_blocks(uint64_t seed, uint32_t frame, uint64_t pixel,
                       uint32_t nblocks, uint32_t *out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t b = 0; b < nblocks; ++b) {
        uint32_t ctr[4] = {(uint32_t)pixel, (uint32_t)(pixel >> 32), frame, b};
        orc_philox4x32_10(ctr, key, out + 4 * b);
    }
}

typedef struct {
    uint32_t key[2], ctr[4];
    uint32_t buf[4];
    int have;     /* uniforms left in buf: 2, 1 or 0 */
} orc_stream;

/* 53-bit uniform in (0, 1) from two 32-bit words. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 9007199254740992.0);
}

static double next_uniform(orc_stream *st)
{
    if (st->have == 0) {
        orc_philox4x32_10(st->ctr, st->key, st->buf);
        st->ctr[3] += 1;
        st->have = 2;
    }
    double u = (st->have == 2) ? u53(st->buf[0], st->buf[1]) : u53(st->buf[2], st->buf[3]);
    st->have -= 1;
    return u;
}

static double poisson_draw(double mean, orc_stream *st)
{
    if (!(mean > 0.0)) return 0.0;
    if (mean < 10.0) {
        /* Knuth: multiply uniforms until the product drops below exp(-mean) */
        double L = exp(-mean), prod = next_uniform(st);
        double k = 0.0;
        while (prod > L) { k += 1.0; prod *= next_uniform(st); }
        return k;
    }
    /* Hormann's PTRS */
    double slam = sqrt(mean), loglam = log(mean);
    double b = 0.931 + 2.53 * slam;
    double a = -0.059 + 0.02483 * b;
    double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (;;) {
        double U = next_uniform(st) - 0.5;
        double V = next_uniform(st);
        double us = 0.5 - fabs(U);
        double k = floor((2.0 * a / us + b) * U + mean + 0.43);
        if (us >= 0.07 && V <= vr) return k;
        if (k < 0.0 || (us < 0.013 && V > us)) continue;
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <=
            -mean + k * loglam - lgamma(k + 1.0))
            return k;
    }
}

/* out[p] = Poisson(mean[p]) with stream (seed, frame, pixel p). */
void orc_poisson_frame(const double *mean, int64_t n, uint64_t seed,
                       uint32_t frame, double *out)
{
    for (int64_t p = 0; p < n; ++p) {
        orc_stream st;
        st.key[0] = (uint32_t)seed; st.key[1] = (uint32_t)(seed >> 32);
        st.ctr[0] = (uint32_t)p; st.ctr[1] = (uint32_t)((uint64_t)p >> 32);
        st.ctr[2] = frame; st.ctr[3] = 0;
        st.have = 0;
        out[p] = poisson_draw(mean[p], &st);
    }
}

/* ---------------------------------------------------------- detector stage */

/*
 * The detector stage that Sec. 2.2 applies to the final echellogram (photon
 * noise, dark current, read-out noise, pixel response non-uniformity,
 * cross-talk), in this order per pixel p = j nx + i:
 *   mu = G[p] F[p] + dark t          (PRNU gain map G, 1 if absent)
 *   N  = Poisson(mu) (stream blocks 0, 1, ...) or mu without shot noise
 *   E  = sum over dy, dx in -1..1 (dy outer) of K[dy+1][dx+1] N[p - (dx, dy)],
 *        FP64 fma in that order, pixels off the detector contributing 0
 *        (charge leaking off the chip is lost)
 *   R  = E + ron Z, Z = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller) from
 *        Philox block 2^31 of the pixel's stream: u1 from its words 0-1,
 *        u2 from words 2-3 (a counter range the Poisson draws never reach)
 *   ADU = min(max(floor(R / gain + bias + 1/2), 0), 2^bits - 1)
 * Computed for the window [x0, x0+w) x [y0, y0+h) of an nx x ny frame;
 * r_out (optional) receives R.
 */
void orc_detector(const double *F, const double *G, int nx, int ny, int x0, int y0, int w,
                  int h, double exposure_s, double dark_e_per_s, int shot_noise,
                  const double *K, double ron_e, double gain, double bias, int bits,
                  uint64_t seed, uint32_t frame, uint16_t *adu_out, double *r_out)
{
    const double dt = dark_e_per_s * exposure_s;
    const double top = (double)((1u << bits) - 1u);
    /* electrons of the window and its one-pixel border */
    int bx0 = x0 - 1, by0 = y0 - 1, bw = w + 2, bh = h + 2;
    double *N = (double *)calloc((size_t)bw * bh, sizeof(double));
    for (int j = 0; j < bh; ++j) {
        int gy = by0 + j;
        if (gy < 0 || gy >= ny) continue;
        for (int i = 0; i < bw; ++i) {
            int gx = bx0 + i;
            if (gx < 0 || gx >= nx) continue;
            int64_t p = (int64_t)gy * nx + gx;
            double g = G ? G[p] : 1.0;
            double mu = fma(g, F[p], dt);
            if (shot_noise) {
                orc_stream st;
                st.key[0] = (uint32_t)seed; st.key[1] = (uint32_t)(seed >> 32);
                st.ctr[0] = (uint32_t)p; st.ctr[1] = (uint32_t)((uint64_t)p >> 32);
                st.ctr[2] = frame; st.ctr[3] = 0;
                st.have = 0;
                N[(size_t)j * bw + i] = poisson_draw(mu, &st);
            } else {
                N[(size_t)j * bw + i] = mu;
            }
        }
    }
    for (int j = 0; j < h; ++j) {
        for (int i = 0; i < w; ++i) {
            int gx = x0 + i, gy = y0 + j;
            int64_t p = (int64_t)gy * nx + gx;
            double e = 0.0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    /* source pixel (gx - dx, gy - dy) in border coordinates */
                    int si = (gx - dx) - bx0, sj = (gy - dy) - by0;
                    e = fma(K[(dy + 1) * 3 + (dx + 1)], N[(size_t)sj * bw + si], e);
                }
            double r = e;
            if (ron_e > 0.0) {
                uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
                uint32_t ctr[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), frame, 0x80000000u};
                uint32_t b[4];
                orc_philox4x32_10(ctr, key, b);
                double u1 = u53(b[0], b[1]), u2 = u53(b[2], b[3]);
                double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                r = fma(ron_e, z, e);
            }
            if (r_out) r_out[(size_t)j * w + i] = r;
            double v = floor(r / gain + bias + 0.5);
            if (v < 0.0) v = 0.0;
            if (v > top) v = top;
            adu_out[(size_t)j * w + i] = (uint16_t)v;
        }
    }
    free(N);
}

/* ------------------------------------------- 1-D extraction and the CCF */

/*
 * Closing the loop from the 2-D frame back to a 1-D spectrum and a radial
 * velocity (Sec. 1: the simulator's frames feed a data-reduction pipeline;
 * Sec. 4.2: spectra extracted along the traced orders, wavelength scale
 * from the dispersion, RV recovered by cross-correlation).
 *
 * Detector-frame wavelength of a format coordinate t: lambda(t) =
 * (t (lmax - lmin) + lmin + lmax) / 2.  The trace's x(t) increases with t
 * on [-1, 1]; the t where x(t) = e is found by bisection (to the last bit).
 */
static double t_at_x(const orc_scene *s, int tr, double e)
{
    const double *cx = s->cx + ORC_NCOEF * tr;
    int dx = s->deg_x[tr];
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (horner(cx, dx, mid) < e) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/*
 * Box extraction of every trace: for pixel column i whose edges i -+ 1/2
 * both fall inside the trace's x range, the trace centre y_c = y(t) at
 * x(t) = i and
 *   E[tr][i] = sum_j |[j - 1/2, j + 1/2) n [y_c - A, y_c + A]| F[j][i]
 * over the detector rows j; other columns get 0.  L[tr][e] (e = 0 .. nx)
 * is the wavelength at the column edge x = e - 1/2, NaN outside the trace.
 */
void orc_extract(const orc_scene *s, const double *F, double A, double *E, double *L)
{
    const int nx = s->nx, ny = s->ny;
    for (int tr = 0; tr < s->n_traces; ++tr) {
        const double *cx = s->cx + ORC_NCOEF * tr, *cy = s->cy + ORC_NCOEF * tr;
        double x0 = horner(cx, s->deg_x[tr], -1.0), x1 = horner(cx, s->deg_x[tr], 1.0);
        double span = s->lmax[tr] - s->lmin[tr];
        for (int e = 0; e <= nx; ++e) {
            double xe = (double)e - 0.5;
            double v = NAN;
            if (xe >= x0 && xe <= x1) {
                double t = t_at_x(s, tr, xe);
                v = 0.5 * (t * span + s->lmin[tr] + s->lmax[tr]);
            }
            L[(size_t)tr * (nx + 1) + e] = v;
        }
        for (int i = 0; i < nx; ++i) {
            double acc = 0.0;
            if (!isnan(L[(size_t)tr * (nx + 1) + i]) && !isnan(L[(size_t)tr * (nx + 1) + i + 1])) {
                double yc = horner(cy, s->deg_y[tr], t_at_x(s, tr, (double)i));
                for (int j = 0; j < ny; ++j) {
                    double ov = overlap((double)j - 0.5, (double)j + 0.5, yc - A, yc + A);
                    if (ov > 0.0) acc += ov * F[(size_t)j * nx + i];
                }
            }
            E[(size_t)tr * nx + i] = acc;
        }
    }
}

/* Moving mean of odd width w over x[0..n-1] (the window clipped to the
 * array, divided by the samples it holds). */
static void box_mean(const double *x, int64_t n, int w, double *y)
{
    int64_t h = w / 2;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = i - h < 0 ? 0 : i - h, b = i + h + 1 > n ? n : i + h + 1;
        double acc = 0.0;
        for (int64_t m = a; m < b; ++m) acc += x[m];
        y[i] = acc / (double)(b - a);
    }
}

/* Template smoothing: three passes of the moving mean of width w (their
 * cascade approximates a Gaussian of variance 3 (w^2 - 1) / 12 samples^2;
 * Wells, IEEE PAMI 8, 1986). */
void orc_smooth3(const double *x, int64_t n, int w, double *y)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    box_mean(x, n, w, y);
    box_mean(y, n, w, t);
    box_mean(t, n, w, y);
    free(t);
}

/* Odd moving-mean width whose three-pass cascade has a standard deviation
 * of sigma_px pixels on a trace with n samples over its x span. */
static int smooth_width(const orc_scene *s, int tr, double sigma_px)
{
    const double *cx = s->cx + ORC_NCOEF * tr;
    double span_px = horner(cx, s->deg_x[tr], 1.0) - horner(cx, s->deg_x[tr], -1.0);
    double sg = sigma_px * (double)s->n[tr] / span_px;
    int w = (int)floor(sqrt(4.0 * sg * sg + 1.0) + 0.5);
    if (w % 2 == 0) w += 1;
    return w < 1 ? 1 : w;
}

/*
 * Cross-correlation of the extracted spectra with the input spectra (Sec.
 * 4.2: RV recovered by cross-correlation of the extracted 1-D spectrum).
 * The template of a trace is its own spectrum slot (photons per sample on
 * the cell-centred rest-frame grid lambda_m = lmin + (m + 1/2) dl) smoothed
 * by orc_smooth3 to about the instrument's resolution (sigma_px pixels),
 * so that lines narrower than a pixel do not alias with the pixel grid.
 * The extracted flux is first divided by the extraction of a flat-field
 * frame when one is given (Ef), which removes the blaze and dispersion
 * trend along the order.  For trial velocity v_k = v0 + k dv (beta_k =
 * v_k / c), column i with centre wavelength lc_i = (L_i + L_{i+1}) / 2
 * sees the template at the fractional sample u_ik = (lc_i / (1 + beta_k) -
 * lmin) / dl - 1/2, linearly interpolated.  The columns used have both
 * edges on the trace, a positive flat (if given) and u_ik within
 * [6h, n - 2 - 6h] (h = (w - 1) / 2) for every trial velocity: twice the
 * smoothing support away from the ends of the trace, where the flux of a
 * column depends on how far the Doppler shift moved the sampled range; with
 * e_i = E_i (/ Ef_i) and e' = e - mean(e) over them,
 *   C[tr][k] = sum_i e'_i S(u_ik).
 * The velocity estimate is the vertex of the parabola through the largest
 * value of sum_tr C[tr][k] (k in 1 .. nv-2) and its two neighbours.
 */
double orc_ccf(const orc_scene *s, const double *E, const double *Ef, const double *L, double v0,
               double dv, int nv, double sigma_px, double *C)
{
    const int nx = s->nx;
    double *tot = (double *)calloc((size_t)nv, sizeof(double));
    double bmin = fmin(v0, v0 + (nv - 1) * dv) / C_LIGHT;
    double bmax = fmax(v0, v0 + (nv - 1) * dv) / C_LIGHT;
    for (int tr = 0; tr < s->n_traces; ++tr) {
        const double *T = s->spec + s->spec_off[s->slot[tr]];
        double lmin = s->lmin[tr], lmax = s->lmax[tr];
        int64_t n = s->n[tr];
        double dl = (lmax - lmin) / (double)n;
        int w = smooth_width(s, tr, sigma_px), h = w / 2;
        double *S = (double *)malloc(sizeof(double) * (size_t)n);
        orc_smooth3(T, n, w, S);
        const double *Lt = L + (size_t)tr * (nx + 1);
        const double *Et = E + (size_t)tr * nx;
        const double *Ft = Ef ? Ef + (size_t)tr * nx : NULL;
        double ulo = 6.0 * h, uhi = (double)(n - 2 - 6 * h);
#define ORC_LC(i) (0.5 * (Lt[i] + Lt[(i) + 1]))
#define ORC_CCF_USE(i) (!isnan(Lt[i]) && !isnan(Lt[(i) + 1]) && (!Ft || Ft[i] > 0.0) && \
                        (ORC_LC(i) / (1.0 + bmax) - lmin) / dl - 0.5 >= ulo && \
                        (ORC_LC(i) / (1.0 + bmin) - lmin) / dl - 0.5 <= uhi)
        double mean = 0.0;
        int cnt = 0;
        for (int i = 0; i < nx; ++i) {
            if (!ORC_CCF_USE(i)) continue;
            mean += Ft ? Et[i] / Ft[i] : Et[i];
            ++cnt;
        }
        if (cnt > 0) mean /= cnt;
        for (int k = 0; k < nv; ++k) {
            double beta = (v0 + k * dv) / C_LIGHT, acc = 0.0;
            for (int i = 0; i < nx; ++i) {
                if (!ORC_CCF_USE(i)) continue;
                double u = (ORC_LC(i) / (1.0 + beta) - lmin) / dl - 0.5;
                int64_t m = (int64_t)floor(u);
                double f = u - (double)m;
                double tv = S[m] * (1.0 - f) + S[m + 1] * f;
                double e = Ft ? Et[i] / Ft[i] : Et[i];
                acc += (e - mean) * tv;
            }
            C[(size_t)tr * nv + k] = acc;
            tot[k] += acc;
        }
#undef ORC_CCF_USE
#undef ORC_LC
        free(S);
    }
    int kb = 1;
    for (int k = 1; k < nv - 1; ++k)
        if (tot[k] > tot[kb]) kb = k;
    double ym = tot[kb - 1], y0 = tot[kb], yp = tot[kb + 1];
    double den = ym - 2.0 * y0 + yp;
    double off = den != 0.0 ? 0.5 * (ym - yp) / den : 0.0;
    free(tot);
    return v0 + dv * ((double)kb + off);
}
