/*
 * Multi-core driver of the FP64 oracle -- TEST INFRASTRUCTURE ONLY (the CPU
 * baseline of the benchmark and the tests that pin this driver to the plain
 * oracle).  It compiles the oracle's own source and adds nothing to its
 * arithmetic: every trace is rendered by the same per-sample scatter as
 * orc_render (Sec. 2 / Sec. 2.2: the frame is the superposition of every
 * sample's PSF integrated over the pixels), traces spread over OpenMP
 * threads, each trace into a private band of rows that holds its footprint.
 * The bands are then added into the frame in trace order, a fixed order, so
 * the result is the same for any thread count (it differs from orc_render's
 * single sum only in where the rounding of the per-trace partial sums falls).
 */
#include "oracle.c"

#include <omp.h>

/* Rows a trace can reach: its y at every 64th sample and at the last, then
 * the footprint's reach plus two rows (y moves far less than a pixel over 64
 * samples of any trace the renderer accepts). */
static void trace_rows(const orc_scene *s, const orc_psf *p, int tr, double beta, int *j0,
                       int *j1)
{
    double ylo = 1e300, yhi = -1e300, x, y;
    for (int64_t k = 0; k < s->n[tr]; k += 64) {
        position(s, tr, k, beta, &x, &y);
        ylo = y < ylo ? y : ylo;
        yhi = y > yhi ? y : yhi;
    }
    position(s, tr, s->n[tr] - 1, beta, &x, &y);
    ylo = y < ylo ? y : ylo;
    yhi = y > yhi ? y : yhi;
    int reach = p->kind == 1 ? p->kh / p->os + 2 : p->half_width + 1;
    int a = (int)floor(ylo) - reach - 2, b = (int)ceil(yhi) + reach + 3;
    *j0 = a < 0 ? 0 : a;
    *j1 = b > s->ny ? s->ny : b;
}

/* Accumulate traces [tr_lo, tr_hi) into frame[ny][nx] (caller zeroes it)
 * with nthreads threads (<= 0: the OpenMP default). */
int orc_render_omp(const orc_scene *s, const orc_psf *p, double rv_mps, double flux_scale,
                   int tr_lo, int tr_hi, double *frame, int nthreads)
{
    const int nt = tr_hi - tr_lo;
    if (nt <= 0) return 0;
    const double beta = rv_mps / C_LIGHT;
    double **band = (double **)calloc((size_t)nt, sizeof(double *));
    int *bj0 = (int *)calloc((size_t)nt, sizeof(int)), *bj1 = (int *)calloc((size_t)nt, sizeof(int));
    if (!band || !bj0 || !bj1) return -1;
    int fail = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (int q = 0; q < nt; ++q) {
        const int tr = tr_lo + q;
        int j0, j1;
        trace_rows(s, p, tr, beta, &j0, &j1);
        if (j1 <= j0) continue;
        double *b = (double *)calloc((size_t)(j1 - j0) * s->nx, sizeof(double));
        double *wt = (double *)malloc(sizeof(double) * orc_footprint_cap(p));
        if (!b || !wt) {
            free(b);
            free(wt);
            fail |= 1;
            continue;
        }
        const double *S = s->spec + s->spec_off[s->slot[tr]];
        const double scale = s->thr[tr] * flux_scale;
        for (int64_t k = 0; k < s->n[tr]; ++k) {
            double x, y;
            position(s, tr, k, beta, &x, &y);
            const double phi = S[k] * scale;
            int i0, jw0, w, h;
            if (orc_sample_weights(p, s->nx, s->ny, x, y, &i0, &jw0, &w, &h, wt)) {
                fail |= 1;
                break;
            }
            for (int r = 0; r < h; ++r) {
                const int j = jw0 + r;
                if (j < 0 || j >= s->ny) continue;
                if (j < j0 || j >= j1) {  /* outside the band: cannot happen */
                    fail |= 2;
                    continue;
                }
                for (int a = 0; a < w; ++a) {
                    const int i = i0 + a;
                    if (i < 0 || i >= s->nx) continue;
                    b[(size_t)(j - j0) * s->nx + i] += phi * wt[r * w + a];
                }
            }
        }
        free(wt);
        band[q] = b;
        bj0[q] = j0;
        bj1[q] = j1;
    }
    for (int q = 0; q < nt; ++q) {  /* fixed order: trace order */
        if (!band[q]) continue;
        const size_t o = (size_t)bj0[q] * s->nx, m = (size_t)(bj1[q] - bj0[q]) * s->nx;
        for (size_t e = 0; e < m; ++e) frame[o + e] += band[q][e];
        free(band[q]);
    }
    free(band);
    free(bj0);
    free(bj1);
    return fail ? -1 : 0;
}
