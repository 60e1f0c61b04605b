/*
 * e2e.h -- C ABI of the MI355X echellogram renderer.
 *
 * The library renders synthetic raw frames of a cross-dispersed echelle
 * spectrograph the way Genoni et al. (2020, "End to end simulators: a
 * flexible and scalable cloud-based architecture", Exp. Astron.) define
 * them: the frame is the superposition, over a fine wavelength grid, of
 * every spectral fiber image (SFI) projected on the detector (Sec. 2), each
 * SFI being the PSF integrated over the pixel areas on a sub-pixel grid
 * (Sec. 2.2), with photon noise added on the final frame (Sec. 2.2).  The
 * spectrograph is described by a database of spectral-format data, PSF maps
 * and throughput per SFI (Sec. 2.1) that is computed once and kept for many
 * simulations; here it is loaded once into device-resident tables.
 *
 * Conventions (every entry point):
 *   - wavelengths in nm (FP64); detector positions in pixels, 0-based, pixel
 *     (i, j) covering [i-1/2, i+1/2) x [j-1/2, j+1/2); frames row-major
 *     [ny][nx] with y = row;
 *   - a trace (one order x fiber x slice) has n samples at
 *     lmin + (k + 1/2)(lmax - lmin)/n; a Doppler shift v moves sample k to
 *     lambda_k (1 + v/c) before the format map;
 *   - x and y of a sample are polynomials in t = (2 lambda' - lmin - lmax) /
 *     (lmax - lmin), coefficients in ascending powers; x must increase
 *     strictly with lambda over the trace and |dy/dx| must stay <= 0.5;
 *   - sample photons = spectrum[slot][k] * throughput * flux_scale;
 *   - flux falling off the detector is dropped.
 * Status codes: 0 = E2E_OK, >0 = still pending, <0 = error.  No C++
 * exception crosses this interface.  e2e_last_error() returns a
 * thread-local message for the calling thread's last failure.
 */
#ifndef E2E_H
#define E2E_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t e2e_status;

#define E2E_OK 0
#define E2E_PENDING 1
#define E2E_EINVAL (-1)       /* null pointer, bad size, bad enum value        */
#define E2E_EFORMAT (-2)      /* trace not monotone / too steep / bad degree   */
#define E2E_EPSF (-3)         /* PSF table not normalised, bad shape           */
#define E2E_ENOMEM (-4)       /* request exceeds the context's HBM budget      */
#define E2E_EAGAIN (-5)       /* serve queue full                              */
#define E2E_ENOTFOUND (-6)    /* unknown handle or ticket                      */
#define E2E_EDEVICE (-7)      /* HIP runtime error (message kept)              */
#define E2E_EBUSY (-8)        /* handle still referenced by in-flight work     */
#define E2E_EUNSUPPORTED (-9) /* valid but not implemented combination        */
#define E2E_EINTERNAL (-10)   /* a device-side consistency check failed        */

typedef struct e2e_ctx e2e_ctx;
typedef uint64_t e2e_format_id;
typedef uint64_t e2e_psf_id;
typedef uint64_t e2e_ticket;

/* element types of spectra and frames */
#define E2E_F32 0
#define E2E_F64 1

/* PSF kinds (Sec. 2.1: an analytic asymmetric Gaussian, or ray-traced maps) */
#define E2E_PSF_GAUSS_ERF 0  /* circular Gaussian, exact pixel integrals       */
#define E2E_PSF_TABLE 1      /* field-varying maps of cell integrals           */
#define E2E_PSF_SEPARABLE 2  /* field-varying axis-aligned Gaussian (sx, sy)   */
#define E2E_PSF_SFI 3        /* fiber image (disc / half) (x) Gaussian, sub-px */

/* fiber image shapes of E2E_PSF_SFI */
#define E2E_FIBER_DISC 0      /* uniform disc of radius fiber_radius           */
#define E2E_FIBER_HALF_UP 1   /* its half at y >= the sample's y               */
#define E2E_FIBER_HALF_DOWN 2 /* its half at y <= the sample's y               */

/* arithmetic of the render path */
#define E2E_PREC_F64 0       /* FP64 positions, FP32 PSF offsets, FP64 sums    */
#define E2E_PREC_F32 1       /* separable only: FP32 weights (fitted normal
                                tail, Numerical Recipes Sec. 6.2) and FP32 sums */
#define E2E_PREC_BF16_HILO 2 /* separable only: bf16 hi/lo MFMA, FP32 sums     */
#define E2E_PREC_F16_HILO 3  /* separable only: fp16 hi/lo MFMA, FP32 sums     */

/* request flags */
#define E2E_FLAG_ASYNC 1u    /* device output: return once enqueued on stream  */

/*
 * One spectral trace: the spectral-format record of Sec. 2.1 (order number,
 * fiber, wavelength range, centroid position as a function of wavelength)
 * plus its throughput (Sec. 2.1: multiplied on the normalised illumination).
 * cx / cy hold deg+1 FP64 coefficients (deg <= 7), copied by the load call.
 */
typedef struct {
    int32_t order, fiber, slice;
    double lambda_min_nm, lambda_max_nm;
    int64_t n_samples;            /* 1 .. 2^31-1                              */
    int32_t deg_x, deg_y;
    const double *cx, *cy;
    double throughput;
    int32_t spectrum_slot;        /* index into e2e_render_req.spectra        */
} e2e_trace_desc;

/*
 * PSF maps (Sec. 2.1).  GAUSS_ERF: sigma (px) and half_width H, the weight
 * of pixel (a+d) on each axis being the normal-CDF difference over the
 * pixel, renormalised over the (2H+1)-wide window around a = floor(x+1/2).
 * TABLE: tables[grid_ny][grid_nx][kh][kw] float32 cell integrals, each node
 * summing to 1 (within 1e-5), oversample cells per pixel, centred on the
 * table centre, nodes spanning the detector edge to edge and interpolated
 * bilinearly at each sample's (x, y); the GPU path needs oversample = 4 and
 * kw = kh in {32, 48}.  SEPARABLE: sigma_xy[grid_ny][grid_nx][2] (sx, sy)
 * interpolated bilinearly, then the GAUSS_ERF rule per axis with half_width.
 * SFI (Sec. 2.2: each spectral fiber image is the surface integral of the
 * fiber's spatial profile convolved with the PSF, computed on a sub-pixel
 * grid): the fiber image is a uniform disc of radius fiber_radius px (or
 * the half of it selected by fiber_shape) centred on the sample position,
 * convolved with the SEPARABLE kind's Gaussian (sigma_xy grid); a pixel's
 * weight is the mean of that density at the centres of its subpixels x
 * subpixels sub-pixels (10 in the paper), over the (2H+1)^2 window around
 * (floor(x+1/2), floor(y+1/2)), renormalised by the window sum.  Limits:
 * half_width 1..7, subpixels 1..16, fiber_radius > 0 with fiber_radius /
 * min(sigma) <= 4 (E2E_EPSF otherwise).
 * All arrays are host memory, copied by the load call.
 */
typedef struct {
    int32_t kind;
    double sigma;
    int32_t half_width;
    int32_t grid_nx, grid_ny;
    int32_t kw, kh, oversample;
    const float *tables;
    const float *sigma_xy;
    double fiber_radius;          /* SFI only                                  */
    int32_t fiber_shape;          /* SFI only: E2E_FIBER_*                     */
    int32_t subpixels;            /* SFI only                                  */
} e2e_psf_desc;

/*
 * One frame to render (Sec. 3's "parameter file": which database, which
 * source, which scenario).  spectra[s] points to the photons per sample of
 * slot s (n_samples of the traces that use it), on the device when
 * spectra_on_device != 0 (then `spectra` itself is still a host array of
 * device pointers).  out is [ny][nx] of out_dtype, on the device when
 * out_on_device != 0.  hip_stream: a hipStream_t, or NULL for the context's
 * stream.  Poisson noise (Sec. 2.2) uses Philox-4x32-10 keyed by (seed) with
 * counter (pixel, frame_index, draw).  All caller buffers are borrowed for
 * the duration of the call (for e2e_serve_submit: until poll completes).
 */
typedef struct {
    e2e_format_id fmt;
    e2e_psf_id psf;
    const void *const *spectra;
    int32_t n_spectra;
    int32_t spectrum_dtype;
    int32_t spectra_on_device;
    double rv_mps;
    double flux_scale;
    uint64_t seed;
    uint32_t frame_index;
    int32_t poisson;
    int32_t precision;
    void *out;
    int32_t out_dtype;
    int32_t out_on_device;
    void *hip_stream;
    uint32_t flags;
} e2e_render_req;

/* Per-request timing of the serve loop.  t_*_us: host clock, microseconds
 * since the context was created.  t_gpu_start_us / t_gpu_end_us: device
 * timestamps (HIP events on the launch's stream, just before its first and
 * after its last kernel), microseconds since the serve loop started; the
 * launches of two requests overlapped on the device when one's start lies
 * before the other's end. */
typedef struct {
    double t_submit_us, t_admit_us, t_launch_us, t_done_us;
    uint64_t footprint_bytes;
    int32_t status;
    int32_t batch_size;           /* requests that shared its launch          */
    double t_gpu_start_us, t_gpu_end_us;
} e2e_render_stats;

typedef struct {
    int32_t max_inflight;         /* requests admitted at once (slots)        */
    int32_t max_queue;            /* queued but not yet admitted              */
    int32_t n_streams;            /* device streams used for overlap          */
    int32_t max_batch;            /* requests merged into one launch          */
} e2e_serve_config;

/* Context bound to one HIP device; hbm_budget_bytes caps the device memory
 * that resident tables plus in-flight renders may use (0 = 90% of free). */
e2e_status e2e_create(e2e_ctx **out, int32_t hip_device, uint64_t hbm_budget_bytes);
/* Drains the serve loop, frees every resident table. */
void e2e_destroy(e2e_ctx *ctx);
/* Message of the calling thread's last failed call ("" if none). */
const char *e2e_last_error(void);
/* Library version string. */
const char *e2e_version(void);

/*
 * Copy a spectral-format database (Sec. 2.1) into device-resident tables.
 * Validation: degrees in 0..7, lmin < lmax, n >= 1, dx/dt > 0 on [-1, 1]
 * (strictly increasing x), |dy/dx| <= 0.5, det_nx/ny in 1..65536.
 * Errors: E2E_EINVAL, E2E_EFORMAT, E2E_ENOMEM, E2E_EDEVICE.
 */
e2e_status e2e_format_load(e2e_ctx *ctx, const e2e_trace_desc *traces, int32_t n_traces,
                           int32_t det_nx, int32_t det_ny, e2e_format_id *out);
/* Copy PSF maps into device-resident tables (pre-binned per pixel phase for
 * TABLE).  Errors: E2E_EINVAL, E2E_EPSF, E2E_ENOMEM, E2E_EDEVICE. */
e2e_status e2e_psf_load(e2e_ctx *ctx, const e2e_psf_desc *psf, e2e_psf_id *out);
/* E2E_EBUSY while a served request still uses the handle. */
e2e_status e2e_format_free(e2e_ctx *ctx, e2e_format_id id);
e2e_status e2e_psf_free(e2e_ctx *ctx, e2e_psf_id id);

/*
 * Render one frame (the plain renderer: one launch per frame, one workgroup
 * per detector tile).  Writes req->out before returning unless
 * E2E_FLAG_ASYNC is set and the output is on the device.
 */
e2e_status e2e_render(e2e_ctx *ctx, const e2e_render_req *req);
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): e2e_render
 * of one frame whose spectra and output are on the device, with every buffer
 * the render needs beyond the caller's inputs and output (planner output,
 * frame record, spectrum pointers, error word, work counter) taken from a
 * fixed 16 MiB device array that each GPU holds until the process ends; the
 * call makes no hipMalloc, hipHostMalloc or hipFree.  Synchronous (returns
 * when the frame is written); E2E_FLAG_ASYNC is ignored.  Limits: at most 64
 * spectrum slots, and planner output of at most about 16 MiB
 * (16 B x tile columns x traces + 32 B x traces), else E2E_ENOMEM with the
 * size in the message; host spectra or output, E2E_EINVAL.  The array is
 * shared by every call on that GPU and keeps the last call's contents: calls
 * that overlap on one GPU (several threads, several contexts) race and must
 * be serialised by the caller.  Results equal e2e_render's bit for bit.
 */
e2e_status e2e_render_noalloc(e2e_ctx *ctx, const e2e_render_req *req);
/*
 * Render n frames of any sizes / formats sharing one PSF kind in one
 * persistent launch that pulls (frame, tile) work items from a queue;
 * results are bitwise identical to e2e_render of each frame.
 */
e2e_status e2e_render_batch(e2e_ctx *ctx, const e2e_render_req *reqs, int32_t n);

/*
 * Waits for hip_stream (NULL: the context's stream) and reports the device
 * consistency checks of every render launched on it since the last
 * synchronous call: E2E_EINTERNAL (message names the check) if any failed,
 * then clears them.  A synchronous e2e_render / e2e_render_batch on the same
 * stream reports them the same way; an E2E_FLAG_ASYNC call never does.
 * Errors: E2E_EINVAL (NULL ctx), E2E_EDEVICE, E2E_EINTERNAL.
 */
e2e_status e2e_sync(e2e_ctx *ctx, void *hip_stream);

/*
 * Continuous-batching request loop (Sec. 3's "size the problem, allocate
 * resources, distribute the work", on one GPU).  e2e_serve_start is
 * optional (defaults apply on first submit).  submit copies the request;
 * host spectra are copied to the device before submit returns.  A request
 * is admitted when a slot and its HBM footprint are free and is merged with
 * other admitted requests into the next launch.  poll waits up to
 * timeout_ms (0 = no wait, <0 = forever) and returns E2E_OK, E2E_PENDING or
 * the request's error; after a non-pending result the ticket is released.
 * Submit and poll are thread-safe.  e2e_serve_stop drains and joins.
 * Launches on different streams overlap on the device only if those streams
 * sit on different hardware queues: HIP gives a process GPU_MAX_HW_QUEUES of
 * them (4 unless set before HIP starts) and assigns streams round-robin, so a
 * process that uses many streams should raise it (the tests and benchmark
 * use 16).
 */
e2e_status e2e_serve_start(e2e_ctx *ctx, const e2e_serve_config *cfg);
e2e_status e2e_serve_submit(e2e_ctx *ctx, const e2e_render_req *req, e2e_ticket *out);
e2e_status e2e_serve_poll(e2e_ctx *ctx, e2e_ticket t, int32_t timeout_ms,
                          e2e_render_stats *stats);
e2e_status e2e_serve_stop(e2e_ctx *ctx);

/*
 * Launch autotuner (the batch / serve orchestration of Sec. 3, sized to one
 * GPU).  Renders the given requests (n = 1: the plain renderer; n > 1: one
 * persistent batch launch) under each candidate launch choice -- work-unit
 * length in tiles (table path: 2, 4, 8, 16) and, for batches, persistent
 * workgroups per CU (1..3) -- times them with HIP events (a warm-up run,
 * then the best of two), and keeps the fastest for the requests' workload
 * shapes (PSF kind and grid, precision, spectrum type, detector size, trace
 * count and degrees).  Later e2e_render, e2e_render_batch and served
 * requests of those shapes use it.  The requests' outputs are written by
 * the runs.  The unit length changes only the fixed order in which a
 * pixel's contributions are summed (results stay deterministic per choice,
 * within rounding of each other); the grid width does not change results.
 * Errors: those of e2e_render_batch; E2E_EINVAL for n < 1 or NULL reqs.
 */
#define E2E_TUNE_MAX 16
typedef struct {
    int32_t chunk, resident;      /* the choice kept                           */
    double ms;                    /* its time per launch                       */
    int32_t n_candidates;
    int32_t cand_chunk[E2E_TUNE_MAX], cand_resident[E2E_TUNE_MAX];
    double cand_ms[E2E_TUNE_MAX];
} e2e_tune_report;
e2e_status e2e_autotune(e2e_ctx *ctx, const e2e_render_req *reqs, int32_t n,
                        e2e_tune_report *report);

/*
 * Photon noise on an existing expected-count frame, in place (Sec. 2.2):
 * frame[p] <- Poisson(frame[p]) with the counter stream of pixel p.
 */
e2e_status e2e_noise_poisson(e2e_ctx *ctx, void *frame, int32_t dtype, int64_t n_pixels,
                             uint64_t seed, uint32_t frame_index, int32_t on_device,
                             void *hip_stream);
/*
 * Detector stage on a rendered frame (Sec. 2.2: the frame of expected
 * photo-electrons is turned into a raw CCD read-out by photon noise plus the
 * detector's own effects -- dark current, read-out noise, pixel response
 * non-uniformity and inter-pixel cross-talk -- then digitised).  For pixel
 * p = y nx + x, in this order:
 *   mu  = G[p] F[p] + dark_e_per_s exposure_s  (one FP64 fma; G = prnu, 1 if
 *         prnu is NULL)
 *   N   = Poisson(mu) from pixel p's counter stream (the stream of
 *         e2e_noise_poisson: Philox blocks 0, 1, ...), or mu if shot_noise = 0
 *   E   = sum over dy = -1..1 (outer), dx = -1..1 (inner) of
 *         xtalk[(dy+1)*3 + dx+1] * N[(x-dx, y-dy)], FP64 fma in that order;
 *         a source pixel off the detector contributes 0 (xtalk[4] is the
 *         charge a pixel keeps, xtalk[(dy+1)*3+dx+1] what it hands to its
 *         neighbour at offset (dx, dy))
 *   R   = E + ron_e Z, Z = sqrt(-2 ln u1) cos(2 pi u2) from Philox block
 *         2^31 of pixel p's stream (u1 from words 0-1, u2 from words 2-3,
 *         53-bit uniforms in (0, 1)); skipped when ron_e = 0
 *   ADU = min(max(floor(R / gain_e_per_adu + bias_adu + 1/2), 0), 2^bits - 1)
 * frame: nx * ny row-major values of frame_dtype (E2E_F32 / E2E_F64) in
 * expected electrons; prnu: NULL or nx * ny FP32 gains; adu_out: nx * ny
 * uint16.  on_device = 1: all three are device pointers and the call is
 * ordered on hip_stream (NULL: the context's stream), returning after the
 * work is enqueued and finished; 0: host pointers, staged through device
 * memory (allocated for the call).  The caller owns all buffers.
 * Errors: E2E_EINVAL for NULL ctx / desc / frame / adu_out, nx < 0, ny
 * outside 0..4194240,
 * bad dtype, bits outside 1..16, gain_e_per_adu <= 0, a negative or
 * non-finite exposure, dark current or read noise, or non-finite cross-talk
 * weights or bias; E2E_ENOMEM, E2E_EDEVICE.
 */
typedef struct {
    double exposure_s;         /* t [s]                                         */
    double dark_e_per_s;       /* dark current [e-/s/pixel]                     */
    double xtalk[9];           /* K[dy+1][dx+1], row-major                      */
    double ron_e;              /* read-out noise sigma [e-]                     */
    double gain_e_per_adu;     /* electrons per ADU                             */
    double bias_adu;           /* offset added before rounding                  */
    uint64_t seed;
    uint32_t frame_index;
    int32_t shot_noise;        /* 1: Poisson draw of mu, 0: mu itself           */
    int32_t bits;              /* ADC resolution, 1..16                         */
    int32_t reserved;
} e2e_detector_desc;
e2e_status e2e_detector(e2e_ctx *ctx, const e2e_detector_desc *d, const void *frame,
                        int32_t frame_dtype, const float *prnu, int32_t nx, int32_t ny,
                        uint16_t *adu_out, int32_t on_device, void *hip_stream);

/*
 * Closing the loop (Sec. 1: the simulated frames feed a data-reduction
 * pipeline; Sec. 4.2: 1-D spectra extracted along the traced orders, a
 * wavelength scale from the dispersion, the radial velocity recovered by
 * cross-correlation).
 *
 * e2e_extract: box extraction of every trace of format `fmt` from a frame
 * [ny][nx] of frame_dtype.  For pixel column i whose edges i -+ 1/2 both
 * lie inside the trace's x range [x(-1), x(1)], with t_c the format
 * coordinate where x(t_c) = i and y_c = y(t_c):
 *   flux[tr][i] = sum_j |[j - 1/2, j + 1/2) n [y_c - A, y_c + A]| F[j][i]
 * over the detector rows (A = aperture_half_px > 0), and 0 for the other
 * columns; edges[tr][e] (e = 0 .. nx) is the detector-frame wavelength
 * (t (lmax - lmin) + lmin + lmax) / 2 at x(t) = e - 1/2, NaN off the trace.
 * flux is [ntr][nx] FP64, edges [ntr][nx+1] FP64.  on_device = 1: all
 * three arrays are device pointers and the work is ordered on hip_stream
 * (NULL: the context's stream); 0: host arrays, staged.  Returns when done.
 * Errors: E2E_EINVAL (NULL pointers, bad dtype, A outside (0, 1e6]),
 * E2E_ENOTFOUND (fmt), E2E_ENOMEM, E2E_EDEVICE.
 */
e2e_status e2e_extract(e2e_ctx *ctx, e2e_format_id fmt, const void *frame, int32_t frame_dtype,
                       double aperture_half_px, double *flux, double *edges, int32_t on_device,
                       void *hip_stream);

/*
 * e2e_ccf: cross-correlation of extracted spectra with the input spectra.
 * The template of trace tr is its spectrum slot (photons per sample on the
 * rest-frame grid lambda_m = lmin + (m + 1/2) dl, dl = (lmax - lmin) / n)
 * smoothed by three passes of a moving mean of odd width w (clipped at the
 * ends; w = the odd integer nearest sqrt(4 s^2 + 1), s = smooth_px n /
 * (x(1) - x(-1)), so the cascade's standard deviation is about smooth_px
 * pixels), which keeps lines narrower than a pixel from aliasing with the
 * pixel grid.  With e_i = flux_i / flat_i (flux_i if flat is NULL), trial
 * velocities v_k = v0 + k dv (k < n_v, beta_k = v_k / c) and the column
 * centre wavelength lc_i = (edges_i + edges_{i+1}) / 2, the template is read
 * at the fractional sample u_ik = (lc_i / (1 + beta_k) - lmin) / dl - 1/2
 * by linear interpolation.  Columns used: both edges finite, flat_i > 0 (if
 * given), u_ik in [6h, n - 2 - 6h] (h = (w - 1) / 2) for every k; with
 * e' = e - mean(e) over them, ccf[tr][k] = sum_i e'_i S(u_ik).  *rv_mps_out
 * receives the vertex of the parabola through the largest value of
 * sum_tr ccf[tr][k] (k in 1 .. n_v - 2) and its two neighbours.
 * on_device: flux / flat / edges / templates / ccf_out are device pointers
 * (templates is still a host array of n_templates pointers).  ccf_out may
 * be NULL.  The library allocates the smoothed templates of up to 64
 * traces at a time (2 n FP64 values per trace) for the call.
 * Errors: E2E_EINVAL (NULL pointers, n_v < 3, dv = 0, smooth_px <= 0, a
 * moving-mean width above 4095 samples, too few templates, bad dtype),
 * E2E_ENOTFOUND, E2E_ENOMEM, E2E_EDEVICE.
 */
typedef struct {
    const double *flux;            /* [ntr][nx]                                */
    const double *flat;            /* [ntr][nx] or NULL                        */
    const double *edges;           /* [ntr][nx+1]                              */
    const void *const *templates;  /* per spectrum slot                        */
    int32_t n_templates;
    int32_t template_dtype;        /* E2E_F32 / E2E_F64                        */
    int32_t on_device;
    int32_t n_v;
    double v0_mps, dv_mps;
    double smooth_px;
    double *ccf_out;               /* [ntr][n_v] or NULL                       */
    void *hip_stream;
} e2e_ccf_req;
e2e_status e2e_ccf(e2e_ctx *ctx, e2e_format_id fmt, const e2e_ccf_req *req, double *rv_mps_out);

/*
 * Raw Philox-4x32-10 blocks (Salmon et al., SC'11) of the noise stream:
 * out_host[(p * blocks + b) * 4 + w] = word w of block b of pixel pixel0+p.
 */
e2e_status e2e_philox_blocks(e2e_ctx *ctx, uint64_t seed, uint32_t frame_index,
                             uint64_t pixel0, int64_t n_pixels, uint32_t blocks,
                             uint32_t *out_host);

/*
 * Kernel timing: with profiling on, the library brackets each launch of its
 * render kernels with HIP events on the launch stream.  e2e_kernel_time
 * returns launches and total milliseconds per kernel name ("render_table",
 * "render_sep", "render_sep_mfma", "render_sfi", "plan", "noise",
 * "detector", "extract", "template_smooth", "ccf"), synchronising first.
 */
e2e_status e2e_set_profiling(e2e_ctx *ctx, int32_t on);
e2e_status e2e_kernel_time(e2e_ctx *ctx, const char *kernel, int64_t *launches,
                           double *total_ms);
e2e_status e2e_reset_kernel_time(e2e_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* E2E_H */
