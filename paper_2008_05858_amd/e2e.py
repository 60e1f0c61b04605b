"""ctypes binding of libe2e (include/e2e.h): the same names, marshalling only.

Every step of rendering runs in the library's HIP kernels; this module only
builds the C structs and converts status codes into exceptions.  It never
falls back to any other implementation: if ``libe2e.so`` is missing it
raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libe2e.so")

E2E_OK, E2E_PENDING = 0, 1
E2E_EINVAL, E2E_EFORMAT, E2E_EPSF, E2E_ENOMEM, E2E_EAGAIN = -1, -2, -3, -4, -5
E2E_ENOTFOUND, E2E_EDEVICE, E2E_EBUSY, E2E_EUNSUPPORTED, E2E_EINTERNAL = -6, -7, -8, -9, -10
E2E_F32, E2E_F64 = 0, 1
E2E_PSF_GAUSS_ERF, E2E_PSF_TABLE, E2E_PSF_SEPARABLE, E2E_PSF_SFI = 0, 1, 2, 3
E2E_FIBER_DISC, E2E_FIBER_HALF_UP, E2E_FIBER_HALF_DOWN = 0, 1, 2
E2E_PREC_F64, E2E_PREC_F32, E2E_PREC_BF16_HILO, E2E_PREC_F16_HILO = 0, 1, 2, 3
E2E_FLAG_ASYNC = 1

STATUS_NAMES = {0: "E2E_OK", 1: "E2E_PENDING", -1: "E2E_EINVAL", -2: "E2E_EFORMAT",
                -3: "E2E_EPSF", -4: "E2E_ENOMEM", -5: "E2E_EAGAIN", -6: "E2E_ENOTFOUND",
                -7: "E2E_EDEVICE", -8: "E2E_EBUSY", -9: "E2E_EUNSUPPORTED",
                -10: "E2E_EINTERNAL"}

EXPORTS = ["e2e_create", "e2e_destroy", "e2e_last_error", "e2e_version", "e2e_format_load",
           "e2e_psf_load", "e2e_format_free", "e2e_psf_free", "e2e_render", "e2e_render_noalloc",
           "e2e_render_batch",
           "e2e_serve_start", "e2e_serve_submit", "e2e_serve_poll", "e2e_serve_stop",
           "e2e_noise_poisson", "e2e_philox_blocks", "e2e_set_profiling", "e2e_kernel_time",
           "e2e_reset_kernel_time", "e2e_autotune", "e2e_detector", "e2e_extract", "e2e_ccf",
           "e2e_sync"]
E2E_TUNE_MAX = 16


class e2e_trace_desc(C.Structure):
    _fields_ = [("order", C.c_int32), ("fiber", C.c_int32), ("slice", C.c_int32),
                ("lambda_min_nm", C.c_double), ("lambda_max_nm", C.c_double),
                ("n_samples", C.c_int64), ("deg_x", C.c_int32), ("deg_y", C.c_int32),
                ("cx", C.POINTER(C.c_double)), ("cy", C.POINTER(C.c_double)),
                ("throughput", C.c_double), ("spectrum_slot", C.c_int32)]


class e2e_psf_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("sigma", C.c_double), ("half_width", C.c_int32),
                ("grid_nx", C.c_int32), ("grid_ny", C.c_int32), ("kw", C.c_int32),
                ("kh", C.c_int32), ("oversample", C.c_int32),
                ("tables", C.POINTER(C.c_float)), ("sigma_xy", C.POINTER(C.c_float)),
                ("fiber_radius", C.c_double), ("fiber_shape", C.c_int32),
                ("subpixels", C.c_int32)]


class e2e_render_req(C.Structure):
    _fields_ = [("fmt", C.c_uint64), ("psf", C.c_uint64), ("spectra", C.POINTER(C.c_void_p)),
                ("n_spectra", C.c_int32), ("spectrum_dtype", C.c_int32),
                ("spectra_on_device", C.c_int32), ("rv_mps", C.c_double),
                ("flux_scale", C.c_double), ("seed", C.c_uint64), ("frame_index", C.c_uint32),
                ("poisson", C.c_int32), ("precision", C.c_int32), ("out", C.c_void_p),
                ("out_dtype", C.c_int32), ("out_on_device", C.c_int32),
                ("hip_stream", C.c_void_p), ("flags", C.c_uint32)]


class e2e_tune_report(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("resident", C.c_int32), ("ms", C.c_double),
                ("n_candidates", C.c_int32),
                ("cand_chunk", C.c_int32 * E2E_TUNE_MAX),
                ("cand_resident", C.c_int32 * E2E_TUNE_MAX),
                ("cand_ms", C.c_double * E2E_TUNE_MAX)]


class e2e_detector_desc(C.Structure):
    _fields_ = [("exposure_s", C.c_double), ("dark_e_per_s", C.c_double),
                ("xtalk", C.c_double * 9), ("ron_e", C.c_double),
                ("gain_e_per_adu", C.c_double), ("bias_adu", C.c_double),
                ("seed", C.c_uint64), ("frame_index", C.c_uint32),
                ("shot_noise", C.c_int32), ("bits", C.c_int32), ("reserved", C.c_int32)]


class e2e_ccf_req(C.Structure):
    _fields_ = [("flux", C.c_void_p), ("flat", C.c_void_p), ("edges", C.c_void_p),
                ("templates", C.POINTER(C.c_void_p)), ("n_templates", C.c_int32),
                ("template_dtype", C.c_int32), ("on_device", C.c_int32), ("n_v", C.c_int32),
                ("v0_mps", C.c_double), ("dv_mps", C.c_double), ("smooth_px", C.c_double),
                ("ccf_out", C.c_void_p), ("hip_stream", C.c_void_p)]


class e2e_render_stats(C.Structure):
    _fields_ = [("t_submit_us", C.c_double), ("t_admit_us", C.c_double),
                ("t_launch_us", C.c_double), ("t_done_us", C.c_double),
                ("footprint_bytes", C.c_uint64), ("status", C.c_int32),
                ("batch_size", C.c_int32), ("t_gpu_start_us", C.c_double),
                ("t_gpu_end_us", C.c_double)]


class e2e_serve_config(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("max_queue", C.c_int32),
                ("n_streams", C.c_int32), ("max_batch", C.c_int32)]


class E2EError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libe2e.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7.
        # Loading it first makes libe2e.so bind to that copy (same soname);
        # loading the system copy first would leave torch unable to start HIP.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.e2e_create.argtypes = [P(C.c_void_p), C.c_int32, C.c_uint64]
        L.e2e_destroy.argtypes = [C.c_void_p]
        L.e2e_destroy.restype = None
        L.e2e_last_error.restype = C.c_char_p
        L.e2e_version.restype = C.c_char_p
        L.e2e_format_load.argtypes = [C.c_void_p, P(e2e_trace_desc), C.c_int32, C.c_int32,
                                      C.c_int32, P(C.c_uint64)]
        L.e2e_psf_load.argtypes = [C.c_void_p, P(e2e_psf_desc), P(C.c_uint64)]
        L.e2e_format_free.argtypes = [C.c_void_p, C.c_uint64]
        L.e2e_psf_free.argtypes = [C.c_void_p, C.c_uint64]
        L.e2e_render.argtypes = [C.c_void_p, P(e2e_render_req)]
        L.e2e_render_noalloc.argtypes = [C.c_void_p, P(e2e_render_req)]
        L.e2e_sync.argtypes = [C.c_void_p, C.c_void_p]
        L.e2e_render_batch.argtypes = [C.c_void_p, P(e2e_render_req), C.c_int32]
        L.e2e_serve_start.argtypes = [C.c_void_p, P(e2e_serve_config)]
        L.e2e_serve_submit.argtypes = [C.c_void_p, P(e2e_render_req), P(C.c_uint64)]
        L.e2e_serve_poll.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, P(e2e_render_stats)]
        L.e2e_serve_stop.argtypes = [C.c_void_p]
        L.e2e_noise_poisson.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64,
                                        C.c_uint64, C.c_uint32, C.c_int32, C.c_void_p]
        L.e2e_philox_blocks.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64,
                                        C.c_int64, C.c_uint32, P(C.c_uint32)]
        L.e2e_set_profiling.argtypes = [C.c_void_p, C.c_int32]
        L.e2e_kernel_time.argtypes = [C.c_void_p, C.c_char_p, P(C.c_int64), P(C.c_double)]
        L.e2e_reset_kernel_time.argtypes = [C.c_void_p]
        L.e2e_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, P(e2e_tune_report)]
        L.e2e_extract.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_int32, C.c_double,
                                  C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.e2e_ccf.argtypes = [C.c_void_p, C.c_uint64, P(e2e_ccf_req), P(C.c_double)]
        L.e2e_detector.argtypes = [C.c_void_p, P(e2e_detector_desc), C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                   C.c_void_p]
        for n in EXPORTS:
            if n not in ("e2e_destroy", "e2e_last_error", "e2e_version"):
                getattr(L, n).restype = C.c_int32
        _lib = L
    return _lib


def check(code):
    if code < 0:
        raise E2EError(code, lib().e2e_last_error().decode(errors="replace"))
    return code


# -- same names as the C ABI ------------------------------------------------

def e2e_create(device=0, hbm_budget_bytes=0):
    h = C.c_void_p()
    check(lib().e2e_create(C.byref(h), device, hbm_budget_bytes))
    return h


def e2e_destroy(ctx):
    lib().e2e_destroy(ctx)


def e2e_last_error():
    return lib().e2e_last_error().decode(errors="replace")


def e2e_version():
    return lib().e2e_version().decode()


def e2e_format_load(ctx, traces, n_traces, det_nx, det_ny):
    out = C.c_uint64()
    check(lib().e2e_format_load(ctx, traces, n_traces, det_nx, det_ny, C.byref(out)))
    return out.value


def e2e_psf_load(ctx, desc):
    out = C.c_uint64()
    check(lib().e2e_psf_load(ctx, C.byref(desc), C.byref(out)))
    return out.value


def e2e_format_free(ctx, fid):
    return check(lib().e2e_format_free(ctx, fid))


def e2e_psf_free(ctx, pid):
    return check(lib().e2e_psf_free(ctx, pid))


def e2e_render(ctx, req):
    return check(lib().e2e_render(ctx, C.byref(req)))


def e2e_render_noalloc(ctx, req):
    return check(lib().e2e_render_noalloc(ctx, C.byref(req)))


def e2e_sync(ctx, stream=None):
    return check(lib().e2e_sync(ctx, stream))


def e2e_render_batch(ctx, reqs):
    arr = (e2e_render_req * len(reqs))(*reqs)
    return check(lib().e2e_render_batch(ctx, arr, len(reqs)))


def e2e_serve_start(ctx, max_inflight=8, max_queue=256, n_streams=2, max_batch=8):
    cfg = e2e_serve_config(max_inflight, max_queue, n_streams, max_batch)
    return check(lib().e2e_serve_start(ctx, C.byref(cfg)))


def e2e_serve_submit(ctx, req):
    t = C.c_uint64()
    check(lib().e2e_serve_submit(ctx, C.byref(req), C.byref(t)))
    return t.value


def e2e_serve_poll(ctx, ticket, timeout_ms=-1):
    st = e2e_render_stats()
    code = check(lib().e2e_serve_poll(ctx, ticket, timeout_ms, C.byref(st)))
    return code, st


def e2e_serve_stop(ctx):
    return check(lib().e2e_serve_stop(ctx))


def e2e_noise_poisson(ctx, frame_ptr, dtype, n_pixels, seed, frame_index, on_device,
                      stream=None):
    return check(lib().e2e_noise_poisson(ctx, frame_ptr, dtype, n_pixels, seed, frame_index,
                                         on_device, stream))


def e2e_detector(ctx, desc, frame_ptr, frame_dtype, prnu_ptr, nx, ny, adu_ptr, on_device,
                 stream=None):
    """Detector stage (PRNU, dark current, shot noise, cross-talk, read noise,
    ADC) of an nx x ny frame into uint16 ADU; pointers as in the C call."""
    return check(lib().e2e_detector(ctx, C.byref(desc), frame_ptr, frame_dtype, prnu_ptr, nx,
                                    ny, adu_ptr, on_device, stream))


def e2e_extract(ctx, fmt, frame_ptr, frame_dtype, aperture_half_px, flux_ptr, edges_ptr,
                on_device, stream=None):
    """Box extraction of every trace: flux [ntr][nx], edge wavelengths [ntr][nx+1]."""
    return check(lib().e2e_extract(ctx, fmt, frame_ptr, frame_dtype, aperture_half_px, flux_ptr,
                                   edges_ptr, on_device, stream))


def e2e_ccf(ctx, fmt, req):
    """CCF of extracted spectra with the smoothed templates; returns the RV (m/s)."""
    rv = C.c_double()
    check(lib().e2e_ccf(ctx, fmt, C.byref(req), C.byref(rv)))
    return rv.value


def e2e_philox_blocks(ctx, seed, frame_index, pixel0, n_pixels, blocks):
    out = (C.c_uint32 * (4 * n_pixels * blocks))()
    check(lib().e2e_philox_blocks(ctx, seed, frame_index, pixel0, n_pixels, blocks, out))
    return out


def e2e_set_profiling(ctx, on):
    return check(lib().e2e_set_profiling(ctx, 1 if on else 0))


def e2e_autotune(ctx, reqs):
    """Time the candidate launch choices on `reqs` and keep the fastest for
    their workload shapes; returns the e2e_tune_report."""
    arr = (e2e_render_req * len(reqs))(*reqs)
    rep = e2e_tune_report()
    check(lib().e2e_autotune(ctx, arr, len(reqs), C.byref(rep)))
    return rep


def e2e_kernel_time(ctx, name):
    n = C.c_int64()
    ms = C.c_double()
    check(lib().e2e_kernel_time(ctx, name.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def e2e_reset_kernel_time(ctx):
    return check(lib().e2e_reset_kernel_time(ctx))
