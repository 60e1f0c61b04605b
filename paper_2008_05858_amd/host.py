"""Argument marshalling from Python objects to the e2e C structs.

A *scene* is any object with ``nx``, ``ny``, ``traces`` (objects with order,
fiber, slice, lmin, lmax, n, cx, cy, thr, slot) and ``psf`` (kind, sigma,
half_width, gx, gy, kw, kh, os, tables, sigma_xy), such as the seeded
workloads of the test suite.  Nothing here computes any part of a frame.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import e2e as E

_KIND = {"erf": E.E2E_PSF_GAUSS_ERF, "table": E.E2E_PSF_TABLE,
         "separable": E.E2E_PSF_SEPARABLE, "sfi": E.E2E_PSF_SFI}
_FIBER = {"disc": E.E2E_FIBER_DISC, "half_up": E.E2E_FIBER_HALF_UP,
          "half_down": E.E2E_FIBER_HALF_DOWN}
PRECISION = {"f64": E.E2E_PREC_F64, "f32": E.E2E_PREC_F32,
             "bf16_hilo": E.E2E_PREC_BF16_HILO, "f16_hilo": E.E2E_PREC_F16_HILO}


def trace_descs(traces):
    """Array of e2e_trace_desc plus the buffers it points into."""
    arr = (E.e2e_trace_desc * len(traces))()
    keep = []
    for i, t in enumerate(traces):
        cx = np.ascontiguousarray(t.cx, np.float64)
        cy = np.ascontiguousarray(t.cy, np.float64)
        keep += [cx, cy]
        arr[i] = E.e2e_trace_desc(int(t.order), int(t.fiber), int(t.slice), float(t.lmin),
                                  float(t.lmax), int(t.n), len(cx) - 1, len(cy) - 1,
                                  cx.ctypes.data_as(C.POINTER(C.c_double)),
                                  cy.ctypes.data_as(C.POINTER(C.c_double)), float(t.thr),
                                  int(t.slot))
    return arr, keep


def psf_desc(p):
    keep = []
    tab = sxy = None
    if getattr(p, "tables", None) is not None:
        tab = np.ascontiguousarray(p.tables, np.float32)
        keep.append(tab)
    if getattr(p, "sigma_xy", None) is not None:
        sxy = np.ascontiguousarray(p.sigma_xy, np.float32)
        keep.append(sxy)
    d = E.e2e_psf_desc(_KIND[p.kind], float(p.sigma), int(p.half_width), int(p.gx), int(p.gy),
                       int(p.kw), int(p.kh), int(p.os),
                       tab.ctypes.data_as(C.POINTER(C.c_float)) if tab is not None else None,
                       sxy.ctypes.data_as(C.POINTER(C.c_float)) if sxy is not None else None,
                       float(getattr(p, "fiber_radius", 0.0)),
                       _FIBER[getattr(p, "fiber_shape", "disc")], int(getattr(p, "subpix", 10)))
    return d, keep


class Loaded:
    """Device-resident format + PSF tables of one scene."""

    def __init__(self, ctx, scene):
        self.ctx = ctx
        arr, keep = trace_descs(scene.traces)
        self.fmt = E.e2e_format_load(ctx, arr, len(scene.traces), scene.nx, scene.ny)
        d, keep2 = psf_desc(scene.psf)
        try:
            self.psf = E.e2e_psf_load(ctx, d)
        except Exception:
            E.e2e_format_free(ctx, self.fmt)
            raise
        self.nx, self.ny = scene.nx, scene.ny
        self.n_slots = max(int(t.slot) for t in scene.traces) + 1

    def free(self):
        E.e2e_format_free(self.ctx, self.fmt)
        E.e2e_psf_free(self.ctx, self.psf)


def make_req(loaded, spectra_ptrs, spectrum_dtype, out_ptr, out_dtype, *, spectra_on_device,
             out_on_device, rv_mps=0.0, flux_scale=1.0, seed=0, frame_index=0, poisson=False,
             precision="f64", stream=None, flags=0):
    """An e2e_render_req; the returned tuple's second item keeps arrays alive."""
    arr = (C.c_void_p * len(spectra_ptrs))(*[C.c_void_p(int(p)) for p in spectra_ptrs])
    r = E.e2e_render_req(loaded.fmt, loaded.psf, C.cast(arr, C.POINTER(C.c_void_p)),
                         len(spectra_ptrs), spectrum_dtype, 1 if spectra_on_device else 0,
                         float(rv_mps), float(flux_scale), int(seed), int(frame_index),
                         1 if poisson else 0, PRECISION.get(precision, precision),
                         C.c_void_p(int(out_ptr)), out_dtype, 1 if out_on_device else 0,
                         C.c_void_p(int(stream)) if stream else None, int(flags))
    return r, arr
