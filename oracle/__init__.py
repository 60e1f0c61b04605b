"""FP64 CPU oracle of the echellogram renderer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library (``include/e2e.h``,
``paper_2008_05858_amd``) never imports, links or calls it.

The arithmetic lives in ``oracle.c`` (plain C, FP64); this module only
marshals :mod:`workloads` scenes into its structs.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class _Scene(C.Structure):
    _fields_ = [("n_traces", C.c_int),
                ("deg_x", C.POINTER(C.c_int)), ("deg_y", C.POINTER(C.c_int)),
                ("cx", C.POINTER(C.c_double)), ("cy", C.POINTER(C.c_double)),
                ("lmin", C.POINTER(C.c_double)), ("lmax", C.POINTER(C.c_double)),
                ("n", C.POINTER(C.c_int64)), ("thr", C.POINTER(C.c_double)),
                ("slot", C.POINTER(C.c_int)), ("spec", C.POINTER(C.c_double)),
                ("spec_off", C.POINTER(C.c_int64)), ("nx", C.c_int), ("ny", C.c_int)]


class _Psf(C.Structure):
    _fields_ = [("kind", C.c_int), ("sigma", C.c_double), ("half_width", C.c_int),
                ("gx", C.c_int), ("gy", C.c_int), ("kw", C.c_int), ("kh", C.c_int),
                ("os", C.c_int), ("tables", C.POINTER(C.c_float)),
                ("sigma_xy", C.POINTER(C.c_float)), ("fiber_radius", C.c_double),
                ("fiber_shape", C.c_int), ("subpix", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Psf), C.c_double,
                                 C.c_double, C.c_int, C.c_int, dp]
        L.orc_render_pixels.argtypes = [C.POINTER(_Scene), C.POINTER(_Psf), C.c_double,
                                        C.c_double, C.c_int, ip, ip, dp]
        L.orc_sample_weights.argtypes = [C.POINTER(_Psf), C.c_int, C.c_int, C.c_double,
                                         C.c_double, ip, ip, ip, ip, dp]
        L.orc_footprint_cap.argtypes = [C.POINTER(_Psf)]
        L.orc_sfi_density.argtypes = [C.c_double] * 3 + [C.c_int] + [C.c_double] * 2
        L.orc_sfi_density.restype = C.c_double
        L.orc_gauss_legendre.argtypes = [C.c_int, dp, dp]
        L.orc_gauss_legendre.restype = None
        L.orc_positions.argtypes = [C.POINTER(_Scene), C.c_int, C.c_double, C.c_int64,
                                    C.c_int64, dp, dp]
        L.orc_positions.restype = None
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_philox4x32_10.restype = None
        L.orc_philox_blocks.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32,
                                        C.POINTER(C.c_uint32)]
        L.orc_philox_blocks.restype = None
        L.orc_poisson_frame.argtypes = [dp, C.c_int64, C.c_uint64, C.c_uint32, dp]
        L.orc_poisson_frame.restype = None
        u16p = C.POINTER(C.c_uint16)
        L.orc_detector.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_double, C.c_double, C.c_int, dp, C.c_double, C.c_double,
                                   C.c_double, C.c_int, C.c_uint64, C.c_uint32, u16p, dp]
        L.orc_detector.restype = None
        L.orc_extract.argtypes = [C.POINTER(_Scene), dp, C.c_double, dp, dp]
        L.orc_extract.restype = None
        L.orc_ccf.argtypes = [C.POINTER(_Scene), dp, dp, dp, C.c_double, C.c_double, C.c_int,
                              C.c_double, dp]
        L.orc_smooth3.argtypes = [dp, C.c_int64, C.c_int, dp]
        L.orc_smooth3.restype = None
        L.orc_ccf.restype = C.c_double
        _lib = L
    return _lib


_lib_omp = None


def lib_omp():
    """The multi-core driver (oracle_omp.c): the same arithmetic, traces over threads."""
    global _lib_omp
    if _lib_omp is None:
        _build.build(force=False)
        L = C.CDLL(_build.LIB_OMP)
        L.orc_render_omp.argtypes = [C.POINTER(_Scene), C.POINTER(_Psf), C.c_double,
                                     C.c_double, C.c_int, C.c_int, C.POINTER(C.c_double),
                                     C.c_int]
        _lib_omp = L
    return _lib_omp


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _Marshalled:
    """Keeps the numpy buffers behind the ctypes structs alive."""

    def __init__(self, sc):
        T = sc.traces
        n = len(T)
        self.deg_x = np.array([len(t.cx) - 1 for t in T], np.int32)
        self.deg_y = np.array([len(t.cy) - 1 for t in T], np.int32)
        self.cx = np.zeros((n, 8)); self.cy = np.zeros((n, 8))
        for i, t in enumerate(T):
            self.cx[i, :len(t.cx)] = t.cx
            self.cy[i, :len(t.cy)] = t.cy
        self.lmin = np.array([t.lmin for t in T], np.float64)
        self.lmax = np.array([t.lmax for t in T], np.float64)
        self.n = np.array([t.n for t in T], np.int64)
        self.thr = np.array([t.thr for t in T], np.float64)
        self.slot = np.array([t.slot for t in T], np.int32)
        used = sorted(set(int(t.slot) for t in T))
        nslot = max(used) + 1
        off = np.zeros(nslot, np.int64)
        parts, pos = [], 0
        for s in range(nslot):
            off[s] = pos
            if s in used:
                a = np.asarray(sc.spectra[s], dtype=np.float64)
                parts.append(a)
                pos += a.size
        self.spec = np.concatenate(parts) if parts else np.zeros(1)
        self.spec_off = off
        self.scene = _Scene(n, _ptr(self.deg_x, C.c_int), _ptr(self.deg_y, C.c_int),
                            _ptr(self.cx, C.c_double), _ptr(self.cy, C.c_double),
                            _ptr(self.lmin, C.c_double), _ptr(self.lmax, C.c_double),
                            _ptr(self.n, C.c_int64), _ptr(self.thr, C.c_double),
                            _ptr(self.slot, C.c_int), _ptr(self.spec, C.c_double),
                            _ptr(self.spec_off, C.c_int64), sc.nx, sc.ny)
        self.psf_keep, self.psf = marshal_psf(sc.psf)


def marshal_psf(p):
    keep = []
    kind = {"erf": 0, "table": 1, "separable": 2, "sfi": 3}[p.kind]
    tab = sxy = None
    if p.tables is not None:
        tab = np.ascontiguousarray(p.tables, dtype=np.float32); keep.append(tab)
    if p.sigma_xy is not None:
        sxy = np.ascontiguousarray(p.sigma_xy, dtype=np.float32); keep.append(sxy)
    s = _Psf(kind, float(p.sigma), int(p.half_width), int(p.gx), int(p.gy),
             int(p.kw), int(p.kh), int(p.os),
             _ptr(tab, C.c_float) if tab is not None else None,
             _ptr(sxy, C.c_float) if sxy is not None else None,
             float(getattr(p, "fiber_radius", 0.0)),
             {"disc": 0, "half_up": 1, "half_down": 2}[getattr(p, "fiber_shape", "disc")],
             int(getattr(p, "subpix", 10)))
    return keep, s


def render(sc, req=None, traces=None):
    """Full FP64 frame [ny][nx] (expected counts, no noise)."""
    rv = req.rv_mps if req is not None else 0.0
    fs = req.flux_scale if req is not None else 1.0
    m = _Marshalled(sc)
    lo, hi = (0, len(sc.traces)) if traces is None else traces
    out = np.zeros((sc.ny, sc.nx), np.float64)
    rc = lib().orc_render(C.byref(m.scene), C.byref(m.psf), rv, fs, lo, hi,
                          _ptr(out, C.c_double))
    if rc != 0:
        raise RuntimeError("oracle render failed")
    return out


def render_omp(sc, req=None, traces=None, threads=0):
    """Full FP64 frame by the multi-core driver: traces over `threads` OpenMP
    threads (0: all), each in its own row band, bands added in trace order."""
    rv = req.rv_mps if req is not None else 0.0
    fs = req.flux_scale if req is not None else 1.0
    m = _Marshalled(sc)
    lo, hi = (0, len(sc.traces)) if traces is None else traces
    out = np.zeros((sc.ny, sc.nx), np.float64)
    rc = lib_omp().orc_render_omp(C.byref(m.scene), C.byref(m.psf), rv, fs, lo, hi,
                                  _ptr(out, C.c_double), int(threads))
    if rc != 0:
        raise RuntimeError("oracle render (multi-core) failed")
    return out


def render_pixels(sc, req, px, py):
    """The same frame evaluated only at pixels (px[q], py[q])."""
    rv = req.rv_mps if req is not None else 0.0
    fs = req.flux_scale if req is not None else 1.0
    m = _Marshalled(sc)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    out = np.zeros(px.size, np.float64)
    rc = lib().orc_render_pixels(C.byref(m.scene), C.byref(m.psf), rv, fs, px.size,
                                 _ptr(px, C.c_int), _ptr(py, C.c_int),
                                 _ptr(out, C.c_double))
    if rc != 0:
        raise RuntimeError("oracle render_pixels failed")
    return out


def sample_weights(psf, nx, ny, x, y):
    """(i0, j0, weights[h][w]) of one sample's footprint at (x, y)."""
    keep, p = marshal_psf(psf)
    cap = lib().orc_footprint_cap(C.byref(p))
    wt = np.zeros(cap, np.float64)
    i0, j0, w, h = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    rc = lib().orc_sample_weights(C.byref(p), nx, ny, float(x), float(y), C.byref(i0),
                                  C.byref(j0), C.byref(w), C.byref(h),
                                  _ptr(wt, C.c_double))
    if rc != 0:
        raise RuntimeError("oracle sample_weights failed")
    return i0.value, j0.value, wt[:w.value * h.value].reshape(h.value, w.value).copy()


SFI_SHAPES = {"disc": 0, "half_up": 1, "half_down": 2}


def sfi_density(u, v, rho, shape, sx, sy):
    """Fiber image (disc / half-disc of radius rho) convolved with the
    axis-aligned Gaussian (sx, sy): photon density at offset (u, v)."""
    return lib().orc_sfi_density(float(u), float(v), float(rho), SFI_SHAPES[shape],
                                 float(sx), float(sy))


def gauss_legendre(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().orc_gauss_legendre(n, _ptr(x, C.c_double), _ptr(w, C.c_double))
    return x, w


def positions(sc, tr, rv_mps, k0, count):
    m = _Marshalled(sc)
    x = np.zeros(count); y = np.zeros(count)
    lib().orc_positions(C.byref(m.scene), tr, rv_mps, k0, count,
                        _ptr(x, C.c_double), _ptr(y, C.c_double))
    return x, y


def philox4x32_10(ctr, key):
    c = np.array(ctr, np.uint32); k = np.array(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def philox_blocks(seed, frame, pixel, nblocks):
    o = np.zeros(4 * nblocks, np.uint32)
    lib().orc_philox_blocks(seed, frame, pixel, nblocks, _ptr(o, C.c_uint32))
    return o


def poisson_frame(mean, seed, frame):
    m = np.ascontiguousarray(mean, np.float64)
    out = np.zeros_like(m)
    lib().orc_poisson_frame(_ptr(m, C.c_double), m.size, seed, frame,
                            _ptr(out, C.c_double))
    return out


def detector(F, *, prnu=None, exposure_s=1.0, dark_e_per_s=0.0, shot_noise=True,
             xtalk=None, ron_e=0.0, gain=1.0, bias=0.0, bits=16, seed=0, frame=0,
             window=None, want_r=False):
    """Detector stage (Sec. 2.2) of an expected-count frame F [ny][nx] (FP64
    oracle): returns uint16 ADU of `window` = (x0, y0, w, h) (default: the
    whole frame), and R (electrons before quantisation) if want_r."""
    F = np.ascontiguousarray(F, np.float64)
    ny, nx = F.shape
    x0, y0, w, h = window if window is not None else (0, 0, nx, ny)
    G = None if prnu is None else np.ascontiguousarray(prnu, np.float64)
    K = np.ascontiguousarray(np.eye(1, 9, 4).reshape(9) if xtalk is None else
                             np.asarray(xtalk, np.float64).reshape(9))
    adu = np.zeros((h, w), np.uint16)
    r = np.zeros((h, w), np.float64) if want_r else None
    lib().orc_detector(_ptr(F, C.c_double), _ptr(G, C.c_double) if G is not None else None,
                       nx, ny, x0, y0, w, h, float(exposure_s), float(dark_e_per_s),
                       1 if shot_noise else 0, _ptr(K, C.c_double), float(ron_e), float(gain),
                       float(bias), int(bits), int(seed), int(frame), _ptr(adu, C.c_uint16),
                       _ptr(r, C.c_double) if want_r else None)
    return (adu, r) if want_r else adu


def extract(sc, frame, aperture_half_px):
    """Box extraction of every trace of a rendered frame [ny][nx] (FP64
    oracle): (E[ntr][nx], L[ntr][nx+1]) -- extracted flux per column and the
    detector-frame wavelength of each column edge (NaN off the trace)."""
    m = _Marshalled(sc)
    F = np.ascontiguousarray(frame, np.float64)
    ntr = len(sc.traces)
    E = np.zeros((ntr, sc.nx)); L = np.zeros((ntr, sc.nx + 1))
    lib().orc_extract(C.byref(m.scene), _ptr(F, C.c_double), float(aperture_half_px),
                      _ptr(E, C.c_double), _ptr(L, C.c_double))
    return E, L


def ccf(sc, E, L, v0, dv, nv, flat=None, smooth_px=1.5):
    """CCF of extracted spectra (divided by the extracted flat, if given)
    against the smoothed input spectra: (C[ntr][nv], rv)."""
    m = _Marshalled(sc)
    E = np.ascontiguousarray(E, np.float64); L = np.ascontiguousarray(L, np.float64)
    Ef = None if flat is None else np.ascontiguousarray(flat, np.float64)
    Cc = np.zeros((len(sc.traces), nv))
    rv = lib().orc_ccf(C.byref(m.scene), _ptr(E, C.c_double),
                       _ptr(Ef, C.c_double) if Ef is not None else None, _ptr(L, C.c_double),
                       float(v0), float(dv), int(nv), float(smooth_px), _ptr(Cc, C.c_double))
    return Cc, rv


def smooth3(x, w):
    """Three passes of the clipped moving mean of odd width w."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros_like(x)
    lib().orc_smooth3(_ptr(x, C.c_double), x.size, int(w), _ptr(y, C.c_double))
    return y
