"""Seeded synthetic inputs shaped like the paper's ESPRESSO / ELT-HIRES frames.

Every random number comes from NumPy's PCG64 seeded explicitly, so a scene is
a pure function of (name, seed).  The shapes follow the paper's description of
its two instruments: cross-dispersed echelle orders whose traces are curved
(Sec. 4.1, Fig. 6), several fibers and pupil slices per order (Sec. 4.1:
two fibers x two slices for ESPRESSO; Sec. 4.2: bundles of fibers for
HIRES), a spectral-format database of per-SFI centroid positions (Sec. 2.1)
stored here as per-trace polynomials, PSF maps per wavelength / field
(Sec. 2.1: asymmetric Gaussians or ray-traced maps) stored as tables of
cell integrals, and a source spectrum in photons per wavelength sample
(Sec. 2, Science Object Module).  The real instruments' optical design
files, spectra and frames are not available; these inputs stand in for them.

Conventions shared with the renderer interface (not arithmetic of it):
  * a trace spans [lmin, lmax] nm with ``n`` samples; the spectrum array of
    that trace's slot holds the photons of sample k, tabulated on the
    cell-centred grid lmin + (k + 1/2) (lmax - lmin) / n;
  * polynomial coefficients are in ascending powers of the normalised
    wavelength t in [-1, 1] and give detector pixels (0-based, pixel centres
    at integers, frame row-major [y][x]);
  * PSF tables are [gy][gx][kh][kw] float32 cell integrals summing to 1,
    kernels centred on the table centre, ``os`` cells per pixel.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

C_LIGHT = 299792458.0  # m/s, exact by definition of the metre


@dataclass
class Trace:
    order: int
    fiber: int
    slice: int
    lmin: float
    lmax: float
    n: int
    cx: List[float]          # x(t) coefficients, ascending powers
    cy: List[float]          # y(t) coefficients, ascending powers
    thr: float               # throughput of this trace
    slot: int                # index of the spectrum this trace reads


@dataclass
class Psf:
    kind: str                          # 'erf' | 'table' | 'separable' | 'sfi'
    sigma: float = 0.0                 # erf: Gaussian sigma in px
    half_width: int = 0                # erf / separable / sfi: footprint radius H
    gx: int = 1
    gy: int = 1
    kw: int = 0
    kh: int = 0
    os: int = 4
    tables: Optional[np.ndarray] = None    # [gy][gx][kh][kw] float32
    sigma_xy: Optional[np.ndarray] = None  # [gy][gx][2] float32 (sx, sy)
    fiber_radius: float = 0.0          # sfi: fiber image radius in px
    fiber_shape: str = "disc"          # sfi: 'disc' | 'half_up' | 'half_down'
    subpix: int = 10                   # sfi: sub-pixels per pixel side


@dataclass
class Scene:
    name: str
    nx: int
    ny: int
    traces: List[Trace]
    psf: Psf
    spectra: List[np.ndarray]          # one array per slot
    out_dtype: str = "f32"             # 'f32' | 'f64'

    @property
    def n_samples(self) -> int:
        return int(sum(t.n for t in self.traces))

    def footprint_px(self) -> int:
        """Pixels in one sample's PSF footprint (the update count per sample)."""
        p = self.psf
        if p.kind in ("erf", "separable", "sfi"):
            return (2 * p.half_width + 1) ** 2
        wx = (p.kw + p.os - 1) // p.os + 1
        wy = (p.kh + p.os - 1) // p.os + 1
        return wx * wy

    def updates(self) -> int:
        return self.n_samples * self.footprint_px()

    def spectrum_bytes(self) -> int:
        return int(sum(s.nbytes for s in self.spectra))


@dataclass
class Request:
    rv_mps: float = 0.0
    flux_scale: float = 1.0
    seed: int = 0
    frame_index: int = 0
    poisson: bool = False
    precision: str = "f64"   # 'f64' | 'f32' | 'bf16_hilo' | 'f16_hilo'


# ---------------------------------------------------------------------------
# spectra

def _sample_grid(lmin: float, lmax: float, n: int) -> np.ndarray:
    return lmin + (np.arange(n, dtype=np.float64) + 0.5) * ((lmax - lmin) / n)


def _absorb_lines(flux: np.ndarray, lam: np.ndarray, centres, depths, sig_nm):
    """Multiply flux by prod(1 - d exp(-((lam - c)/s)^2 / 2)) (lines within 8 s)."""
    step = (lam[-1] - lam[0]) / max(len(lam) - 1, 1)
    for c, d, s in zip(centres, depths, sig_nm):
        lo = int(np.floor((c - 8 * s - lam[0]) / step)) - 1
        hi = int(np.ceil((c + 8 * s - lam[0]) / step)) + 2
        lo, hi = max(lo, 0), min(hi, len(lam))
        if lo >= hi:
            continue
        z = (lam[lo:hi] - c) / s
        flux[lo:hi] *= 1.0 - d * np.exp(-0.5 * z * z)


def stellar_spectrum(lam: np.ndarray, line_c, line_d, line_s, cont=1e4):
    flux = np.full(lam.shape, cont, dtype=np.float64)
    sel = (line_c > lam[0] - 10 * line_s) & (line_c < lam[-1] + 10 * line_s)
    _absorb_lines(flux, lam, line_c[sel], line_d[sel], line_s[sel])
    return flux


def fabry_perot(lam: np.ndarray, finesse=12.0, fsr_nm=0.02, peak=1e4):
    """Airy transmission with coefficient of finesse F = (2 finesse / pi)^2."""
    F = (2.0 * finesse / np.pi) ** 2
    s = np.sin(np.pi * lam / fsr_nm)
    return peak / (1.0 + F * s * s)


# ---------------------------------------------------------------------------
# PSF tables

def elliptical_gaussian_tables(rng, gx, gy, kw, kh, os_, smin=1.0, smax=1.6,
                               sub=4):
    """Cell integrals of rotated elliptical Gaussians, one kernel per node.

    Each cell integral is a sub x sub Gauss-Legendre quadrature; each kernel
    is normalised to sum 1 in FP64 and stored as float32.
    """
    xg, wg = np.polynomial.legendre.leggauss(sub)
    # cell a spans [-kw/(2 os) + a/os, ... + 1/os) px relative to the centre
    ax = (-kw / (2.0 * os_) + (np.arange(kw)[:, None] + 0.5 + 0.5 * xg[None, :]) / os_)
    ay = (-kh / (2.0 * os_) + (np.arange(kh)[:, None] + 0.5 + 0.5 * xg[None, :]) / os_)
    X = ax.reshape(-1)[None, :]
    Y = ay.reshape(-1)[:, None]
    W = np.outer(np.tile(wg, kh), np.tile(wg, kw))
    tabs = np.empty((gy, gx, kh, kw), dtype=np.float32)
    for l in range(gy):
        for m in range(gx):
            s1, s2 = np.sort(rng.uniform(smin, smax, 2))[::-1]
            th = rng.uniform(0.0, np.pi)
            c, s = np.cos(th), np.sin(th)
            u = c * X + s * Y
            v = -s * X + c * Y
            g = np.exp(-0.5 * ((u / s1) ** 2 + (v / s2) ** 2)) * W
            cell = g.reshape(kh, sub, kw, sub).sum(axis=(1, 3))
            cell /= cell.sum()
            tabs[l, m] = cell.astype(np.float32)
    return tabs


# ---------------------------------------------------------------------------
# echelle geometry

def _echelle(rng, *, nx, ny, orders, G, n_fib, n_sli, n_samp, xc, xh,
             a_bounds, b_total, y0, pitch, offsets, x_slice_offset,
             ext=1.05):
    traces: List[Trace] = []
    for oi, m in enumerate(orders):
        lc = G / m
        half = ext * lc / (2.0 * m)
        lmin, lmax = lc - half, lc + half
        a = [rng.uniform(-b, b) for b in a_bounds]
        bw = rng.dirichlet(np.ones(3)) * rng.uniform(0.3, 1.0) * b_total
        bsg = rng.choice([-1.0, 1.0], 3)
        b = list(bw * bsg)
        ym = y0 + pitch * oi
        for f in range(n_fib):
            for s in range(n_sli):
                off = offsets[f * n_sli + s]
                cx = [xc + (x_slice_offset if s % 2 == 1 else 0.0), xh] + a
                cy = [ym + off] + b
                traces.append(Trace(order=int(m), fiber=f, slice=s, lmin=lmin,
                                    lmax=lmax, n=int(n_samp), cx=cx, cy=cy,
                                    thr=1.0 / n_sli, slot=oi * n_fib + f))
    return traces


def _spectra_for(traces, n_fib, fiber_kind, rng, n_lines, lam_lo, lam_hi, G,
                 dtype, ext=1.05, depth_hi=0.95):
    line_c = rng.uniform(lam_lo, lam_hi, n_lines)
    line_d = rng.uniform(0.0, depth_hi, n_lines)
    fw_samp = rng.uniform(2.0, 6.0, n_lines)
    nslot = max(t.slot for t in traces) + 1
    spectra: List[Optional[np.ndarray]] = [None] * nslot
    for t in traces:
        if spectra[t.slot] is not None:
            continue
        lam = _sample_grid(t.lmin, t.lmax, t.n)
        kind = fiber_kind[t.fiber]
        if kind == "star":
            # line FWHM given in samples of the order that holds the line
            step = (t.lmax - t.lmin) / t.n
            s_nm = fw_samp * step / 2.3548200450309493
            spec = stellar_spectrum(lam, line_c, line_d, s_nm)
        elif kind == "fp":
            spec = fabry_perot(lam)
        else:
            spec = np.full(lam.shape, 1e4)
        spectra[t.slot] = spec.astype(dtype)
    return spectra


# ---------------------------------------------------------------------------
# named scenes

CONFIG_NOTES: Dict[str, str] = {
    "c0": "512x256 FP64, 1 trace (500-505 nm over 480 px), 20,000 samples, "
          "erf Gaussian sigma=1.2 px on 11x11",
    "c1": "9216x9216 FP32, 85 orders x 2 fibers x 2 slices, 1e6 samples per "
          "trace, 11x11 nodes of 32x32 x4 elliptical-Gaussian tables",
    "c2": "c1 geometry, separable PSF: 11x11 nodes of (sx, sy) in [1.0,1.6], R=8",
    "c3v": "4096x4096, 40 orders x 1 fiber x 2 slices, 1e6 samples, c1 PSF kind",
    "c4": "6144x6144, 120 orders x 4 fibers x 3 slices, 2e6 samples, 15x15 "
          "nodes of 48x48 x4 tables",
    "c5_sfi": "4096x4096, 40 orders x 2 fibers, 12288 samples per trace (~3 per px, "
              "10 per resolution element), explicit SFI: disc rho=1.5 px (x) Gaussian "
              "(sx, sy) in [0.8, 1.2] on 11x11 nodes, 11x11 px at 0.1-px sub-sampling",
}


def _c0(seed, **kw):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = kw.get("n", 20000)
    a2, a3 = rng.dirichlet(np.ones(2)) * rng.uniform(0.5, 3.0) * rng.choice([-1.0, 1.0], 2)
    b1, b2 = rng.dirichlet(np.ones(2)) * rng.uniform(5.0, 20.0) * rng.choice([-1.0, 1.0], 2)
    tr = Trace(order=0, fiber=0, slice=0, lmin=500.0, lmax=505.0, n=n,
               cx=[256.0, 240.0, float(a2), float(a3)],
               cy=[128.0, float(b1), float(b2)], thr=1.0, slot=0)
    # 50 absorption lines, multiplicative, centres >= 50 samples from the ends
    ck = rng.uniform(50, n - 50, 50)
    dep = rng.uniform(0.1, 0.9, 50)
    fw = rng.uniform(2.0, 6.0, 50)
    k = np.arange(n, dtype=np.float64)
    spec = np.full(n, 1e4)
    for c, d, f in zip(ck, dep, fw):
        s = f / 2.3548200450309493
        spec *= 1.0 - d * np.exp(-0.5 * ((k - c) / s) ** 2)
    psf = Psf(kind="erf", sigma=kw.get("sigma", 1.2),
              half_width=kw.get("half_width", 5))
    return Scene("c0", 512, 256, [tr], psf, [spec.astype(np.float64)], "f64")


def _espresso(seed, *, nx, ny, orders, n_samp, gx, kwid, psf_kind, name,
              n_fib=2, n_sli=2, xc=None, xh=None, y0=300.0, pitch=100.0,
              n_lines=20000, spec_dtype=np.float32, out_dtype="f32",
              fiber_kind=("star", "fp"), a_scale=1.0, b_total=20.0,
              sep_R=8, G=61600.0, sfi=None, sig_range=(1.0, 1.6)):
    rng = np.random.Generator(np.random.PCG64(seed))
    xc = nx / 2.0 if xc is None else xc
    xh = 4300.0 * nx / 9216.0 if xh is None else xh
    offsets = [-15.0 + 10.0 * i for i in range(n_fib * n_sli)]
    traces = _echelle(rng, nx=nx, ny=ny, orders=orders, G=G, n_fib=n_fib,
                      n_sli=n_sli, n_samp=n_samp, xc=xc, xh=xh,
                      a_bounds=[50.0 * a_scale, 100.0 * a_scale, 20.0 * a_scale],
                      b_total=b_total, y0=y0, pitch=pitch, offsets=offsets,
                      x_slice_offset=0.85)
    lam_lo = min(t.lmin for t in traces)
    lam_hi = max(t.lmax for t in traces)
    spectra = _spectra_for(traces, n_fib, list(fiber_kind), rng, n_lines,
                           lam_lo, lam_hi, G, spec_dtype)
    if psf_kind == "table":
        tabs = elliptical_gaussian_tables(rng, gx, gx, kwid, kwid, 4)
        psf = Psf(kind="table", gx=gx, gy=gx, kw=kwid, kh=kwid, os=4,
                  tables=tabs)
    elif psf_kind == "sfi":
        # explicit SFI (Sec. 2.2): fiber disc (or half) of radius rho px,
        # Gaussian PSF field on the node grid, sub-pixel sampling
        sig = rng.uniform(*sig_range, (gx, gx, 2)).astype(np.float32)
        psf = Psf(kind="sfi", gx=gx, gy=gx, half_width=sfi.get("H", 5), sigma_xy=sig,
                  fiber_radius=sfi.get("rho", 1.5), fiber_shape=sfi.get("shape", "disc"),
                  subpix=sfi.get("S", 10))
    else:
        sig = rng.uniform(*sig_range, (gx, gx, 2)).astype(np.float32)
        psf = Psf(kind="separable", gx=gx, gy=gx, half_width=sep_R,
                  sigma_xy=sig)
    return Scene(name, nx, ny, traces, psf, spectra, out_dtype)


def _hires(seed, *, nx=6144, ny=6144, n_orders=120, n_samp=2_000_000, gx=15,
           kwid=48, name="c4", n_lines=20000, spec_dtype=np.float32,
           y0=36.0, pitch=51.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    G = 95000.0
    orders = list(range(100, 100 + n_orders))
    n_fib, n_sli = 4, 3
    offsets = [-22.0 + 4.0 * i for i in range(n_fib * n_sli)]
    traces = _echelle(rng, nx=nx, ny=ny, orders=orders, G=G, n_fib=n_fib,
                      n_sli=n_sli, n_samp=n_samp, xc=nx / 2.0,
                      xh=2900.0 * nx / 6144.0,
                      a_bounds=[35.0, 70.0, 14.0], b_total=14.0,
                      y0=y0, pitch=pitch, offsets=offsets,
                      x_slice_offset=0.0)
    lam_lo = min(t.lmin for t in traces)
    lam_hi = max(t.lmax for t in traces)
    spectra = _spectra_for(traces, n_fib, ["star", "star", "fp", "flat"], rng,
                           n_lines, lam_lo, lam_hi, G, spec_dtype)
    tabs = elliptical_gaussian_tables(rng, gx, gx, kwid, kwid, 4)
    psf = Psf(kind="table", gx=gx, gy=gx, kw=kwid, kh=kwid, os=4, tables=tabs)
    return Scene(name, nx, ny, traces, psf, spectra, "f32")


def _mini_table(seed, nx=512, ny=452, n_orders=4, n_samp=20000, **kw):
    return _espresso(seed, nx=nx, ny=ny, orders=list(range(78, 78 + n_orders)),
                     n_samp=n_samp, gx=kw.pop("gx", 11), kwid=kw.pop("kwid", 32),
                     psf_kind="table", name=kw.pop("name", "mini_table"),
                     xh=kw.pop("xh", 262.0), y0=kw.pop("y0", 60.0),
                     pitch=kw.pop("pitch", 100.0), n_lines=kw.pop("n_lines", 600),
                     a_scale=kw.pop("a_scale", 0.06), b_total=kw.pop("b_total", 6.0),
                     **kw)


SCENES = {
    "c0": lambda seed=1000, **kw: _c0(seed, **kw),
    "c1": lambda seed=1001, **kw: _espresso(
        seed, nx=9216, ny=9216, orders=list(range(78, 163)), n_samp=1_000_000,
        gx=11, kwid=32, psf_kind="table", name="c1", **kw),
    "c2": lambda seed=1002, **kw: _espresso(
        seed, nx=9216, ny=9216, orders=list(range(78, 163)), n_samp=1_000_000,
        gx=11, kwid=0, psf_kind="separable", name="c2", **kw),
    "c3v": lambda seed=1003, **kw: _espresso(
        seed, nx=4096, ny=4096, orders=list(range(78, 118)), n_samp=1_000_000,
        gx=11, kwid=32, psf_kind="table", name="c3v", n_fib=1, n_sli=2,
        fiber_kind=("star",), xh=1900.0, y0=100.0, pitch=100.0, **kw),
    "c4": lambda seed=1004, **kw: _hires(seed, **kw),
    "c5_sfi": lambda seed=1005, **kw: _espresso(
        seed, nx=4096, ny=4096, orders=list(range(78, 118)), n_samp=12288, gx=11, kwid=0,
        psf_kind="sfi", name="c5_sfi", n_sli=1, xh=1900.0, y0=100.0, pitch=100.0,
        sig_range=(0.8, 1.2), sfi=kw.pop("sfi", {"rho": 1.5, "shape": "disc", "S": 10, "H": 5}),
        **kw),
    # reduced shapes the oracle renders in seconds; several tiles + ragged tails
    "mini_table": lambda seed=2001, **kw: _mini_table(seed, **kw),
    "mini_sep": lambda seed=2002, **kw: _espresso(
        seed, nx=512, ny=452, orders=list(range(78, 82)), n_samp=20000, gx=11,
        kwid=0, psf_kind="separable", name="mini_sep", xh=262.0, y0=60.0,
        pitch=100.0, n_lines=600, a_scale=0.06, b_total=6.0, **kw),
    "mini_hires": lambda seed=2004, **kw: _hires(
        seed, nx=600, ny=420, n_orders=7, n_samp=12000, gx=15, kwid=48,
        name="mini_hires", n_lines=400, y0=40.0, **kw),
    "mini_sfi": lambda seed=2005, **kw: _espresso(
        seed, nx=120, ny=72, orders=[80], n_samp=kw.pop("n_samp", 200), gx=2, kwid=0,
        psf_kind="sfi", name="mini_sfi", n_fib=1, n_sli=1, fiber_kind=("star",),
        xh=40.0, y0=51.0, n_lines=20, a_scale=0.01, b_total=3.0, spec_dtype=np.float64,
        out_dtype="f64", sig_range=(0.7, 1.2),
        sfi=kw.pop("sfi", {"rho": 1.1, "shape": "disc", "S": 10, "H": 5}), **kw),
    "mini_c3v": lambda seed=2003, **kw: _mini_table(
        seed, nx=384, ny=320, n_orders=3, n_samp=15000, n_fib=1,
        fiber_kind=("star",), name="mini_c3v", xh=170.0, **kw),
}


def scene(name: str, seed: Optional[int] = None, **kw) -> Scene:
    f = SCENES[name]
    return f(**kw) if seed is None else f(seed, **kw)


def request(rng_or_seed=None, *, rv_range=(0.0, 0.0), flux_range=(1.0, 1.0),
            **kw) -> Request:
    rng = (rng_or_seed if isinstance(rng_or_seed, np.random.Generator)
           else np.random.Generator(np.random.PCG64(rng_or_seed or 0)))
    rv = rng.uniform(*rv_range) if rv_range[1] > rv_range[0] else rv_range[0]
    fs = rng.uniform(*flux_range) if flux_range[1] > flux_range[0] else flux_range[0]
    return Request(rv_mps=float(rv), flux_scale=float(fs), **kw)


def with_traces(sc: Scene, idx) -> Scene:
    """A copy of a scene restricted to some traces (spectra shared)."""
    return dataclasses.replace(sc, traces=[sc.traces[i] for i in idx])


def detector_frame(nx: int, ny: int, seed: int = 0, *, spacing: float = 27.0,
                   sigma: float = 1.6, peak: float = 7e5, bg: float = 20.0,
                   dtype=np.float32) -> np.ndarray:
    """Expected photo-electrons [ny][nx] with an echellogram's value mix, for
    the detector stage: curved bright bands every `spacing` rows (Gaussian
    cross profile, blaze-shaped along x, peak about `peak`) over a faint
    background (Sec. 4.1 frames reach a few 1e5 e- per pixel in their
    orders)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.arange(nx, dtype=np.float32)[None, :]
    y = np.arange(ny, dtype=np.float32)[:, None]
    ph = np.float32(rng.uniform(0.0, 2 * np.pi))
    curve = np.float32(0.5 * spacing) * np.sin(np.float32(2.6 * np.pi / max(nx, 1)) * x + ph)
    d = np.mod(y - curve, np.float32(spacing)) - np.float32(0.5 * spacing)
    blaze = np.float32(peak) * (np.float32(0.2) + np.float32(0.8) *
                                np.sin(np.float32(np.pi) * (x + 0.5) / np.float32(max(nx, 1))) ** 2)
    F = np.float32(bg) + blaze * np.exp(np.float32(-0.5) * (d / np.float32(sigma)) ** 2)
    return np.ascontiguousarray(F.astype(dtype, copy=False))


def prnu_map(nx: int, ny: int, seed: int = 0, rms: float = 0.01) -> np.ndarray:
    """Pixel response map [ny][nx] (FP32): 1 + rms * N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed + 0x5EED))
    g = rng.standard_normal((ny, nx), dtype=np.float32)
    return np.ascontiguousarray(np.float32(1.0) + np.float32(rms) * g)


# Cross-talk kernel K[dy+1][dx+1] of a deep-depletion CCD: a pixel keeps
# ~97.6 % of its charge and hands the rest to its four / eight neighbours,
# slightly more along the read-out columns (values illustrative).
XTALK_CCD = np.array([[0.0010, 0.0060, 0.0010],
                      [0.0040, 0.9760, 0.0040],
                      [0.0010, 0.0060, 0.0010]], dtype=np.float64)


def aliasing_flat(per_res: float, subpix: int, *, seed: int = 3001, length_px: float = 1000.0,
                  px_per_res: float = 4.5, rho: float = 2.0, sigma: float = 0.8,
                  half_width: int = 5, ny: int = 32) -> Scene:
    """Flat-field segment of one order, shaped after Fig. 4's ESPRESSO blue
    arm (resolution element 0.02 A sampled by about 4.5 px, 10 SFIs per
    element): a straight trace across `length_px` px, a constant spectrum of
    `per_res` samples per resolution element, explicit SFIs (fiber disc of
    radius rho px, Gaussian PSF sigma px) at `subpix` sub-pixels per pixel.
    Photons per sample are set so that the trace's central row receives
    about 4e4 e- per pixel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx = int(length_px) + 4 * half_width + 8
    n = int(round(length_px / px_per_res * per_res))
    x0 = 2 * half_width + 4 + rng.uniform(0.0, 1.0)
    lc, span = 450.0, 0.002 * length_px / px_per_res           # nm; 0.02 A per element
    tr = Trace(order=146, fiber=0, slice=0, lmin=lc - span / 2, lmax=lc + span / 2, n=n,
               cx=[x0 + length_px / 2, length_px / 2], cy=[ny / 2 + rng.uniform(-0.5, 0.5)],
               thr=1.0, slot=0)
    # central-row fraction of a disc (x) Gaussian image, about 0.2 for these sizes
    phot = 4e4 / 0.21 * px_per_res / per_res
    sxy = np.full((1, 1, 2), sigma, np.float32)
    psf = Psf(kind="sfi", half_width=half_width, sigma_xy=sxy, fiber_radius=rho,
              fiber_shape="disc", subpix=subpix)
    return Scene("aliasing_flat", nx, ny, [tr], psf, [np.full(n, phot, np.float32)], "f64")
