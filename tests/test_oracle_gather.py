"""Pin of the oracle's per-pixel gather form against its scatter form.

Every full-size parity test evaluates the oracle one pixel at a time
(`render_pixels`: for each trace, the samples whose footprint can reach the
pixel are found by bisection on the monotone x(lambda), and only those are
summed).  The scatter form (`render`) is the plain definition: every sample
of every trace spread over its whole footprint (Sec. 2, Sec. 2.2).  Both
sum the same products in the same order (trace ascending, sample
ascending), so a pixel must come out identical; a reach or bisection
mistake in the gather form (a sample dropped at a footprint edge, an
off-by-one at a trace end, a Doppler shift applied on one side only) would
show up here and not move blame onto the GPU.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from workloads import Psf, Request, Scene, Trace, scene
from workloads.synth import with_traces


def _pick_pixels(frame, n_lit, n_rand, seed):
    """Corners, edge strips, lit pixels (weighted to the bright ones) and
    uniform random pixels."""
    ny, nx = frame.shape
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)}
    for i in np.linspace(0, nx - 1, 12).astype(int):
        pts.add((int(i), 0))
        pts.add((int(i), ny - 1))
    for j in np.linspace(0, ny - 1, 12).astype(int):
        pts.add((0, int(j)))
        pts.add((nx - 1, int(j)))
    jj, ii = np.nonzero(frame > 0)
    if jj.size:
        w = frame[jj, ii] / frame[jj, ii].sum()
        for q in rng.choice(jj.size, size=min(n_lit, jj.size), replace=False, p=w):
            pts.add((int(ii[q]), int(jj[q])))
        # and the dim fringe of the footprints, where reach mistakes live
        dim = np.nonzero(frame[jj, ii] < 1e-3 * frame.max())[0]
        for q in rng.choice(dim, size=min(n_lit // 2, dim.size), replace=False):
            pts.add((int(ii[q]), int(jj[q])))
    for _ in range(n_rand):
        pts.add((int(rng.integers(0, nx)), int(rng.integers(0, ny))))
    p = np.array(sorted(pts))
    return p[:, 0], p[:, 1]


def _off_edge_table_scene():
    """A tabulated-PSF trace that starts left of the detector, leaves through
    the right edge and grazes the bottom edge, with a field grid of 2 x 2."""
    rng = np.random.default_rng(11)
    u = (np.arange(32) + 0.5) / 4 - 4
    tabs = np.zeros((2, 2, 32, 32), np.float32)
    for a in range(2):
        for b in range(2):
            sx, sy = rng.uniform(1.0, 1.6, 2)
            K = np.exp(-0.5 * (u[:, None] ** 2 / sy ** 2 + u[None, :] ** 2 / sx ** 2))
            tabs[a, b] = (K / K.sum()).astype(np.float32)
    psf = Psf(kind="table", gx=2, gy=2, kw=32, kh=32, os=4, tables=tabs)
    n = 3000
    tr = Trace(0, 0, 0, 600.0, 603.0, n, [60.0, 70.0, 3.0, -1.5], [2.2, 1.4, 0.8], 0.7, 0)
    spec = rng.uniform(0.5, 1.5, n) * 1e4
    return Scene("off_edge_table", 120, 40, [tr], psf, [spec.astype(np.float32)], "f32")


def _sfi_edges(**kw):
    """An explicit-SFI trace running over the left, right and bottom edges
    (x from -6 to 126 px on a 120-px detector)."""
    sc = scene("mini_sfi", **kw)
    t = sc.traces[0]
    return dataclasses.replace(sc, traces=[dataclasses.replace(t, cx=[60.0, 66.0],
                                                               cy=[1.3, 0.4])])


def _hires_third():
    sc = scene("mini_hires")
    return with_traces(sc, list(range(0, len(sc.traces), 3)))


# (name, scene, request, lit pixels, random pixels): the explicit-SFI oracle
# spends ~10 ms per sample window, so its cases sample fewer pixels
CASES = [
    ("c0", lambda: scene("c0"), Request(rv_mps=-2150.0, flux_scale=1.5), 300, 150),
    ("mini_table", lambda: scene("mini_table"), Request(rv_mps=9.25, flux_scale=0.37), 300, 150),
    ("mini_hires", _hires_third, Request(rv_mps=-3.0), 300, 150),
    ("mini_sep", lambda: scene("mini_sep"), Request(rv_mps=4.0), 300, 150),
    ("mini_sfi_disc", lambda: _sfi_edges(n_samp=80, sfi={"rho": 1.1, "shape": "disc", "S": 4,
                                                          "H": 5}),
     Request(rv_mps=500.0), 70, 20),
    ("mini_sfi_half", lambda: _sfi_edges(n_samp=60, sfi={"rho": 1.3, "shape": "half_up",
                                                          "S": 3, "H": 6}),
     Request(rv_mps=-800.0), 70, 20),
    ("off_edge_table", _off_edge_table_scene, Request(rv_mps=3.0, flux_scale=2.0), 300, 150),
]


@pytest.mark.parametrize("name,make,rq,n_lit,n_rand", CASES, ids=[c[0] for c in CASES])
def test_gather_form_equals_scatter_form(name, make, rq, n_lit, n_rand):
    sc = make()
    full = oracle.render(sc, rq)
    px, py = _pick_pixels(full, n_lit, n_rand, seed=len(name))
    assert px.size >= 100
    g = oracle.render_pixels(sc, rq, px, py)
    ref = full[py, px]
    peak = float(full.max())
    err = float(np.max(np.abs(g - ref))) / peak
    print(f"[{name}] {px.size} px, {int(np.count_nonzero(ref))} lit: "
          f"max |gather - scatter| / peak = {err:.1e}")
    assert err <= 1e-13
    # pixels no sample reaches are exactly zero in both forms
    assert np.array_equal(g == 0.0, ref == 0.0)
