"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances come from the requirement the paper states for a frame
(Sec. 1, Sec. 2.2): photocentres within 1e-5 px; per pixel we hold every
frame to 1e-6 of its peak.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from workloads import Psf, Request, Scene, Trace, scene
from workloads import metrics

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _gu():
    from tests import gpu_util
    return gpu_util


def _report(name, g, o):
    err = metrics.max_rel_err(g, o)
    print(f"[{name}] max|dF|/peak = {err:.3e}  peak={o.max():.6g}  sum rel={abs(g.sum()-o.sum())/o.sum():.2e}",
          flush=True)
    return err


@pytest.fixture(scope="module")
def mini_table():
    return scene("mini_table")


def test_c0_erf_frame(capsys):
    sc = scene("c0")
    print("case c0 erf FP64", flush=True)
    g = _gu().render(sc)
    o = oracle.render(sc)
    assert _report("c0", g, o) < TOL


def test_c0_erf_frame_with_rv_and_flux():
    sc = scene("c0")
    rq = Request(rv_mps=-2150.0, flux_scale=3.5)
    print("case c0 rv=-2150 fs=3.5", flush=True)
    g = _gu().render(sc, rq)
    o = oracle.render(sc, rq)
    assert _report("c0-rv", g, o) < TOL


def test_mini_table_frame(mini_table):
    print("case mini_table", flush=True)
    g = _gu().render(mini_table)
    o = oracle.render(mini_table)
    assert _report("mini_table", g, o) < TOL


def test_mini_table_rv_flux(mini_table):
    rq = Request(rv_mps=9.25, flux_scale=0.37)
    print("case mini_table rv", flush=True)
    g = _gu().render(mini_table, rq)
    o = oracle.render(mini_table, rq)
    assert _report("mini_table-rv", g, o) < TOL


def test_mini_hires_frame():
    sc = scene("mini_hires")
    print("case mini_hires (48x48 tables, 15x15 nodes, 12 traces/order)", flush=True)
    g = _gu().render(sc)
    o = oracle.render(sc)
    assert _report("mini_hires", g, o) < TOL


@pytest.mark.parametrize("nx,out", [(509, "f64"), (510, "f32"), (508, "f64")])
def test_table_frame_widths_and_fp64_out(nx, out):
    """Table path on frames whose width is not a multiple of four pixels (the
    tile write-out then stores pixel by pixel instead of four at a time) and
    with FP64 output, against the oracle."""
    sc = scene("mini_table", nx=nx, out_dtype=out)
    rq = Request(rv_mps=2.0)
    print(f"case mini_table nx={nx} out={out}", flush=True)
    g = _gu().render(sc, rq)
    o = oracle.render(sc, rq)
    assert g.dtype == (np.float64 if out == "f64" else np.float32)
    assert _report(f"mini_table nx={nx} {out}", g, o) < TOL


@pytest.mark.parametrize("seed", [2001, 2011])
def test_table_steep_traces(seed):
    """Table path on traces close to the steepest the format loader accepts
    (|dy/dx| up to 0.44 / 0.48, against 0.5): a column's samples change
    deposit row every couple of columns, an item spans tens of bands, the
    windows of neighbouring columns start on different rows, and a segment
    can reach past the rows a tile carries into the next (it is then taken
    up again there).  Against the oracle, with a Doppler shift."""
    sc = scene("mini_table", seed=seed, b_total=70.0)
    rq = Request(rv_mps=-4.0, flux_scale=1.7)
    print(f"case mini_table steep seed={seed}", flush=True)
    g = _gu().render(sc, rq)
    o = oracle.render(sc, rq)
    assert _report(f"mini_table steep {seed}", g, o) < TOL


def test_table_trace_off_detector_edges():
    """A table-path trace that starts left of the detector, leaves through the
    right edge and grazes row 0 (120 x 40 px: three tile columns, the last
    ragged, one tile row plus a ragged one; 2 x 2 field nodes), and the same
    trace moved to graze the last row, against the oracle."""
    from tests.test_oracle_gather import _off_edge_table_scene
    sc = _off_edge_table_scene()
    t = sc.traces[0]
    top = dataclasses.replace(sc, name="off_edge_last_row",
                              traces=[dataclasses.replace(t, cy=[37.6, 1.4, 0.8])])
    rq = Request(rv_mps=3.0, flux_scale=2.0)
    for s_ in (sc, top):
        print(f"case {s_.name}", flush=True)
        g = _gu().render(s_, rq)
        o = oracle.render(s_, rq)
        assert _report(s_.name, g, o) < TOL


def test_mini_sep_frame():
    sc = scene("mini_sep")
    print("case mini_sep FP64 accumulation", flush=True)
    g = _gu().render(sc)
    o = oracle.render(sc)
    assert _report("mini_sep", g, o) < TOL


def test_determinism_bitwise(mini_table):
    print("case determinism", flush=True)
    a = _gu().render(mini_table, Request(rv_mps=3.0))
    b = _gu().render(mini_table, Request(rv_mps=3.0))
    assert np.array_equal(a, b)


def test_batch_equals_single_bitwise():
    gu = _gu()
    from paper_2008_05858_amd import Loaded
    scs = [scene("mini_table"), scene("mini_c3v"), scene("mini_table", seed=77)]
    rqs = [Request(rv_mps=1.0, flux_scale=2.0), Request(rv_mps=-4.0, flux_scale=0.5),
           Request(rv_mps=7.0)]
    lds = [Loaded(gu.ctx(), s) for s in scs]
    print("case batch of 3 uneven frames", flush=True)
    outs = gu.render_batch(scs, rqs, lds)
    for sc, rq, ld, ob in zip(scs, rqs, lds, outs):
        single = gu.render(sc, rq, loaded=ld)
        assert np.array_equal(ob, single)
    o = oracle.render(scs[1], rqs[1])
    assert _report("batch mini_c3v", outs[1], o) < TOL
    for ld in lds:
        ld.free()


@pytest.mark.parametrize("prec", ["f64", "f16_hilo"])
def test_separable_batch_equals_single_bitwise(prec):
    """The separable kernels' persistent (work-list) launch gives the same
    bits as their plain launch, frame by frame, and matches the oracle: the
    VALU kernel (f64) and the MFMA kernel (f16_hilo).  c0's circular PSF has
    no reduced-precision form and renders at f64 in both cases."""
    gu = _gu()
    from paper_2008_05858_amd import Loaded
    scs = [scene("mini_sep"), scene("mini_sep", seed=31), scene("c0")]
    rqs = [Request(rv_mps=2.5, flux_scale=1.5, precision=prec),
           Request(rv_mps=-6.0, precision=prec), Request(rv_mps=0.4)]
    lds = [Loaded(gu.ctx(), s) for s in scs]
    print(f"case separable batch of mini_sep x2 + c0, precision {prec}", flush=True)
    for grp in ((0, 1), (2,)):
        outs = gu.render_batch([scs[i] for i in grp], [rqs[i] for i in grp], [lds[i] for i in grp])
        for i, ob in zip(grp, outs):
            assert np.array_equal(ob, gu.render(scs[i], rqs[i], loaded=lds[i])), i
    o = oracle.render(scs[1], rqs[1])
    g = gu.render(scs[1], rqs[1], loaded=lds[1])
    assert _report("sep batch mini_sep seed 31", g, o) < TOL
    for ld in lds:
        ld.free()


def _line_scene(kind, x0=300.5, n=4001, lines=(1000, 2000, 3000)):
    spec = np.zeros(n)
    for k in lines:
        spec[k] = 1e5
    if kind == "erf":
        psf = Psf(kind="erf", sigma=1.2, half_width=7)
    else:
        u = (np.arange(32) + 0.5) / 4 - 4
        K = np.exp(-0.5 * (u[:, None] ** 2 / 1.3 ** 2 + u[None, :] ** 2 / 1.1 ** 2)).astype(np.float32)
        K /= K.sum()
        psf = Psf(kind="table", gx=1, gy=1, kw=32, kh=32, os=4, tables=K[None, None])
    tr = Trace(0, 0, 0, 600.0, 606.0, n, [x0, 250.0, 4.0, -3.0], [64.3, 3.0, 1.5], 1.0, 0)
    return Scene("lines", 640, 128, [tr], psf, [spec.astype(np.float32)], "f64")


@pytest.mark.parametrize("kind", ["erf", "table"])
def test_isolated_line_photocentres(kind):
    """Photocentre of isolated lines: GPU vs oracle within 1e-6 px (the
    requirement is 1e-5 px), and, for the erf kernel, vs the format position."""
    sc = _line_scene(kind)
    print(f"case photocentre {kind}", flush=True)
    g = _gu().render(sc)
    o = oracle.render(sc)
    t = sc.traces[0]
    for k in (1000, 2000, 3000):
        x, y = oracle.positions(sc, 0, 0.0, k, 1)
        i0, j0 = int(round(x[0])) - 12, int(round(y[0])) - 12
        cg = metrics.centroid(g[j0:j0 + 25, i0:i0 + 25], i0, j0)
        co = metrics.centroid(o[j0:j0 + 25, i0:i0 + 25], i0, j0)
        print(f"  line k={k}: gpu-oracle dx={cg[0]-co[0]:.2e} dy={cg[1]-co[1]:.2e}", flush=True)
        assert abs(cg[0] - co[0]) < 1e-6 and abs(cg[1] - co[1]) < 1e-6
        if kind == "erf":
            assert abs(cg[0] - x[0]) < 1e-5 and abs(cg[1] - y[0]) < 1e-5


def test_doppler_centroid_shift_on_gpu():
    sc = _line_scene("erf", lines=(2000,))
    print("case doppler", flush=True)
    g0 = _gu().render(sc)
    g1 = _gu().render(sc, Request(rv_mps=10.0))
    t = sc.traces[0]
    x0, _ = oracle.positions(sc, 0, 0.0, 2000, 1)
    x1, _ = oracle.positions(sc, 0, 10.0, 2000, 1)
    dc = metrics.centroid(g1)[0] - metrics.centroid(g0)[0]
    assert abs(dc - (x1[0] - x0[0])) < 1e-6


def test_flux_conservation_gpu():
    """The frame holds every photon of samples whose footprint is on chip
    (the superposition of Sec. 2 / Sec. 2.2 loses nothing).  The oracle holds
    this to 1e-12; the GPU path takes the pixel weights in FP32 on
    pixel-relative offsets (FP64 sums), so its bound is 1e-6 relative."""
    sc = scene("c0")
    g = _gu().render(sc, Request(flux_scale=2.0))
    tot = sc.spectra[0].sum() * 2.0
    assert abs(g.sum() - tot) / tot < 1e-6


# bound on max |dF| / peak per precision variant of the separable path: the
# FP64-summing and fp16 hi/lo paths meet the 1e-6 frame requirement; the
# FP32-summing and bf16 hi/lo ones (hi/lo bf16 keeps ~16 mantissa bits) are
# held to about twice what they measure here (2.0e-6 and 1.5e-6)
SEP_BOUNDS = {"f64": 1e-6, "f32": 4e-6, "f16_hilo": 1e-6, "bf16_hilo": 3e-6}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16_hilo", "bf16_hilo"])
def test_separable_precision_variants(prec):
    sc = scene("mini_sep")
    rq = Request(rv_mps=4.0, precision=prec)
    print(f"case mini_sep precision={prec}", flush=True)
    g = _gu().render(sc, rq)
    o = oracle.render(sc, rq)
    err = _report(f"mini_sep-{prec}", g, o)
    # photocentre of the brightest trace window, gpu vs oracle
    j, i = np.unravel_index(np.argmax(o), o.shape)
    j0, i0 = max(j - 8, 0), max(i - 20, 0)
    cg = metrics.centroid(g[j0:j + 9, i0:i + 21], i0, j0)
    co = metrics.centroid(o[j0:j + 9, i0:i + 21], i0, j0)
    print(f"  photocentre shift x {cg[0]-co[0]:.2e} px, y {cg[1]-co[1]:.2e} px", flush=True)
    assert err < SEP_BOUNDS[prec]
    # the paper's photocentre budget (Sec. 1, Sec. 2.2): 1e-5 px
    assert np.isfinite(cg).all() and np.isfinite(co).all()
    assert abs(cg[0] - co[0]) <= 1e-5 and abs(cg[1] - co[1]) <= 1e-5


def _steep_sep_scene():
    """mini_sep's instrument with traces near the steepest accepted slope
    (|dy/dx| up to 0.48)."""
    from workloads.synth import _espresso
    return _espresso(2011, nx=512, ny=452, orders=list(range(78, 82)), n_samp=20000, gx=11,
                     kwid=0, psf_kind="separable", name="mini_sep_steep", xh=262.0, y0=60.0,
                     pitch=100.0, n_lines=600, a_scale=0.06, b_total=70.0)


def _off_edge_sep_scene():
    """A separable-PSF trace entering and leaving through the side edges of a
    120 x 40 px detector and grazing row 0, on a 2 x 2 field grid."""
    rng = np.random.default_rng(12)
    sig = rng.uniform(1.0, 1.6, (2, 2, 2)).astype(np.float32)
    psf = Psf(kind="separable", gx=2, gy=2, half_width=8, sigma_xy=sig)
    n = 3000
    tr = Trace(0, 0, 0, 600.0, 603.0, n, [60.0, 70.0, 3.0, -1.5], [2.2, 1.4, 0.8], 0.7, 0)
    spec = rng.uniform(0.5, 1.5, n) * 1e4
    return Scene("off_edge_sep", 120, 40, [tr], psf, [spec.astype(np.float32)], "f32")


@pytest.mark.parametrize("prec", ["f64", "f32", "f16_hilo", "bf16_hilo"])
def test_separable_steep_and_off_edge(prec):
    """The separable path (VALU at FP64 / FP32, MFMA at fp16 / bf16 hi-lo) on
    steep traces, whose windows cross tile rows along the trace, and on a
    trace running over the detector's edges, against the oracle, each
    precision held to its bound."""
    for sc in (_steep_sep_scene(), _off_edge_sep_scene()):
        rq = Request(rv_mps=-3.0, flux_scale=1.3, precision=prec)
        print(f"case {sc.name} precision={prec}", flush=True)
        g = _gu().render(sc, rq)
        o = oracle.render(sc, rq)
        assert _report(f"{sc.name}-{prec}", g, o) < SEP_BOUNDS[prec]
