"""Parity at the benchmark's full sizes, on sampled pixels the oracle
evaluates one by one (its per-pixel gather form), plus flux sums.

The ESPRESSO-shaped frame is rendered exactly as bench.py times it: a
persistent batch launch of several frames with their own Doppler shifts and
exposure scales.
"""
import numpy as np
import pytest

import oracle
from workloads import Request, scene

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _gu():
    from tests import gpu_util
    return gpu_util


def _sample_pixels(frame, n_bright, n_rand, seed):
    rng = np.random.default_rng(seed)
    thr = 0.05 * frame.max()
    jj, ii = np.nonzero(frame > thr)
    pick = rng.choice(len(jj), size=min(n_bright, len(jj)), replace=False)
    rj = rng.integers(0, frame.shape[0], n_rand)
    ri = rng.integers(0, frame.shape[1], n_rand)
    return np.concatenate([ii[pick], ri]), np.concatenate([jj[pick], rj])


def _check(name, sc, rq, g, n_bright=160, n_rand=40, seed=0):
    px, py = _sample_pixels(g, n_bright, n_rand, seed)
    o = oracle.render_pixels(sc, rq, px, py)
    peak = float(g.max())
    err = np.max(np.abs(g[py, px] - o)) / peak
    print(f"[{name}] {len(px)} sampled px: max|dF|/peak = {err:.3e} (peak {peak:.4g})", flush=True)
    return err


def test_c1_batch_sampled():
    from paper_2008_05858_amd import Loaded
    gu = _gu()
    sc = scene("c1")
    ld = Loaded(gu.ctx(), sc)
    rqs = [Request(rv_mps=-7.5, flux_scale=3.1), Request(rv_mps=9.0, flux_scale=0.4)]
    print("case c1 full frame x2, persistent batch", flush=True)
    outs = gu.render_batch([sc, sc], rqs, [ld, ld])
    for b, (g, rq) in enumerate(zip(outs, rqs)):
        assert _check(f"c1 frame {b}", sc, rq, g, seed=b) < TOL
    # flux: every trace lies on the detector with its whole footprint
    tot = sum(float(sc.spectra[t.slot].astype(np.float64).sum()) * t.thr for t in sc.traces)
    rel = abs(outs[0].astype(np.float64).sum() - tot * rqs[0].flux_scale) / (tot * rqs[0].flux_scale)
    print(f"  flux sum rel error {rel:.2e}", flush=True)
    assert rel < 1e-6
    ld.free()


def test_c3_uneven_batch_sampled():
    from paper_2008_05858_amd import Loaded
    gu = _gu()
    a, b = scene("c1"), scene("c3v")
    la, lb = Loaded(gu.ctx(), a), Loaded(gu.ctx(), b)
    rqs = [Request(rv_mps=3.3, flux_scale=9.0), Request(rv_mps=-4.4, flux_scale=0.2),
           Request(rv_mps=0.7, flux_scale=5.0)]
    print("case c3: c1 + 2 x 4096^2 variant frames in one launch", flush=True)
    outs = gu.render_batch([b, a, b], rqs, [lb, la, lb])
    assert _check("c3 variant 0", b, rqs[0], outs[0], n_bright=80, n_rand=20, seed=3) < TOL
    assert _check("c3 c1", a, rqs[1], outs[1], n_bright=80, n_rand=20, seed=4) < TOL
    assert _check("c3 variant 1", b, rqs[2], outs[2], n_bright=80, n_rand=20, seed=5) < TOL
    la.free()
    lb.free()


SEP_BOUNDS = {"f64": 1e-6, "f32": 2e-5, "f16_hilo": 2e-6, "bf16_hilo": 2e-4}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16_hilo", "bf16_hilo"])
def test_c2_precision_variants_sampled(prec):
    sc = scene("c2")
    rq = Request(rv_mps=2.0, precision=prec)
    print(f"case c2 full frame, precision {prec}", flush=True)
    g = _gu().render(sc, rq)
    assert _check(f"c2 {prec}", sc, rq, g, n_bright=120, n_rand=30, seed=7) < SEP_BOUNDS[prec]


def test_c4_hires_sampled():
    sc = scene("c4")
    rq = Request(rv_mps=-1.0)
    print("case c4 HIRES-shaped full frame", flush=True)
    g = _gu().render(sc, rq)
    assert _check("c4", sc, rq, g, n_bright=12, n_rand=4, seed=9) < TOL


def test_separable_one_and_two_pixel_kernels_agree_bitwise():
    """Small launches of the separable kernel run one pixel per thread, large
    ones two; both add each pixel's products in the same groups of four
    samples, so a frame gets the same bits from either."""
    from paper_2008_05858_amd import Loaded
    gu = _gu()
    small, big = scene("mini_sep"), scene("c2")
    ls, lb = Loaded(gu.ctx(), small), Loaded(gu.ctx(), big)
    rq = Request(rv_mps=1.25)
    print("case mini_sep alone (one pixel per thread) vs batched with c2 (two)", flush=True)
    alone = gu.render(small, rq, loaded=ls)
    outs = gu.render_batch([small, big], [rq, Request(rv_mps=2.0)], [ls, lb])
    assert np.array_equal(alone, outs[0])
    ls.free()
    lb.free()
