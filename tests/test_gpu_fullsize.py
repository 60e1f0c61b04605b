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
        err, n = _strat_check(f"c1 frame {b}", sc, rq, g, n_each=35, seed=b)
        assert n >= 200 and err < TOL
    # flux: every trace lies on the detector with its whole footprint
    tot = sum(float(sc.spectra[t.slot].astype(np.float64).sum()) * t.thr for t in sc.traces)
    rel = abs(outs[0].astype(np.float64).sum() - tot * rqs[0].flux_scale) / (tot * rqs[0].flux_scale)
    print(f"  flux sum rel error {rel:.2e}", flush=True)
    assert rel < 1e-6
    ld.free()


def test_dense_sampling_table():
    """Densely sampled traces: 2e7 samples per trace over ~480 px, about 1e4
    per quarter-pixel slot column, where the table path's first guess of a
    column's first sample (an inverse quadratic over the tile's segment) can be
    hundreds of samples off.  The render must find every column's samples
    exactly (no device error) and match the oracle; 16 sampled pixels keep the
    oracle's per-pixel gather (about 1 s per pixel here) short."""
    gu = _gu()
    sc = scene("mini_table", n_samp=20_000_000)
    rq = Request(rv_mps=39.0)
    print("case mini_table with 2e7 samples per trace", flush=True)
    g = gu.render(sc, rq)
    err = _check("mini_table dense", sc, rq, g, n_bright=12, n_rand=4, seed=3)
    assert err < TOL


def _strat_check(name, sc, rq, g, tw=56, th=32, n_each=25, seed=0):
    """Parity at stratified pixels: tile-boundary and carry rows, tile-column
    edges, node-cell boundary lines, bright pixels, trace ends, anywhere."""
    from workloads import metrics
    gx, gy = int(sc.psf.gx), int(sc.psf.gy)
    nxl = [m * (sc.nx - 1) / (gx - 1) for m in range(gx)] if gx > 1 else []
    nyl = [m * (sc.ny - 1) / (gy - 1) for m in range(gy)] if gy > 1 else []
    px, py = metrics.stratified_pixels(g, tw, th, node_x=nxl, node_y=nyl, n_each=n_each,
                                       seed=seed)
    o = oracle.render_pixels(sc, rq, px, py)
    peak = float(g.max())
    err = float(np.max(np.abs(g[py, px] - o)) / peak)
    print(f"[{name}] {len(px)} stratified px: max|dF|/peak = {err:.3e} (peak {peak:.4g})",
          flush=True)
    return err, len(px)


def test_c3_configured_batch():
    """The batched configuration as configured: 64 renders of uneven size in
    one persistent launch (captured graph), 32 ESPRESSO-shaped 9216^2 frames
    and 32 of the 4096^2 40-order 1-fiber variant in a seeded order, each with
    its own Doppler shift (U[-10, 10] m/s) and exposure (U[1e3, 1e5]),
    Poisson noise on every other frame.  Checked: stratified oracle parity on
    four noiseless frames, bitwise equality with single renders on four
    frames, and the noisy frames equal to e2e_noise_poisson applied to the
    noiseless single render (same seed and frame index)."""
    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    ctx = gu.ctx()
    a, b = scene("c1"), scene("c3v")
    la, lb = P.Loaded(ctx, a), P.Loaded(ctx, b)
    spa, sdt = gu.device_spectra(a)
    spb, _ = gu.device_spectra(b)
    rng = np.random.Generator(np.random.PCG64(1003))
    kinds = rng.permutation(np.array([0] * 32 + [1] * 32))
    outs, rr, keep, meta = [], [], [], []
    for f, kd in enumerate(kinds):
        sc, ld, sp = (a, la, spa) if kd == 0 else (b, lb, spb)
        rq = Request(rv_mps=float(rng.uniform(-10, 10)),
                     flux_scale=float(rng.uniform(1e3, 1e5) / 1e4), seed=99, frame_index=f,
                     poisson=bool(f % 2))
        o, odt = gu.out_tensor(sc)
        r, k = gu.request_for(ld, sc, sp, sdt, o, odt, rq)
        outs.append(o)
        rr.append(r)
        keep.append(k)
        meta.append((sc, ld, rq))
    torch.cuda.synchronize()
    print("case c3: 64 uneven frames, one persistent launch", flush=True)
    E.e2e_render_batch(ctx, rr)
    E.e2e_render_batch(ctx, rr)  # a replay of the captured graph gives the same frames
    quiet = [f for f in range(64) if f % 2 == 0]
    noisy = [f for f in range(64) if f % 2 == 1]
    pick_q = [next(f for f in quiet if kinds[f] == 0), next(f for f in quiet if kinds[f] == 1),
              [f for f in quiet if kinds[f] == 0][-1], [f for f in quiet if kinds[f] == 1][-1]]
    for f in pick_q:
        sc, ld, rq = meta[f]
        g = outs[f].cpu().numpy()
        err, n = _strat_check(f"c3 frame {f} ({'c1' if kinds[f] == 0 else 'variant'})", sc, rq,
                              g, seed=f)
        assert n >= 150 and err < TOL
        # bitwise: the same request rendered alone
        assert np.array_equal(g, gu.render(sc, rq, loaded=ld)), f
    pick_n = [next(f for f in noisy if kinds[f] == 0), next(f for f in noisy if kinds[f] == 1),
              [f for f in noisy if kinds[f] == 0][-1], [f for f in noisy if kinds[f] == 1][-1]]
    for f in pick_n:
        sc, ld, rq = meta[f]
        quiet_rq = Request(rv_mps=rq.rv_mps, flux_scale=rq.flux_scale)
        o, odt = gu.out_tensor(sc)
        r, k = gu.request_for(ld, sc, spa if kinds[f] == 0 else spb, sdt, o, odt, quiet_rq)
        E.e2e_render(ctx, r)
        E.e2e_noise_poisson(ctx, o.data_ptr(), odt, sc.nx * sc.ny, rq.seed, f, 1, None)
        same = np.array_equal(outs[f].cpu().numpy(), o.cpu().numpy())
        print(f"  c3 noisy frame {f}: equal to render + e2e_noise_poisson: {same}", flush=True)
        assert same
    la.free()
    lb.free()


# bound on max |dF| / peak per precision variant of the separable path at
# full size: the FP64-summing and fp16 hi/lo paths hold the 1e-6 frame bar;
# the FP32-summing and bf16 hi/lo ones are held to about twice what they
# measure (1.1e-6 and 1.4e-6 of the peak)
SEP_BOUNDS = {"f64": 1e-6, "f32": 2.5e-6, "f16_hilo": 1e-6, "bf16_hilo": 3e-6}


@pytest.mark.parametrize("prec", ["f64", "f32", "f16_hilo", "bf16_hilo"])
def test_c2_precision_variants_sampled(prec):
    sc = scene("c2")
    rq = Request(rv_mps=2.0, precision=prec)
    print(f"case c2 full frame, precision {prec}", flush=True)
    g = _gu().render(sc, rq)
    mfma = prec in ("f16_hilo", "bf16_hilo")
    err, n = _strat_check(f"c2 {prec}", sc, rq, g, tw=64 if mfma else 16, th=32 if mfma else 16,
                          seed=7)
    assert n >= 150 and err < SEP_BOUNDS[prec]


def test_c4_hires_sampled():
    sc = scene("c4")
    rq = Request(rv_mps=-1.0)
    print("case c4 HIRES-shaped full frame", flush=True)
    g = _gu().render(sc, rq)
    err, n = _strat_check("c4", sc, rq, g, tw=52, th=32, n_each=35, seed=9)
    assert n >= 200 and err < TOL


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
