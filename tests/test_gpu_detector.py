"""Detector stage on the GPU (Sec. 2.2: PRNU, dark current, shot noise,
inter-pixel cross-talk, read-out noise, ADC) through the C ABI, against the
FP64 oracle.  Without random draws the stage is fma / divide / floor only
and must match bit for bit; with draws, ADU agree wherever the two libms
agree on the Poisson acceptance tests and on log / cos of the read-noise
pair (a last-bit difference moves an ADU only when R / gain + bias sits on
a rounding boundary)."""
import numpy as np
import pytest

import oracle
from workloads import XTALK_CCD, detector_frame, prnu_map

pytestmark = pytest.mark.gpu


def _gpu_detector(F, G, desc_kw, on_device=True):
    import torch
    from paper_2008_05858_amd import e2e as E
    from tests import gpu_util
    ny, nx = F.shape
    d = E.e2e_detector_desc()
    K = np.asarray(desc_kw.get("xtalk", np.eye(1, 9, 4)), np.float64).reshape(9)
    for q in range(9):
        d.xtalk[q] = float(K[q])
    d.exposure_s = desc_kw.get("exposure_s", 1.0)
    d.dark_e_per_s = desc_kw.get("dark_e_per_s", 0.0)
    d.ron_e = desc_kw.get("ron_e", 0.0)
    d.gain_e_per_adu = desc_kw.get("gain", 1.0)
    d.bias_adu = desc_kw.get("bias", 0.0)
    d.seed = desc_kw.get("seed", 0)
    d.frame_index = desc_kw.get("frame", 0)
    d.shot_noise = 1 if desc_kw.get("shot_noise", True) else 0
    d.bits = desc_kw.get("bits", 16)
    dt = E.E2E_F64 if F.dtype == np.float64 else E.E2E_F32
    if on_device:
        tf = torch.from_numpy(F).to("cuda")
        tg = torch.from_numpy(G).to("cuda") if G is not None else None
        to = torch.zeros((ny, nx), dtype=torch.int16, device="cuda")
        torch.cuda.synchronize()
        E.e2e_detector(gpu_util.ctx(), d, tf.data_ptr(), dt,
                       tg.data_ptr() if tg is not None else None, nx, ny, to.data_ptr(), 1)
        return to.cpu().numpy().view(np.uint16)
    out = np.zeros((ny, nx), np.uint16)
    E.e2e_detector(gpu_util.ctx(), d, F.ctypes.data, dt,
                   G.ctypes.data if G is not None else None, nx, ny, out.ctypes.data, 0)
    return out


def _oracle(F, G, kw, window=None):
    return oracle.detector(F.astype(np.float64), prnu=None if G is None else G.astype(np.float64),
                           exposure_s=kw.get("exposure_s", 1.0),
                           dark_e_per_s=kw.get("dark_e_per_s", 0.0),
                           shot_noise=kw.get("shot_noise", True), xtalk=kw.get("xtalk"),
                           ron_e=kw.get("ron_e", 0.0), gain=kw.get("gain", 1.0),
                           bias=kw.get("bias", 0.0), bits=kw.get("bits", 16),
                           seed=kw.get("seed", 0), frame=kw.get("frame", 0), window=window)


NOISE_FREE = dict(exposure_s=900.0, dark_e_per_s=0.011, shot_noise=False, xtalk=XTALK_CCD,
                  ron_e=0.0, gain=1.37, bias=1000.0, bits=16)


@pytest.mark.parametrize("nx,ny,dtype", [(131, 77, np.float64), (64, 48, np.float32),
                                         (1, 1, np.float64), (17, 1, np.float32),
                                         (1, 33, np.float64)])
def test_noise_free_bitwise(nx, ny, dtype):
    print(f"case detector noise-free {nx}x{ny} {np.dtype(dtype).name}", flush=True)
    F = detector_frame(nx, ny, 11, peak=9e4, dtype=dtype)
    G = prnu_map(nx, ny, 11)
    g = _gpu_detector(F, G, NOISE_FREE)
    o = _oracle(F, G, NOISE_FREE)
    assert np.array_equal(g, o), np.argwhere(g != o)[:5]


def test_clipping_and_bits():
    print("case detector clipping", flush=True)
    F = np.array([[0.0, 1.0, 4094.4, 4094.6, 5e4, 1e9]], np.float64)
    for bits, bias in ((12, 0.0), (16, -3.0), (1, 0.0)):
        kw = dict(shot_noise=False, bits=bits, bias=bias, gain=1.0)
        g = _gpu_detector(F, None, kw)
        o = _oracle(F, None, kw)
        assert np.array_equal(g, o)
        assert g.max() <= (1 << bits) - 1 and g[0, -1] == (1 << bits) - 1
    g = _gpu_detector(F, None, dict(shot_noise=False, bits=12))
    assert list(g[0]) == [0, 1, 4094, 4095, 4095, 4095]


def test_with_noise_matches_oracle():
    print("case detector shot + read noise 300x200", flush=True)
    F = detector_frame(300, 200, 5, peak=2e5)
    G = prnu_map(300, 200, 5)
    kw = dict(NOISE_FREE, shot_noise=True, ron_e=3.2, seed=0xC0FFEE, frame=9)
    g = _gpu_detector(F, G, kw)
    o = _oracle(F, G, kw)
    same = np.mean(g == o)
    print(f"identical ADU: {same:.6f}", flush=True)
    assert same == 1.0
    # the host-pointer path stages the same computation
    h = _gpu_detector(F, G, kw, on_device=False)
    assert np.array_equal(g, h)
    # a different frame index draws a different realisation
    g2 = _gpu_detector(F, G, dict(kw, frame=10))
    assert np.mean(g2 != g) > 0.5


def test_read_noise_law():
    """Flat frame, no shot noise, no cross-talk: ADU - bias is N(mu, ron)
    rounded, so its mean is mu and its variance ron^2 + 1/12."""
    print("case detector read-noise law", flush=True)
    mu, ron = 250.0, 4.0
    F = np.full((512, 512), mu, np.float64)
    g = _gpu_detector(F, None, dict(shot_noise=False, ron_e=ron, bias=100.0, seed=3))
    v = g.astype(np.float64) - 100.0
    n = v.size
    assert abs(v.mean() - mu) < 5 * ron / np.sqrt(n)
    assert abs(v.var() / (ron * ron + 1.0 / 12.0) - 1.0) < 0.02


def test_errors():
    from paper_2008_05858_amd import e2e as E
    F = np.ones((4, 4), np.float64)
    for bad in (dict(bits=0), dict(bits=17), dict(gain=0.0), dict(gain=-1.0),
                dict(ron_e=-1.0), dict(exposure_s=float("nan")),
                dict(xtalk=[0, 0, 0, 0, float("inf"), 0, 0, 0, 0])):
        with pytest.raises(E.E2EError) as ei:
            _gpu_detector(F, None, bad, on_device=False)
        assert ei.value.code == E.E2E_EINVAL
    # an empty frame is a no-op
    assert _gpu_detector(np.ones((0, 5), np.float64), None, {}, on_device=False).size == 0


def test_c1_full_frame_sampled_windows():
    """9216 x 9216 FP32 frame (the size of the ESPRESSO-like frames) with the
    launch shapes used for timing; the oracle evaluates sampled windows (the
    corners, edges and interior) on its own."""
    import torch
    print("case detector c1 full frame 9216x9216", flush=True)
    nx = ny = 9216
    F = detector_frame(nx, ny, 1001)
    G = prnu_map(nx, ny, 1001)
    kw = dict(NOISE_FREE, shot_noise=True, ron_e=3.0, seed=12345, frame=2)
    g = _gpu_detector(F, G, kw)
    del G
    torch.cuda.empty_cache()
    F64 = F.astype(np.float64)
    G64 = prnu_map(nx, ny, 1001).astype(np.float64)
    rng = np.random.default_rng(7)
    wins = [(0, 0, 40, 40), (nx - 40, ny - 40, 40, 40), (0, ny - 40, 40, 40),
            (nx - 40, 0, 40, 40), (4600, 0, 64, 8), (0, 4600, 8, 64)]
    wins += [(int(rng.integers(0, nx - 48)), int(rng.integers(0, ny - 48)), 48, 48)
             for _ in range(6)]
    tot = same = 0
    for (x0, y0, w, h) in wins:
        o = oracle.detector(F64, prnu=G64, exposure_s=kw["exposure_s"],
                            dark_e_per_s=kw["dark_e_per_s"], shot_noise=True,
                            xtalk=kw["xtalk"], ron_e=kw["ron_e"], gain=kw["gain"],
                            bias=kw["bias"], bits=16, seed=kw["seed"], frame=kw["frame"],
                            window=(x0, y0, w, h))
        s = g[y0:y0 + h, x0:x0 + w]
        same += int(np.sum(s == o))
        tot += o.size
    print(f"[c1 detector] {tot} sampled px, identical ADU {same / tot:.6f}", flush=True)
    assert same / tot == 1.0
