"""Photon noise on the GPU (Sec. 2.2): the Philox stream must equal the
oracle's bit for bit; the Poisson counts agree with the oracle's wherever the
two libms agree on the acceptance tests, and follow the Poisson law."""
import ctypes as C

import numpy as np
import pytest
from scipy import stats

import oracle
from workloads import Request, scene

pytestmark = pytest.mark.gpu


def _gu():
    from tests import gpu_util
    return gpu_util


def test_philox_stream_bitwise():
    from paper_2008_05858_amd import e2e as E
    c = _gu().ctx()
    for seed, frame, p0 in [(0, 0, 0), (0xDEADBEEF12345678, 7, 123456789), (42, 3, (1 << 33) + 5)]:
        g = np.frombuffer(E.e2e_philox_blocks(c, seed, frame, p0, 64, 3), dtype=np.uint32)
        o = np.concatenate([oracle.philox_blocks(seed, frame, p0 + p, 3) for p in range(64)])
        assert np.array_equal(g, o)


def test_poisson_counts_match_oracle_and_law():
    import torch
    from paper_2008_05858_amd import e2e as E
    c = _gu().ctx()
    means = np.repeat([0.0, 0.3, 5.0, 9.99, 10.0, 50.0, 1e4, 1e7], 20000).astype(np.float64)
    t = torch.from_numpy(means.copy()).to("cuda")
    torch.cuda.synchronize()
    E.e2e_noise_poisson(c, t.data_ptr(), E.E2E_F64, means.size, 99, 4, 1)
    g = t.cpu().numpy()
    o = oracle.poisson_frame(means, 99, 4)
    same = np.mean(g == o)
    print(f"identical counts: {same:.6f}", flush=True)
    assert same == 1.0
    for lam in (0.3, 5.0, 9.99, 10.0, 50.0, 1e4, 1e7):
        d = g[means == lam]
        assert abs(d.mean() - lam) < 5 * np.sqrt(lam / d.size)
        assert abs(d.var() / lam - 1) < 0.05
    assert np.all(g[means == 0.0] == 0)


def test_render_with_noise_equals_noise_on_render():
    import torch
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    sc = scene("mini_table")
    a = gu.render(sc, Request(rv_mps=1.0, seed=77, frame_index=5, poisson=True))
    b = gu.render(sc, Request(rv_mps=1.0))
    t = torch.from_numpy(b.copy()).to("cuda")
    torch.cuda.synchronize()
    E.e2e_noise_poisson(gu.ctx(), t.data_ptr(), E.E2E_F32, b.size, 77, 5, 1)
    assert np.array_equal(a, t.cpu().numpy())
    # a different frame index draws a different realisation
    c = gu.render(sc, Request(rv_mps=1.0, seed=77, frame_index=6, poisson=True))
    assert not np.array_equal(a, c)
