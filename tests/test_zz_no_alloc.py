"""GPU: the allocation-free render (e2e_render_noalloc) equals e2e_render.

Two calls in a row on one context, the second with a smaller frame and a
different PSF path, each compared bit for bit with e2e_render of the same
request and with the FP64 oracle at the per-pixel bar; then the limits: a
planner output beyond the fixed device array is refused with E2E_ENOMEM and
host buffers with E2E_EINVAL, before anything is launched.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from workloads import Request, metrics, scene

pytestmark = pytest.mark.gpu


def _gu():
    from tests import gpu_util
    return gpu_util


def _noalloc(gu, sc, rq):
    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    ld = P.Loaded(gu.ctx(), sc)
    specs, sdt = gu.device_spectra(sc)
    out, odt = gu.out_tensor(sc)
    r, keep = gu.request_for(ld, sc, specs, sdt, out, odt, rq)
    torch.cuda.synchronize()
    E.e2e_render_noalloc(gu.ctx(), r)
    res = out.cpu().numpy()
    ref = gu.render(sc, rq, loaded=ld)
    ld.free()
    return res, ref


@pytest.mark.parametrize("first,second", [("mini_hires", "c0")])
def test_noalloc_equals_render_twice(first, second):
    gu = _gu()
    for name, rq in ((first, Request(rv_mps=3.0, flux_scale=1.7)),
                     (second, Request(rv_mps=-2.0, flux_scale=0.6))):
        sc = scene(name)
        print(f"case noalloc {name} {sc.nx}x{sc.ny}", flush=True)
        got, ref = _noalloc(gu, sc, rq)
        assert np.array_equal(got, ref), f"{name}: noalloc differs from e2e_render"
        err = metrics.max_rel_err(got, oracle.render(sc, rq))
        print(f"  bitwise equal to e2e_render; max|dF|/peak vs oracle = {err:.3e}")
        assert err < 1e-6


def test_noalloc_limits():
    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    sc = scene("mini_table")
    # planner output 16 B per (tile column, trace): 9216 px wide x 7000 traces
    # needs ~18 MiB, beyond the 16 MiB array
    t = sc.traces[0]
    big = dataclasses.replace(sc, nx=9216, traces=[t] * 7000)
    print("case noalloc limits", flush=True)
    ld = P.Loaded(gu.ctx(), big)
    specs, sdt = gu.device_spectra(big)
    out = torch.zeros(1, dtype=torch.float32, device="cuda")
    r, keep = gu.request_for(ld, big, specs, sdt, out, E.E2E_F32)
    with pytest.raises(E.E2EError) as ei:
        E.e2e_render_noalloc(gu.ctx(), r)
    assert ei.value.code == E.E2E_ENOMEM
    assert "limit" in str(ei.value)
    ld.free()
    # host output is refused
    ld = P.Loaded(gu.ctx(), sc)
    specs, sdt = gu.device_spectra(sc)
    host = np.zeros((sc.ny, sc.nx), np.float32)
    r, keep = P.make_req(ld, [s.data_ptr() for s in specs], sdt, host.ctypes.data, E.E2E_F32,
                         spectra_on_device=True, out_on_device=False)
    with pytest.raises(E.E2EError) as ei:
        E.e2e_render_noalloc(gu.ctx(), r)
    assert ei.value.code == E.E2E_EINVAL
    ld.free()
