"""GPU tests of the launch autotuner (batch/serve orchestration, Sec. 3 sized
to one GPU): it times every candidate, keeps the fastest for the workload
shape, and renders made with the kept choice still match the oracle and are
deterministic; batch and single renders share the choice."""
import numpy as np
import pytest

import oracle
from workloads import Request, scene

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _gu():
    from tests import gpu_util
    return gpu_util


def test_autotune_single_then_render_matches_oracle():
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    ctx = E.e2e_create(0, 0)
    sc = scene("mini_table")
    ld = P.Loaded(ctx, sc)
    specs, sdt = gu.device_spectra(sc)
    out, odt = gu.out_tensor(sc)
    rq = Request(rv_mps=2.5)
    r, k = gu.request_for(ld, sc, specs, sdt, out, odt, rq)
    print("case autotune mini_table n=1", flush=True)
    rep = E.e2e_autotune(ctx, [r])
    cands = [(rep.cand_chunk[i], rep.cand_resident[i], rep.cand_ms[i])
             for i in range(rep.n_candidates)]
    print("candidates", cands, "kept", rep.chunk, rep.resident, flush=True)
    assert rep.n_candidates == 4
    assert sorted(c for c, _, _ in cands) == [2, 4, 8, 16]
    assert rep.chunk in (2, 4, 8, 16)
    assert rep.ms == pytest.approx(min(ms for _, _, ms in cands))
    a = gu.render(sc, rq, loaded=ld, context=ctx)
    b = gu.render(sc, rq, loaded=ld, context=ctx)
    assert np.array_equal(a, b)
    o = oracle.render(sc, rq)
    err = np.max(np.abs(a - o)) / o.max()
    print(f"tuned render max|dF|/peak = {err:.3e}", flush=True)
    assert err < TOL
    ld.free()
    E.e2e_destroy(ctx)


def test_autotune_batch_keeps_batch_equal_to_single():
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    ctx = E.e2e_create(0, 0)
    scs = [scene("mini_table"), scene("mini_c3v")]
    lds = [P.Loaded(ctx, s) for s in scs]
    rqs = [Request(rv_mps=-1.0, flux_scale=2.0), Request(rv_mps=4.0)]
    keep, reqs = [], []
    for sc, ld, rq in zip(scs, lds, rqs):
        specs, sdt = gu.device_spectra(sc)
        out, odt = gu.out_tensor(sc)
        r, k = gu.request_for(ld, sc, specs, sdt, out, odt, rq)
        keep.append((specs, out, k))
        reqs.append(r)
    print("case autotune batch of 2", flush=True)
    rep = E.e2e_autotune(ctx, reqs)
    print("kept", rep.chunk, rep.resident, "of", rep.n_candidates, flush=True)
    assert rep.n_candidates == 12
    assert rep.resident in (1, 2, 3)
    outs = gu.render_batch(scs, rqs, lds, context=ctx)
    for sc, rq, ld, ob in zip(scs, rqs, lds, outs):
        assert np.array_equal(ob, gu.render(sc, rq, loaded=ld, context=ctx))
    for ld in lds:
        ld.free()
    E.e2e_destroy(ctx)
