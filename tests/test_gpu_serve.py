"""GPU tests of batching (graph replays) and the continuous-batching serve loop.

A frame depends only on its own request, so it must be bitwise identical when
rendered alone, inside a batch launch, or inside a served mix.
"""
import threading

import numpy as np
import pytest

from workloads import Request, scene

pytestmark = pytest.mark.gpu


def _gu():
    from tests import gpu_util
    return gpu_util


def test_batch_graph_replays_match_eager():
    """Several replays of the captured batch graph, with eager work and
    synchronisation between them, each equal to single-frame renders."""
    import torch
    gu = _gu()
    from paper_2008_05858_amd import Loaded
    scs = [scene("mini_table"), scene("mini_c3v")]
    lds = [Loaded(gu.ctx(), s) for s in scs]
    for rep in range(3):
        rqs = [Request(rv_mps=1.5 * rep - 2.0, flux_scale=1.0 + rep),
               Request(rv_mps=-3.0 * rep, flux_scale=0.5)]
        print(f"case batch replay {rep}", flush=True)
        outs = gu.render_batch(scs, rqs, lds)
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work
        for sc, rq, ld, ob in zip(scs, rqs, lds, outs):
            assert np.array_equal(ob, gu.render(sc, rq, loaded=ld)), rep
    for ld in lds:
        ld.free()


def test_serve_mix_equals_alone():
    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    ctx = E.e2e_create(0, 0)
    scs = {"t": scene("mini_table"), "c0": scene("c0"), "h": scene("mini_hires"),
           "s": scene("mini_sfi")}
    lds = {k: P.Loaded(ctx, v) for k, v in scs.items()}
    dev = {k: gu.device_spectra(v) for k, v in scs.items()}
    rng = np.random.default_rng(5)
    plan = [(["t", "c0", "h", "s"][i % 4], float(rng.uniform(-10, 10)),
             float(rng.uniform(0.5, 2))) for i in range(20)]
    # references: alone, plain renderer
    refs = []
    for name, rv, fs in plan:
        refs.append(gu.render(scs[name], Request(rv_mps=rv, flux_scale=fs), loaded=lds[name],
                              context=ctx))
    E.e2e_serve_start(ctx, max_inflight=6, max_queue=64, n_streams=3, max_batch=4)
    outs = [None] * len(plan)
    tickets = [None] * len(plan)
    keep = []

    def submit(idx):
        name, rv, fs = plan[idx]
        sc = scs[name]
        specs, sdt = dev[name]
        out, odt = gu.out_tensor(sc)
        r, k = gu.request_for(lds[name], sc, specs, sdt, out, odt, Request(rv_mps=rv, flux_scale=fs))
        keep.append((r, k, out))
        outs[idx] = out
        tickets[idx] = E.e2e_serve_submit(ctx, r)

    torch.cuda.synchronize()
    print("case serve: 20 requests (table, erf, HIRES tables, explicit SFI) from 3 threads", flush=True)
    ths = [threading.Thread(target=lambda s=s: [submit(i) for i in range(s, len(plan), 3)])
           for s in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    stats = []
    for t in tickets:
        code, st = E.e2e_serve_poll(ctx, t, 60000)
        assert code == E.E2E_OK
        stats.append(st)
    for i, (o, ref) in enumerate(zip(outs, refs)):
        assert np.array_equal(o.cpu().numpy(), ref), i
    for st in stats:
        assert st.t_submit_us <= st.t_admit_us <= st.t_launch_us <= st.t_done_us
        assert st.batch_size >= 1 and st.footprint_bytes > 0
    print("batch sizes", [s.batch_size for s in stats], flush=True)
    # errors stay with their request and poisoned nothing
    with pytest.raises(P.E2EError) as ei:
        E.e2e_serve_poll(ctx, 999999, 0)
    assert ei.value.code == E.E2E_ENOTFOUND
    bad, _k = gu.request_for(lds["t"], scs["t"], *dev["t"], *gu.out_tensor(scs["t"]), None)
    bad.fmt = 424242
    with pytest.raises(P.E2EError) as ei:
        E.e2e_serve_submit(ctx, bad)
    assert ei.value.code == E.E2E_ENOTFOUND
    E.e2e_serve_stop(ctx)
    for ld in lds.values():
        ld.free()
    E.e2e_destroy(ctx)


def test_serve_admission_by_footprint():
    """With HBM for one frame at a time, a stream of requests completes one
    launch after another; a request that can never fit is refused at submit."""
    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    sc = scene("mini_table")
    ntx = -(-sc.nx // 56)
    # resident tables: per node the fp16 hi/lo tap fragments, [2][4 phases]
    # [dd + 2 rows][padded slot offsets][4 band rows]; per trace its record
    dd = (sc.psf.kw + 2) // 4 + 1
    sp = (sc.psf.kw + 3 + 7) // 8 * 8
    tables = sc.psf.gx * sc.psf.gy * 2 * 4 * (dd + 2) * sp * 4 * 2 + len(sc.traces) * 176
    footprint = sc.nx * sc.ny * 4 + ntx * len(sc.traces) * 16
    ctx = E.e2e_create(0, tables + int(1.5 * footprint))
    ld = P.Loaded(ctx, sc)
    specs, sdt = gu.device_spectra(sc)
    outs, tk, keep = [], [], []
    torch.cuda.synchronize()
    print("case serve admission: one frame of HBM", flush=True)
    for i in range(6):
        out, odt = gu.out_tensor(sc)
        r, k = gu.request_for(ld, sc, specs, sdt, out, odt, Request(rv_mps=float(i)))
        keep.append((r, k))
        outs.append(out)
        tk.append(E.e2e_serve_submit(ctx, r))
    for t in tk:
        code, st = E.e2e_serve_poll(ctx, t, 60000)
        assert code == E.E2E_OK
        assert st.batch_size == 1
    ref = gu.render(sc, Request(rv_mps=5.0))
    assert np.array_equal(outs[5].cpu().numpy(), ref)
    E.e2e_serve_stop(ctx)
    ld.free()
    E.e2e_destroy(ctx)

    ctx = E.e2e_create(0, tables + footprint // 2)
    ld = P.Loaded(ctx, sc)
    out, odt = gu.out_tensor(sc)
    r, k = gu.request_for(ld, sc, specs, sdt, out, odt, Request())
    with pytest.raises(P.E2EError) as ei:
        E.e2e_serve_submit(ctx, r)
    assert ei.value.code == E.E2E_ENOMEM
    with pytest.raises(P.E2EError) as ei:
        E.e2e_format_free(ctx, 99999)
    assert ei.value.code == E.E2E_ENOTFOUND
    E.e2e_serve_stop(ctx)
    ld.free()
    E.e2e_destroy(ctx)


def test_serve_overlap_on_device():
    """Two requests on two streams of the serve loop: the second is launched,
    and starts on the device, before the first has finished; each frame is
    bitwise the one the plain renderer makes alone."""
    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    gu = _gu()
    ctx = E.e2e_create(0, 0)
    sc = scene("mini_table", n_samp=20_000_000)  # 3.2e8 samples: over a millisecond each
    ld = P.Loaded(ctx, sc)
    specs, sdt = gu.device_spectra(sc)
    rqs = [Request(rv_mps=4.0, flux_scale=1.3), Request(rv_mps=-7.0, flux_scale=0.8)]
    refs = [gu.render(sc, rq, loaded=ld, context=ctx) for rq in rqs]
    outs, keep = [], []
    for rq in rqs:
        o, odt = gu.out_tensor(sc)
        r, k = gu.request_for(ld, sc, specs, sdt, o, odt, rq)
        outs.append(o)
        keep.append((r, k))
    E.e2e_serve_start(ctx, max_inflight=4, max_queue=16, n_streams=2, max_batch=1)
    torch.cuda.synchronize()
    print("case serve overlap on two streams", flush=True)
    # the first round captures each stream's launch graph; the second is timed
    for rnd in range(2):
        tk = [E.e2e_serve_submit(ctx, r) for r, _ in keep]
        st = []
        for t in tk:
            code, s = E.e2e_serve_poll(ctx, t, -1)
            assert code == E.E2E_OK
            st.append(s)
    a, b = st
    print(f"  launch {a.t_launch_us:.0f} / {b.t_launch_us:.0f} us, done {a.t_done_us:.0f} / "
          f"{b.t_done_us:.0f} us; device {a.t_gpu_start_us:.0f}-{a.t_gpu_end_us:.0f} and "
          f"{b.t_gpu_start_us:.0f}-{b.t_gpu_end_us:.0f} us")
    assert b.t_launch_us < a.t_done_us
    assert b.t_gpu_start_us < a.t_gpu_end_us and a.t_gpu_start_us < b.t_gpu_end_us
    for o, ref in zip(outs, refs):
        assert np.array_equal(o.cpu().numpy(), ref)
    E.e2e_serve_stop(ctx)
    ld.free()
    E.e2e_destroy(ctx)
