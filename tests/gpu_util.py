"""Helpers for the GPU tests: scene -> device buffers -> C ABI -> numpy."""
import numpy as np

import paper_2008_05858_amd as P
from paper_2008_05858_amd import e2e as E

_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        _ctx = E.e2e_create(0, 0)
    return _ctx


def device_spectra(scene):
    import torch
    specs = [torch.from_numpy(np.ascontiguousarray(s)).to("cuda") for s in scene.spectra]
    dt = E.E2E_F64 if scene.spectra[0].dtype == np.float64 else E.E2E_F32
    return specs, dt


def out_tensor(scene, dtype=None):
    import torch
    odt = dtype or scene.out_dtype
    t = torch.zeros((scene.ny, scene.nx), dtype=torch.float64 if odt == "f64" else torch.float32,
                    device="cuda")
    return t, (E.E2E_F64 if odt == "f64" else E.E2E_F32)


def request_for(loaded, scene, specs, sdt, out, odt, req=None, **kw):
    r = dict(rv_mps=0.0, flux_scale=1.0, seed=0, frame_index=0, poisson=False, precision="f64")
    if req is not None:
        r.update(rv_mps=req.rv_mps, flux_scale=req.flux_scale, seed=req.seed,
                 frame_index=req.frame_index, poisson=req.poisson, precision=req.precision)
    r.update(kw)
    return P.make_req(loaded, [s.data_ptr() for s in specs], sdt, out.data_ptr(), odt,
                      spectra_on_device=True, out_on_device=True, **r)


def render(scene, req=None, loaded=None, out_dtype=None, context=None, **kw):
    """One frame through e2e_render (on `context`, default the shared one)."""
    import torch
    c = context if context is not None else ctx()
    own = loaded is None
    loaded = loaded or P.Loaded(c, scene)
    specs, sdt = device_spectra(scene)
    out, odt = out_tensor(scene, out_dtype)
    r, keep = request_for(loaded, scene, specs, sdt, out, odt, req, **kw)
    torch.cuda.synchronize()
    E.e2e_render(c, r)
    res = out.cpu().numpy()
    if own:
        loaded.free()
    return res


def render_batch(scenes, reqs, loadeds, context=None):
    import torch
    c = context if context is not None else ctx()
    outs, rr, keeps = [], [], []
    for sc, rq, ld in zip(scenes, reqs, loadeds):
        specs, sdt = device_spectra(sc)
        out, odt = out_tensor(sc)
        r, keep = request_for(ld, sc, specs, sdt, out, odt, rq)
        outs.append(out)
        rr.append(r)
        keeps.append((specs, keep))
    torch.cuda.synchronize()
    E.e2e_render_batch(c, rr)
    return [o.cpu().numpy() for o in outs]
