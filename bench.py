"""Benchmark: ESPRESSO-shaped synthetic echellograms on one MI355X.

A step renders a batch of B frames of the 9216 x 9216, 85-order x 2-fiber x
2-slice, 1e6-samples-per-trace workload (11 x 11 field nodes of 32 x 32 x4
tabulated PSFs) in one persistent launch through the C ABI (a captured HIP
graph: planner, counter reset, render), every frame with its own Doppler
shift (U[-10, 10] m/s) and exposure scale.  Inputs are resident in HBM
before the timed region.  Prints one JSON line with:

* value: whole-job sample-PSF-pixel updates/s over the K timed steps;
* roofline: render_table against the 78.6 TFLOP/s ALU peak, flops counted as
  the deposit + stencil form (table_flops_frame), the kernel's time from HIP
  events on its stream (eager launches); traffic from the committed
  FETCH_SIZE / WRITE_SIZE summary while the kernel source is unchanged;
* cpu_baseline: the FP64 oracle on the host's cores (OpenMP driver) and on
  one core, on a bounded sample of the same frame;
* accuracy: per-pixel error / peak at stratified pixels and photocentre
  shifts (px and cm/s) of the timed frame, C2 at each precision and C3;
* secondary: C2 precision variants, noise, detector stage, extraction + CCF,
  aliasing sweep, C4, explicit SFIs, C3 (64 uneven frames in one launch);
* serve: the served C0/C1/C4 mix at 20 req/s and a load sweep.

  python bench.py [--steps K] [--warmup W] [--batch B] [--gpus 1]
  python bench.py --profile-once | --profile-sep PREC | --copy-calibration MIB
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# enough hardware queues that the serve loop's streams do not share one (HIP
# maps streams round-robin onto GPU_MAX_HW_QUEUES queues, 4 by default; two
# streams on one queue serialise); set before HIP initialises
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

METRIC = "sample·PSF-px updates/s + frames/s (ESPRESSO-shaped); p50/p99 render latency"
PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_ALU = 78.6e12         # flop/s, FP64 vector FMA (= FP32 FMA without packed math)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def table_flops_per_sample(sc):
    """Arithmetic of the exact deposit + stencil form, per wavelength sample.

    position: t (1 FMA), x Horner (deg_x FMA), y Horner (deg_y FMA), slot
    phases (2 FMA + 2 sub), node fractions (2 mul + 2 sub); deposits: 4 x
    and 4 y factors (8 mul, 4 sub) and 16 FMA; stencil: every deposit cell
    (2 x-slots x 2 rows per sample, shared by the samples that fall in one
    slot) meets a (kw/os+1)^2-pixel stencil per node, 4 nodes.
    """
    t = sc.traces[0]
    dx, dy = len(t.cx) - 1, len(t.cy) - 1
    per_sample = 2 * (1 + dx + dy) + 2 * 2 + 2 + 4 + 12 + 2 * 16
    # deposit cells per sample: slots per pixel / samples per pixel x rows
    xspan = abs(np.polynomial.polynomial.polyval(1.0, t.cx) - np.polynomial.polynomial.polyval(-1.0, t.cx))
    samples_per_px = t.n / xspan
    cells = (sc.psf.os / samples_per_px) * 2.0 * 4
    foot = (sc.psf.kw // sc.psf.os + 1) ** 2
    return per_sample + cells * 2 * foot


def table_flops_frame(sc):
    """Algorithmic flops of one table-path frame in the deposit + stencil form
    (the count the hot-path table states): each sample's 16 CIC deposits
    (2 x-slots x 2 rows x 4 nodes) at 2 flop each; then every non-zero
    deposit cell meets one (kw/os + 1)^2-tap stencil at 2 flop per tap.  A
    trace covers 4 slot columns per pixel of its x-span, each with 2 quarter
    rows (its samples' CIC pair) in each of 4 node layers."""
    P = np.polynomial.polynomial
    slots = 0.0
    for t in sc.traces:
        x0 = float(np.clip(P.polyval(-1.0, t.cx), -0.5, sc.nx - 0.5))
        x1 = float(np.clip(P.polyval(1.0, t.cx), -0.5, sc.nx - 0.5))
        slots += 4.0 * abs(x1 - x0)
    cells = slots * 2 * 4
    taps = (sc.psf.kw // sc.psf.os + 1) ** 2
    return 32.0 * sc.n_samples + 2.0 * taps * cells


def node_lines(sc):
    """Detector columns / rows of the PSF node grid (node m at m (n-1)/(g-1))."""
    gx, gy = int(sc.psf.gx), int(sc.psf.gy)
    xs = [m * (sc.nx - 1) / (gx - 1) for m in range(gx)] if gx > 1 else []
    ys = [m * (sc.ny - 1) / (gy - 1) for m in range(gy)] if gy > 1 else []
    return xs, ys


def gpu_samples(frame_t, sc, rq, tw, th, seed=0, n_each=30, n_win=4):
    """Pixel values of a rendered GPU frame at stratified pixels and in small
    windows around isolated line images, kept for the CPU leg's accuracy
    report (the oracle runs only there)."""
    from workloads import metrics
    g = frame_t.cpu().numpy().astype(np.float64)
    nxl, nyl = node_lines(sc)
    px, py = metrics.stratified_pixels(g, tw, th, node_x=nxl, node_y=nyl, n_each=n_each,
                                       seed=seed)
    wins = [(i0, j0, g[j0:j0 + 5, i0:i0 + 5].copy())
            for i0, j0 in metrics.line_windows(g, n=n_win, half=2, seed=seed)]
    return {"scene": sc, "req": rq, "px": px, "py": py, "g": g[py, px], "peak": float(g.max()),
            "windows": wins, "sum": float(g.sum())}


def measured_traffic():
    """HBM bytes per timed launch from the committed FETCH_SIZE / WRITE_SIZE
    counter summary (copy-calibrated), or None when render_table's source or
    the host code that orders its work list has changed since the counters
    were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "render_table_c1_batch4_hbm_traffic.md")
    csrc = os.path.join(ROOT, "paper_2008_05858_amd", "csrc")

    def sha(name):
        return hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest()
    try:
        txt = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", txt, re.S).group(1))
        same = (rec.get("kernel_source_sha256") == sha("k_table.hip") and
                rec.get("host_source_sha256") == sha("api.cpp"))
    except (OSError, AttributeError, ValueError):
        return None
    return rec["hbm_bytes_per_launch"] if same else None


def cpu_info():
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(nproc, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else nproc
    return model, nproc, threads


def cpu_leg(sc, samples, log):
    """The FP64 oracle on the host: its timing on bounded samples of the timed
    workload (one core, then every core the process may use), and the
    accuracy report of the GPU frames sampled in the timed runs (max |dF| /
    peak at stratified pixels; photocentres of isolated line images in px and
    cm/s; the paper's budget is 1e-5 px, about 1 cm/s)."""
    import oracle
    from workloads import metrics
    from workloads.synth import with_traces
    model, nproc, threads = cpu_info()
    mid = len(sc.traces) // 2
    one = with_traces(sc, [mid, mid + 1])
    t0 = time.perf_counter()
    oracle.render(one)
    dt1 = time.perf_counter() - t0
    upd1 = one.updates() / dt1
    ntr = min(len(sc.traces), 6 * threads)
    lo = max(0, min(len(sc.traces) - ntr, mid - ntr // 2))
    many = with_traces(sc, list(range(lo, lo + ntr)))
    log(f"cpu baseline: {threads} threads on {ntr} traces")
    t0 = time.perf_counter()
    oracle.render_omp(many, threads=threads)
    dtn = time.perf_counter() - t0
    updn = many.updates() / dtn
    base = {"value": updn, "unit": "sample·PSF-px updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{ntr} of {len(sc.traces)} traces (1e6 samples each, 81-px footprint) of "
                      f"the timed ESPRESSO-shaped frame, FP64, {threads} OpenMP threads "
                      f"(traces over threads, fixed-order sum), {dtn:.1f} s; single core: 2 "
                      f"traces, {dt1:.1f} s",
            "frames_per_s": updn / sc.updates(), "single_core_value": upd1,
            "single_core_frames_per_s": upd1 / sc.updates(), "cpu_model": model, "nproc": nproc}
    acc = {}
    for name, smp in samples.items():
        osc, rq = smp["scene"], smp["req"]
        o = oracle.render_pixels(osc, rq, smp["px"], smp["py"])
        err = float(np.max(np.abs(smp["g"] - o)) / smp["peak"])
        shifts = []
        for i0, j0, gw in smp["windows"]:
            jj, ii = np.mgrid[j0:j0 + 5, i0:i0 + 5]
            ow = oracle.render_pixels(osc, rq, ii.ravel(), jj.ravel()).reshape(5, 5)
            cg, co = metrics.centroid(gw, i0, j0), metrics.centroid(ow, i0, j0)
            lam, dxdl = metrics.dispersion_at(osc, cg[0], cg[1])
            dxp = cg[0] - co[0]
            shifts.append((abs(dxp), abs(100.0 * metrics.px_to_mps(dxp, lam, dxdl))))
        rec = {"pixels": int(len(smp["px"])), "max_abs_dF_over_peak": err,
               "photocentre_windows": len(shifts)}
        if shifts:
            rec["max_photocentre_shift_px"] = max(v[0] for v in shifts)
            rec["max_photocentre_shift_cm_s"] = max(v[1] for v in shifts)
        if "expected_sum" in smp:
            rec["flux_sum_rel_err"] = abs(smp["sum"] - smp["expected_sum"]) / smp["expected_sum"]
        acc[name] = rec
        log(f"accuracy {name}: {rec}")
    return base, acc


def serve_kinds(E, P, torch, ctx, c1, ld1, specs1, log):
    """The served workloads (tables and spectra resident on the device)."""
    from workloads import scene
    log("building c0 and c4 workloads for the serve mix")
    c0, c4 = scene("c0"), scene("c4")
    ld0, ld4 = P.Loaded(ctx, c0), P.Loaded(ctx, c4)
    sp0 = [torch.from_numpy(s).to("cuda") for s in c0.spectra]
    sp4 = [torch.from_numpy(s).to("cuda") for s in c4.spectra]
    return {"c0": (c0, ld0, sp0, E.E2E_F64, torch.float64, E.E2E_F64),
            "c1": (c1, ld1, specs1, E.E2E_F32, torch.float32, E.E2E_F32),
            "c4": (c4, ld4, sp4, E.E2E_F32, torch.float32, E.E2E_F32)}


def serve_bench(E, P, torch, ctx, kinds, n_req, rate, log, seed=777):
    """Served mix (C0 : C1 : C4 = 0.68 : 0.30 : 0.02) with Poisson arrivals;
    format / PSF tables and spectra resident; latency submit -> done."""
    import threading
    c0, c1, c4 = kinds["c0"][0], kinds["c1"][0], kinds["c4"][0]
    rng = np.random.Generator(np.random.PCG64(seed))
    names = rng.choice(["c0", "c1", "c4"], size=n_req, p=[0.68, 0.30, 0.02])
    gaps = rng.exponential(1.0 / rate, size=n_req)
    pool = {k: [torch.empty((v[0].ny, v[0].nx), dtype=v[4], device="cuda") for _ in range(8)]
            for k, v in kinds.items()}
    E.e2e_serve_start(ctx, max_inflight=8, max_queue=512, n_streams=3, max_batch=4)
    torch.cuda.synchronize()
    tickets, keep = [None] * n_req, []
    sem = {k: threading.Semaphore(8) for k in kinds}
    slot = {k: 0 for k in kinds}
    done_evt = []

    def submitter():
        t0 = time.perf_counter()
        tnext = t0
        for i, nm in enumerate(names):
            tnext += gaps[i]
            while time.perf_counter() < tnext:
                time.sleep(min(0.002, max(0.0, tnext - time.perf_counter())))
            sc, ld, sp, sdt, tdt, odt = kinds[nm]
            sem[nm].acquire()
            out = pool[nm][slot[nm] % 8]
            slot[nm] += 1
            r, k = P.make_req(ld, [s.data_ptr() for s in sp], sdt, out.data_ptr(), odt,
                              spectra_on_device=True, out_on_device=True,
                              rv_mps=float(rng.uniform(-10, 10)))
            keep.append((r, k))
            tickets[i] = E.e2e_serve_submit(ctx, r)
        done_evt.append(time.perf_counter())

    th = threading.Thread(target=submitter)
    t_start = time.perf_counter()
    th.start()
    lat = {k: [] for k in kinds}
    allat = []
    for i in range(n_req):
        while tickets[i] is None:
            time.sleep(0.0005)
        code, st = E.e2e_serve_poll(ctx, tickets[i], -1)
        sem[names[i]].release()
        ms = (st.t_done_us - st.t_submit_us) / 1e3
        lat[names[i]].append(ms)
        allat.append(ms)
    t_end = time.perf_counter()
    th.join()
    E.e2e_serve_stop(ctx)
    upd = {"c0": c0.updates(), "c1": c1.updates(), "c4": c4.updates()}
    tot_upd = sum(upd[n] for n in names)
    return {"requests": n_req, "rate_per_s": rate,
            "mix": {k: int(np.sum(names == k)) for k in kinds},
            "frames_per_s": n_req / (t_end - t_start),
            "updates_per_s": tot_upd / (t_end - t_start),
            "latency_ms_p50": float(np.percentile(allat, 50)),
            "latency_ms_p99": float(np.percentile(allat, 99)),
            "by_kind_ms_p50_p99": {k: [float(np.percentile(v, 50)), float(np.percentile(v, 99))]
                                   for k, v in lat.items() if v}}


def secondary(E, P, torch, ctx, sc1, ld1, specs1, log, samples):
    """Measurements of the other rows of the path, beside the headline:
    separable PSF (VALU FP64/FP32 and MFMA fp16/bf16 hi/lo) on the C2 frame,
    Poisson noise on the C1 frame (HBM-bound: read + write the frame), and a
    HIRES-shaped C4 frame on the table path.  Kernel times are HIP-event
    averages over `reps` launches after one warm-up."""
    from workloads import scene
    res = {}
    reps = 3

    def kernel_ms(render, name):
        render()
        torch.cuda.synchronize()
        E.e2e_reset_kernel_time(ctx)
        E.e2e_set_profiling(ctx, True)
        for _ in range(reps):
            render()
        E.e2e_set_profiling(ctx, False)
        n, ms = E.e2e_kernel_time(ctx, name)
        return ms / max(n, 1)

    log("secondary: c2 separable precision variants")
    c2 = scene("c2")
    ld2 = P.Loaded(ctx, c2)
    sp2 = [torch.from_numpy(s).to("cuda") for s in c2.spectra]
    out2 = torch.empty((c2.ny, c2.nx), dtype=torch.float32, device="cuda")
    upd2 = c2.updates()
    sep = {}
    for prec, kname in (("f64", "render_sep"), ("f32", "render_sep"),
                        ("f16_hilo", "render_sep_mfma"), ("bf16_hilo", "render_sep_mfma")):
        r, k = P.make_req(ld2, [s.data_ptr() for s in sp2], E.E2E_F32, out2.data_ptr(),
                          E.E2E_F32, spectra_on_device=True, out_on_device=True, rv_mps=2.0,
                          precision=prec)
        ms = kernel_ms(lambda: E.e2e_render(ctx, r), kname)
        sep[prec] = {"kernel": kname, "kernel_ms": ms, "updates_per_s": upd2 / (ms / 1e3),
                     "frames_per_s": 1e3 / ms}
        from workloads import Request
        mfma = kname == "render_sep_mfma"
        samples[f"c2_{prec}"] = gpu_samples(out2, c2, Request(rv_mps=2.0), 64 if mfma else 16,
                                            32 if mfma else 16, seed=11, n_each=20)
    res["c2_separable"] = {"updates_per_frame": upd2, "footprint_px": (2 * c2.psf.half_width + 1) ** 2,
                           "by_precision": sep}
    ld2.free()
    del sp2, out2

    log("secondary: poisson noise on the c1 frame")
    out1 = torch.empty((sc1.ny, sc1.nx), dtype=torch.float32, device="cuda")
    r, k = P.make_req(ld1, [s.data_ptr() for s in specs1], E.E2E_F32, out1.data_ptr(),
                      E.E2E_F32, spectra_on_device=True, out_on_device=True, rv_mps=1.0,
                      poisson=True, seed=7)
    ms = kernel_ms(lambda: E.e2e_render(ctx, r), "noise")
    nbytes = 2 * sc1.nx * sc1.ny * 4
    res["noise_c1"] = {"kernel_ms": ms, "bytes_per_launch": nbytes,
                       "achieved_GBps": nbytes / (ms / 1e3) / 1e9,
                       "hbm_frac": nbytes / (ms / 1e3) / PEAK_HBM}

    log("secondary: detector stage on the c1 frame")
    from workloads import XTALK_CCD, prnu_map
    g1 = torch.from_numpy(prnu_map(sc1.nx, sc1.ny, 1001)).to("cuda")
    adu = torch.empty((sc1.ny, sc1.nx), dtype=torch.int16, device="cuda")
    det = {}
    for label, shot, ron in (("shot_read_noise", 1, 3.0), ("noise_free", 0, 0.0)):
        d = E.e2e_detector_desc()
        for q, v in enumerate(XTALK_CCD.reshape(9)):
            d.xtalk[q] = float(v)
        d.exposure_s, d.dark_e_per_s, d.ron_e = 900.0, 0.011, ron
        d.gain_e_per_adu, d.bias_adu, d.bits, d.shot_noise = 1.37, 1000.0, 16, shot
        d.seed, d.frame_index = 5, 1

        def run(d=d):
            E.e2e_detector(ctx, d, out1.data_ptr(), E.E2E_F32, g1.data_ptr(), sc1.nx, sc1.ny,
                           adu.data_ptr(), 1)
        px = sc1.nx * sc1.ny
        ms = kernel_ms(run, "detector")
        # algorithmic bytes: FP32 frame + FP32 gains in, uint16 ADU out
        nb = px * (4 + 4 + 2)
        det[label] = {"kernel_ms": ms, "bytes_per_launch": nb,
                      "achieved_GBps": nb / (ms / 1e3) / 1e9,
                      "hbm_frac": nb / (ms / 1e3) / PEAK_HBM, "px_per_s": px / (ms / 1e3)}
    res["detector_c1"] = det
    del out1, g1, adu

    log("secondary: c1 extraction + CCF (closing the loop)")
    import ctypes as C
    import dataclasses as dc
    out1 = torch.empty((sc1.ny, sc1.nx), dtype=torch.float32, device="cuda")
    flat1 = dc.replace(sc1, spectra=[np.full_like(s_, 1e4) for s_ in sc1.spectra])
    ldf = P.Loaded(ctx, flat1)
    spf = [torch.from_numpy(s_).to("cuda") for s_ in flat1.spectra]
    r, k = P.make_req(ldf, [s_.data_ptr() for s_ in spf], E.E2E_F32, out1.data_ptr(), E.E2E_F32,
                      spectra_on_device=True, out_on_device=True)
    E.e2e_render(ctx, r)
    ntr = len(sc1.traces)
    flux = torch.empty((ntr, sc1.nx), dtype=torch.float64, device="cuda")
    flatx = torch.empty_like(flux)
    edges = torch.empty((ntr, sc1.nx + 1), dtype=torch.float64, device="cuda")
    E.e2e_extract(ctx, ld1.fmt, out1.data_ptr(), E.E2E_F32, 4.5, flatx.data_ptr(),
                  edges.data_ptr(), 1)
    v_in = 1234.5
    r, k = P.make_req(ld1, [s_.data_ptr() for s_ in specs1], E.E2E_F32, out1.data_ptr(),
                      E.E2E_F32, spectra_on_device=True, out_on_device=True, rv_mps=v_in)
    E.e2e_render(ctx, r)
    tm = (C.c_void_p * len(specs1))(*[s_.data_ptr() for s_ in specs1])
    cc = torch.empty((ntr, 101), dtype=torch.float64, device="cuda")
    creq = E.e2e_ccf_req(flux.data_ptr(), flatx.data_ptr(), edges.data_ptr(), tm, len(specs1),
                         E.E2E_F32, 1, 101, -5000.0, 100.0, 1.5, cc.data_ptr(), None)
    rv_box = []

    def loop():
        E.e2e_extract(ctx, ld1.fmt, out1.data_ptr(), E.E2E_F32, 4.5, flux.data_ptr(),
                      edges.data_ptr(), 1)
        rv_box.append(E.e2e_ccf(ctx, ld1.fmt, creq))
    ms_x = kernel_ms(loop, "extract")
    ms_s = kernel_ms(loop, "template_smooth")
    ms_c = kernel_ms(loop, "ccf")
    res["loop_c1"] = {"extract_ms": ms_x, "template_smooth_ms_per_group": ms_s,
                      "template_smooth_ms": ms_s * ((ntr + 63) // 64), "ccf_ms_per_group": ms_c,
                      "ccf_ms": ms_c * ((ntr + 63) // 64), "traces": ntr, "n_v": 101,
                      "rv_injected_mps": v_in, "rv_recovered_mps": rv_box[-1]}
    ldf.free()
    del spf, flux, flatx, edges, cc, out1

    log("secondary: aliasing study (flat fields, wavelength step x sub-pixel sampling)")
    from workloads.synth import aliasing_flat
    from workloads.metrics import aliasing_level
    cfg = [(p_, s_) for p_ in (1, 1.5, 2, 2.5, 3, 5, 10, 20) for s_ in (1, 2, 5, 10)]
    scs = [aliasing_flat(p_, s_, length_px=1000.0) for p_, s_ in cfg]
    lds = [P.Loaded(ctx, sc_) for sc_ in scs]
    sps = [[torch.from_numpy(x_).to("cuda") for x_ in sc_.spectra] for sc_ in scs]
    outs = [torch.empty((sc_.ny, sc_.nx), dtype=torch.float64, device="cuda") for sc_ in scs]
    rqs, keep = [], []
    for sc_, ld_, sp_, o_ in zip(scs, lds, sps, outs):
        r_, k_ = P.make_req(ld_, [x_.data_ptr() for x_ in sp_], E.E2E_F32, o_.data_ptr(),
                            E.E2E_F64, spectra_on_device=True, out_on_device=True)
        rqs.append(r_)
        keep.append(k_)
    ms = kernel_ms(lambda: E.e2e_render_batch(ctx, rqs), "render_sfi")
    table = {}
    for (p_, s_), sc_, o_ in zip(cfg, scs, outs):
        a_ = aliasing_level(o_.cpu().numpy(), sc_)
        table[f"{p_}/{s_}"] = [a_["row_ripple"], a_["row_photon"]]
    res["aliasing_sweep"] = {"frames": len(cfg), "batch_ms": ms,
                             "sfi": int(sum(sc_.n_samples for sc_ in scs)),
                             "key": "SFIs per resolution element / sub-pixels",
                             "row_ripple_vs_photon": table}
    for ld_ in lds:
        ld_.free()
    del sps, outs

    log("secondary: c4 HIRES-shaped frame")
    c4 = scene("c4")
    ld4 = P.Loaded(ctx, c4)
    sp4 = [torch.from_numpy(s).to("cuda") for s in c4.spectra]
    out4 = torch.empty((c4.ny, c4.nx), dtype=torch.float32, device="cuda")
    r, k = P.make_req(ld4, [s.data_ptr() for s in sp4], E.E2E_F32, out4.data_ptr(),
                      E.E2E_F32, spectra_on_device=True, out_on_device=True, rv_mps=-1.0)
    ms = kernel_ms(lambda: E.e2e_render(ctx, r), "render_table")
    res["c4_table"] = {"kernel_ms": ms, "updates_per_s": c4.updates() / (ms / 1e3),
                       "frames_per_s": 1e3 / ms, "samples": c4.n_samples}
    ld4.free()
    del sp4, out4

    log("secondary: c5 explicit-SFI frame")
    c5 = scene("c5_sfi")
    ld5 = P.Loaded(ctx, c5)
    sp5 = [torch.from_numpy(s).to("cuda") for s in c5.spectra]
    out5 = torch.empty((c5.ny, c5.nx), dtype=torch.float32, device="cuda")
    r, k = P.make_req(ld5, [s.data_ptr() for s in sp5], E.E2E_F32, out5.data_ptr(),
                      E.E2E_F32, spectra_on_device=True, out_on_device=True, rv_mps=500.0)
    ms = kernel_ms(lambda: E.e2e_render(ctx, r), "render_sfi")
    n_sfi = c5.n_samples
    w = 2 * c5.psf.half_width + 1
    res["c5_sfi"] = {"kernel_ms": ms, "sfi": n_sfi, "sfi_per_s": n_sfi / (ms / 1e3),
                     "subpixel_evals_per_s": n_sfi * w * w * c5.psf.subpix ** 2 / (ms / 1e3),
                     "window_px": w, "subpixels": c5.psf.subpix,
                     "fiber_radius_px": c5.psf.fiber_radius,
                     "paper_s_per_sfi_k80": 0.17,
                     "sfi_rate_vs_paper_k80": n_sfi / (ms / 1e3) * 0.17}
    ld5.free()
    return res


def c3_bench(E, P, torch, ctx, sc1, ld1, specs1, log, samples, n_frames=64):
    """The batched configuration: n_frames renders of uneven size in one
    persistent launch through the captured-graph path, half ESPRESSO-shaped
    (9216^2) and half a 4096^2, 40-order, 1-fiber variant in a seeded order,
    each with its own Doppler shift (U[-10, 10] m/s) and exposure (U[1e3, 1e5]
    photons per sample at the continuum), Poisson noise on every other frame."""
    from workloads import Request, scene
    log("c3: building the 4096^2 variant")
    v = scene("c3v")
    ldv = P.Loaded(ctx, v)
    spv = [torch.from_numpy(x).to("cuda") for x in v.spectra]
    rng = np.random.Generator(np.random.PCG64(1003))
    kinds = rng.permutation(np.array([0] * (n_frames // 2) + [1] * (n_frames - n_frames // 2)))
    outs, rr, keep, meta = [], [], [], []
    stream = torch.cuda.current_stream().cuda_stream  # the benchmark's own stream
    assert stream, "c3_bench needs a non-default current stream"
    for f, kd in enumerate(kinds):
        sc, ld, sp = (sc1, ld1, specs1) if kd == 0 else (v, ldv, spv)
        rq = Request(rv_mps=float(rng.uniform(-10, 10)),
                     flux_scale=float(rng.uniform(1e3, 1e5) / 1e4), seed=99,
                     frame_index=f, poisson=bool(f % 2))
        o = torch.empty((sc.ny, sc.nx), dtype=torch.float32, device="cuda")
        r, k = P.make_req(ld, [x.data_ptr() for x in sp], E.E2E_F32, o.data_ptr(), E.E2E_F32,
                          spectra_on_device=True, out_on_device=True, rv_mps=rq.rv_mps,
                          flux_scale=rq.flux_scale, seed=rq.seed, frame_index=f,
                          poisson=rq.poisson, stream=stream, flags=E.E2E_FLAG_ASYNC)
        outs.append(o)
        rr.append(r)
        keep.append(k)
        meta.append((sc, rq))
    torch.cuda.synchronize()
    log("c3: autotune + warm-up")
    tune = E.e2e_autotune(ctx, rr)
    E.e2e_render_batch(ctx, rr)
    E.e2e_sync(ctx, stream)
    reps = 3
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        E.e2e_render_batch(ctx, rr)
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    E.e2e_sync(ctx, stream)
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    # kernel split of one eager launch
    E.e2e_reset_kernel_time(ctx)
    E.e2e_set_profiling(ctx, True)
    E.e2e_render_batch(ctx, rr)
    E.e2e_set_profiling(ctx, False)
    E.e2e_sync(ctx, stream)
    split = {k: E.e2e_kernel_time(ctx, k)[1] for k in ("plan", "render_table", "noise")}
    upd = sum(sc.updates() for sc, _ in meta)
    # a noiseless frame of each kind for the accuracy report
    for kd, name in ((0, "c3_c1_frame"), (1, "c3_variant_frame")):
        f = next(i for i in range(n_frames) if kinds[i] == kd and not meta[i][1].poisson)
        samples[name] = gpu_samples(outs[f], meta[f][0], meta[f][1], 56, 32, seed=30 + kd,
                                    n_each=20)
    rec = {"frames": n_frames, "c1_frames": int((kinds == 0).sum()),
           "variant_frames": int((kinds == 1).sum()), "poisson_frames": n_frames // 2,
           "ms_per_launch": ms, "wall_ms_per_launch": 1e3 * wall, "frames_per_s": n_frames / (ms / 1e3),
           "updates_per_s": upd / (ms / 1e3), "kernel_ms_eager": split,
           "autotune": {"chunk_tiles": tune.chunk, "workgroups_per_cu": tune.resident},
           "path": "render_batch, captured HIP graph (one persistent launch)"}
    del outs
    ldv.free()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--plain-frames", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=120,
                    help="served HIRES-shaped mix; 0 skips it")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrivals per second")
    ap.add_argument("--c3-frames", type=int, default=64,
                    help="frames of the batched configuration (0 skips it)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the separable / noise / HIRES-shaped measurements")
    ap.add_argument("--profile-once", action="store_true",
                    help="one batch launch of the timed configuration, then exit (for counters)")
    ap.add_argument("--profile-sep", default="", metavar="PREC",
                    help="two C2 separable renders at PREC (f64, f32, f16_hilo, bf16_hilo), "
                         "then exit (for counters)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one device copy of MIB MiB and exit (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(frames shard by detector row bands with no collective; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2008_05858_amd as P
    from paper_2008_05858_amd import e2e as E
    from workloads import scene

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB")
        return
    if args.profile_sep:
        c2 = scene("c2")
        ctx = E.e2e_create(0, 0)
        ld2 = P.Loaded(ctx, c2)
        sp2 = [torch.from_numpy(s).to("cuda") for s in c2.spectra]
        out2 = torch.empty((c2.ny, c2.nx), dtype=torch.float32, device="cuda")
        r, k = P.make_req(ld2, [s.data_ptr() for s in sp2], E.E2E_F32, out2.data_ptr(),
                          E.E2E_F32, spectra_on_device=True, out_on_device=True, rv_mps=2.0,
                          precision=args.profile_sep)
        for _ in range(2):
            E.e2e_render(ctx, r)
        torch.cuda.synchronize()
        log(f"two c2 renders at {args.profile_sep} done")
        ld2.free()
        E.e2e_destroy(ctx)
        return
    log("building c1 workload")
    sc = scene("c1")
    ctx = E.e2e_create(0, 0)
    ld = P.Loaded(ctx, sc)
    specs = [torch.from_numpy(s).to("cuda") for s in sc.spectra]
    B = args.batch
    outs = [torch.empty((sc.ny, sc.nx), dtype=torch.float32, device="cuda") for _ in range(B)]
    rng = np.random.Generator(np.random.PCG64(4242))
    # an explicit stream (the default stream's handle is 0, which the library
    # reads as "the context's stream"): the launches and the events that time
    # them share it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    sptr = stream.cuda_stream

    last_params = []

    def reqs_for(step):
        rr, keep = [], []
        last_params.clear()
        for b in range(B):
            rv, fs = float(rng.uniform(-10, 10)), float(rng.uniform(1e3, 1e5) / 1e4)
            r, k = P.make_req(ld, [s.data_ptr() for s in specs], E.E2E_F32, outs[b].data_ptr(),
                              E.E2E_F32, spectra_on_device=True, out_on_device=True,
                              rv_mps=rv, flux_scale=fs,
                              seed=1234, frame_index=step * B + b, stream=sptr,
                              flags=E.E2E_FLAG_ASYNC)
            rr.append(r)
            keep.append(k)
            last_params.append((rv, fs))
        return rr, keep

    torch.cuda.synchronize()
    if args.profile_once:
        rr, keep = reqs_for(0)
        E.e2e_render_batch(ctx, rr)
        torch.cuda.synchronize()
        log(f"one batch launch of {B} frames done")
        ld.free()
        E.e2e_destroy(ctx)
        return
    log("warmup")
    for w in range(args.warmup):
        rr, keep = reqs_for(w)
        E.e2e_render_batch(ctx, rr)
    torch.cuda.synchronize()

    # launch autotuning on the timed configuration (not timed); the plain
    # renderer below uses the same work-unit length
    rr, keep = reqs_for(0)
    tune = E.e2e_autotune(ctx, rr)
    tune_rec = {"chunk_tiles": tune.chunk, "workgroups_per_cu": tune.resident,
                "ms_per_launch": tune.ms,
                "candidates": [[tune.cand_chunk[i], tune.cand_resident[i], round(tune.cand_ms[i], 4)]
                               for i in range(tune.n_candidates)]}
    log(f"autotune: chunk {tune.chunk} tiles, {tune.resident} workgroups/CU, {tune.ms:.3f} ms")
    torch.cuda.synchronize()

    # timed region: K steps on the captured-graph path (profiling off),
    # events on the launch stream around each batch launch
    all_reqs = [reqs_for(s) for s in range(args.steps)]
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (rr, keep), (a, b) in zip(all_reqs, evs):
        a.record()
        E.e2e_render_batch(ctx, rr)
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    E.e2e_sync(ctx, sptr)  # device checks of the asynchronous launches
    graph_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    elapsed = t1 - t0
    frames = args.steps * B
    upd_frame = sc.updates()
    value = frames * upd_frame / elapsed
    ms_step = 1e3 * elapsed / args.steps
    log(f"batch: {frames} frames in {elapsed:.3f} s; {graph_ms:.3f} ms per graph launch")

    # the kernel split (eager launches, a HIP event pair around each kernel)
    E.e2e_reset_kernel_time(ctx)
    E.e2e_set_profiling(ctx, True)
    for s_ in range(3):
        rr, keep = reqs_for(s_)
        E.e2e_render_batch(ctx, rr)
    E.e2e_set_profiling(ctx, False)
    E.e2e_sync(ctx, sptr)
    n_tab, ms_tab = E.e2e_kernel_time(ctx, "render_table")
    n_plan, ms_plan = E.e2e_kernel_time(ctx, "plan")
    log(f"render_table {ms_tab / max(n_tab, 1):.3f} ms per launch (eager)")

    # accuracy samples of the last timed launch's frame 0 (its request drawn
    # first in reqs_for for the last step)
    from workloads import Request
    last_rv, last_fs = last_params[0]
    samples = {}
    samples["c1_timed_frame"] = gpu_samples(outs[0], sc, Request(rv_mps=last_rv, flux_scale=last_fs),
                                            56, 32, seed=1)
    samples["c1_timed_frame"]["expected_sum"] = last_fs * sum(
        float(sc.spectra[t.slot].astype(np.float64).sum()) * t.thr for t in sc.traces)

    # plain single-frame renderer: per-frame latency
    lat = []
    for f in range(args.plain_frames):
        r, k = P.make_req(ld, [s.data_ptr() for s in specs], E.E2E_F32, outs[0].data_ptr(),
                          E.E2E_F32, spectra_on_device=True, out_on_device=True,
                          rv_mps=float(rng.uniform(-10, 10)), stream=sptr)
        torch.cuda.synchronize()
        a = time.perf_counter()
        E.e2e_render(ctx, r)
        lat.append(1e3 * (time.perf_counter() - a))
    plain_fps = 1e3 / float(np.mean(lat[2:] if len(lat) > 4 else lat))

    # roofline of the dominant kernel (render_table), per launch = B frames
    avg_s = (ms_tab / max(n_tab, 1)) / 1e3
    flops_launch = B * table_flops_frame(sc)
    alt_flops_launch = B * sc.n_samples * table_flops_per_sample(sc)
    # algorithmic bytes: the frames share one spectrum set, read once per launch
    bytes_launch = sc.spectrum_bytes() + B * sc.nx * sc.ny * 4
    alu = flops_launch / avg_s
    hbm = bytes_launch / avg_s
    traffic = measured_traffic()
    roof = {"bound": "alu", "achieved": alu / 1e12, "peak": PEAK_ALU / 1e12, "unit": "TFLOP/s",
            "frac": alu / PEAK_ALU, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_over_algorithmic": (traffic / bytes_launch) if traffic else None,
            "kernel": "render_table", "kernel_ms": avg_s * 1e3,
            "graph_launch_ms": graph_ms,
            "algorithmic_flops_per_launch": flops_launch,
            "flop_count": "16 CIC deposits x 2 flop per sample + (kw/os+1)^2 taps x 2 flop per "
                          "non-zero deposit cell (4 slot columns per px of x-span x 2 rows x 4 "
                          "node layers per trace)",
            "alt_count": {"flops_per_sample": table_flops_per_sample(sc),
                          "achieved": alt_flops_launch / avg_s / 1e12,
                          "frac": alt_flops_launch / avg_s / PEAK_ALU},
            "hbm_view": {"achieved_GBps": hbm / 1e9, "frac": hbm / PEAK_HBM,
                         "algorithmic_bytes_per_launch": bytes_launch}}
    res = {"metric": METRIC, "value": value, "unit": "sample·PSF-px updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "c1: ESPRESSO-shaped 9216x9216, 85 orders x 2 fibers x "
                                  "2 slices, 1e6 samples/trace, 11x11 nodes of 32x32 x4 tables",
                      "frames_per_step": B, "mode": "render_batch (persistent, captured graph)",
                      "updates_per_frame": upd_frame, "out_dtype": "f32",
                      "precision": "FP64 positions and moment sums; stencil products fp16 "
                                   "hi/lo on MFMA with FP32 accumulation; FP64 tile sums; "
                                   "FP32 output"},
           "frames_per_s": frames / elapsed, "plain_frames_per_s": plain_fps,
           "latency_ms_p50": float(np.percentile(lat, 50)),
           "latency_ms_p99": float(np.percentile(lat, 99)),
           "plan_ms_per_launch": ms_plan / max(n_plan, 1),
           "autotune": tune_rec,
           "roofline": roof}
    if not args.no_secondary:
        res["secondary"] = secondary(E, P, torch, ctx, sc, ld, specs, log, samples)
        if args.c3_frames > 0:
            log("secondary: c3 batch")
            res["secondary"]["c3_batch"] = c3_bench(E, P, torch, ctx, sc, ld, specs, log, samples,
                                                    n_frames=args.c3_frames)
    if args.serve_requests > 0:
        kinds = serve_kinds(E, P, torch, ctx, sc, ld, specs, log)
        res["serve"] = serve_bench(E, P, torch, ctx, kinds, args.serve_requests,
                                   args.serve_rate, log)
        res["latency_ms_p50"] = res["serve"]["latency_ms_p50"]
        res["latency_ms_p99"] = res["serve"]["latency_ms_p99"]
        res["latency_source"] = "served HIRES-shaped mix, submit to done"
        res["plain_latency_ms_p50"] = float(np.percentile(lat, 50))
        sweep = []
        for rate, n in ((5.0, 20), (20.0, 40), (80.0, 60), (200.0, 80)):
            log(f"serve sweep: {rate:g} req/s")
            r_ = serve_bench(E, P, torch, ctx, kinds, n, rate, log, seed=int(rate))
            sweep.append({k: r_[k] for k in ("rate_per_s", "requests", "frames_per_s",
                                             "latency_ms_p50", "latency_ms_p99")})
        res["serve"]["load_sweep"] = sweep
        kinds["c0"][1].free()
        kinds["c4"][1].free()
        del kinds
    if not args.no_cpu_baseline:
        log("cpu leg: oracle timing and the accuracy report")
        res["cpu_baseline"], res["accuracy"] = cpu_leg(sc, samples, log)
    print(json.dumps(res), flush=True)
    ld.free()
    E.e2e_destroy(ctx)


if __name__ == "__main__":
    main()
