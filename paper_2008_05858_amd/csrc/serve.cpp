// Continuous-batching request loop.  The paper's cloud layer (Sec. 3) sizes
// each simulation from its database, allocates compute accordingly and
// distributes the work; on one GPU that becomes: admit a request when a slot
// and its HBM footprint are free, merge the admitted requests that share a
// PSF kind into one persistent batch launch, and keep several such launches
// in flight on separate streams so new arrivals start while earlier frames
// are still rendering.  Format and PSF tables stay resident; each request's
// frame depends only on its own inputs, so it is bitwise the same alone or
// in any mix.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <string>
#include <thread>

#include "api_internal.h"

using namespace e2e;

namespace e2e {

struct SReq {
    e2e_ticket id = 0;
    e2e_render_req r{};
    std::vector<const void *> specs;       // per slot (device pointers once admitted)
    std::vector<void *> host_stage;        // pinned copies of host spectra
    std::vector<size_t> spec_bytes;
    std::vector<void *> dev_owned;         // device buffers freed on completion
    void *user_out = nullptr;
    void *out_stage = nullptr;             // pinned copy of the frame (host output)
    size_t out_bytes = 0;
    uint64_t footprint = 0;
    FormatRes *fmt = nullptr;
    PsfRes *psf = nullptr;
    e2e_render_stats st{};
    e2e_status status = E2E_PENDING;
    std::string msg;
    bool done = false;
};

struct Flight {
    int stream = -1;
    hipEvent_t ev0 = nullptr, ev = nullptr;  // before the first, after the last kernel
    std::vector<SReq *> reqs;
    e2e_status launch_status = E2E_OK;
};

struct Server {
    e2e_serve_config cfg{};
    std::thread th;
    std::mutex m;
    std::condition_variable cv, cv_done;
    std::deque<SReq *> queue;
    std::vector<Flight> flights;
    std::map<e2e_ticket, SReq *> all;
    std::vector<hipStream_t> streams;
    std::vector<bool> stream_busy;
    hipEvent_t ref = nullptr;              // device time zero of the loop
    uint64_t reserved = 0;
    int admitted = 0;
    e2e_ticket next = 1;
    bool stop = false;
};

}  // namespace e2e

// Device and host buffers of a finished request, released without S->m held
// (hipFree can wait on other streams' work).
static void release(SReq *q)
{
    for (void *p : q->dev_owned) hipFree(p);
    q->dev_owned.clear();
    for (void *p : q->host_stage) hipHostFree(p);
    q->host_stage.clear();
    if (q->out_stage) hipHostFree(q->out_stage);
    q->out_stage = nullptr;
}

// Bookkeeping of a finished request (S->m held).
static void finish(e2e_ctx *ctx, Server *S, SReq *q, e2e_status st, const std::string &msg)
{
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (q->fmt) q->fmt->refs--;
        if (q->psf) q->psf->refs--;
    }
    q->st.t_done_us = now_us(ctx);
    q->msg = msg;
    q->st.status = st;
    q->status = st;
    q->done = true;
    S->reserved -= q->footprint;
    S->admitted -= 1;
}

// Upload host spectra and allocate device (and pinned) frames for an
// admitted request; called without S->m held.
static e2e_status stage_in(SReq *q, hipStream_t s)
{
    hipError_t e;
    for (size_t i = 0; i < q->specs.size(); ++i) {
        if (q->r.spectra_on_device || !q->host_stage[i]) continue;
        void *d = nullptr;
        if ((e = hipMalloc(&d, q->spec_bytes[i])) != hipSuccess) return hip_fail(e, "serve spectra");
        q->dev_owned.push_back(d);
        if ((e = hipMemcpyAsync(d, q->host_stage[i], q->spec_bytes[i], hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return hip_fail(e, "serve spectra upload");
        q->specs[i] = d;
    }
    if (!q->r.out_on_device) {
        void *d = nullptr;
        if ((e = hipMalloc(&d, q->out_bytes)) != hipSuccess) return hip_fail(e, "serve frame");
        q->dev_owned.push_back(d);
        q->r.out = d;
        if ((e = hipHostMalloc(&q->out_stage, q->out_bytes)) != hipSuccess) {
            q->out_stage = nullptr;
            return hip_fail(e, "serve frame staging");
        }
    }
    q->r.spectra = q->specs.data();
    q->r.spectra_on_device = 1;
    q->r.out_on_device = 1;
    q->r.flags |= E2E_FLAG_ASYNC;
    q->r.hip_stream = s;
    return E2E_OK;
}

// Requests of one launch: the queue head, then later requests of the same
// PSF kind / table size / precision / spectrum type (look-ahead, queue order
// kept), while slots and memory last.  S->m held.
static std::vector<SReq *> take_group(e2e_ctx *ctx, Server *S, uint64_t avail)
{
    std::vector<SReq *> group;
    for (auto it = S->queue.begin(); it != S->queue.end() &&
                                     (int)group.size() < S->cfg.max_batch &&
                                     S->admitted < S->cfg.max_inflight;) {
        SReq *q = *it;
        if (!group.empty()) {
            const SReq *g0 = group[0];
            if (q->psf->kind != g0->psf->kind || q->psf->kw != g0->psf->kw ||
                q->r.precision != g0->r.precision ||
                q->r.spectrum_dtype != g0->r.spectrum_dtype) {
                ++it;
                continue;
            }
        }
        if (S->reserved + q->footprint > avail) {
            if (group.empty()) break;  // the head waits for memory; nothing overtakes it
            ++it;
            continue;
        }
        it = S->queue.erase(it);
        S->reserved += q->footprint;
        S->admitted += 1;
        q->st.t_admit_us = now_us(ctx);
        group.push_back(q);
    }
    return group;
}

static void loop(e2e_ctx *ctx, Server *S)
{
    hipSetDevice(ctx->dev);
    std::unique_lock<std::mutex> lk(S->m);
    for (;;) {
        // reap finished launches: take them out under the lock, copy frames
        // and free buffers without it, then publish the results
        std::vector<Flight> done;
        for (size_t i = 0; i < S->flights.size();) {
            Flight &f = S->flights[i];
            hipError_t q = f.launch_status == E2E_OK ? hipEventQuery(f.ev) : hipSuccess;
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (f.launch_status == E2E_OK && q != hipSuccess) f.launch_status = hip_fail(q, "serve launch");
            S->stream_busy[f.stream] = false;
            done.push_back(f);
            S->flights.erase(S->flights.begin() + i);
        }
        if (!done.empty()) {
            lk.unlock();
            std::vector<std::pair<e2e_status, std::string>> res;
            for (Flight &f : done) {
                e2e_status st = f.launch_status;
                if (st == E2E_OK) {
                    std::lock_guard<std::mutex> g(ctx->mu);
                    Scratch *sc = scratch_for(ctx, S->streams[f.stream]);
                    st = sc ? take_err_word(sc, S->streams[f.stream]) : E2E_EDEVICE;
                }
                std::string msg = st != E2E_OK ? e2e_last_error() : "";
                float a = 0.f, b = 0.f;
                if (f.ev0 && f.ev && hipEventElapsedTime(&a, S->ref, f.ev0) == hipSuccess &&
                    hipEventElapsedTime(&b, S->ref, f.ev) == hipSuccess) {
                    for (SReq *r : f.reqs) {
                        r->st.t_gpu_start_us = 1e3 * (double)a;
                        r->st.t_gpu_end_us = 1e3 * (double)b;
                    }
                }
                for (SReq *r : f.reqs) {
                    if (st == E2E_OK && r->user_out) memcpy(r->user_out, r->out_stage, r->out_bytes);
                    release(r);
                    res.emplace_back(st, msg);
                }
                if (f.ev0) hipEventDestroy(f.ev0);
                if (f.ev) hipEventDestroy(f.ev);
            }
            lk.lock();
            size_t k = 0;
            for (Flight &f : done)
                for (SReq *r : f.reqs) {
                    finish(ctx, S, r, res[k].first, res[k].second);
                    ++k;
                }
            S->cv_done.notify_all();
        }

        // admit and launch while a stream, slots and memory are free
        for (;;) {
            if (S->queue.empty()) break;
            int si = -1;
            for (size_t k = 0; k < S->streams.size(); ++k)
                if (!S->stream_busy[k]) { si = (int)k; break; }
            if (si < 0) break;
            uint64_t avail;
            {
                std::lock_guard<std::mutex> g(ctx->mu);
                avail = ctx->budget > ctx->used ? ctx->budget - ctx->used : 0;
            }
            std::vector<SReq *> group = take_group(ctx, S, avail);
            if (group.empty()) break;
            S->stream_busy[si] = true;
            Flight f;
            f.stream = si;
            f.reqs = group;
            hipStream_t s = S->streams[si];
            lk.unlock();
            std::vector<e2e_render_req> rr;
            for (SReq *q : group) {
                e2e_status st = stage_in(q, s);
                if (st != E2E_OK) f.launch_status = st;
                rr.push_back(q->r);
            }
            const double tl = now_us(ctx);
            for (SReq *q : group) {
                q->st.t_launch_us = tl;
                q->st.batch_size = (int32_t)group.size();
            }
            if (f.launch_status == E2E_OK) {
                hipEventCreate(&f.ev0);
                hipEventRecord(f.ev0, s);
                f.launch_status = run_frames(ctx, rr.data(), (int)rr.size(), true);
            }
            if (f.launch_status == E2E_OK) {
                // host frames come back on the same stream, before the event
                for (SReq *q : group) {
                    if (!q->user_out) continue;
                    hipError_t e = hipMemcpyAsync(q->out_stage, q->r.out, q->out_bytes,
                                                  hipMemcpyDeviceToHost, s);
                    if (e != hipSuccess) f.launch_status = hip_fail(e, "serve download");
                }
                hipEventCreate(&f.ev);
                hipEventRecord(f.ev, s);
            }
            lk.lock();
            S->flights.push_back(f);
        }

        if (S->stop && S->queue.empty() && S->flights.empty()) break;
        if (S->flights.empty())
            S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
        else
            S->cv.wait_for(lk, std::chrono::microseconds(100));
    }
}

extern "C" e2e_status e2e_serve_start(e2e_ctx *ctx, const e2e_serve_config *cfg)
{
    if (!ctx) return fail(E2E_EINVAL, "NULL context");
    std::lock_guard<std::mutex> g(ctx->srv_mu);
    if (ctx->srv) return E2E_OK;
    hipSetDevice(ctx->dev);
    auto S = std::make_unique<Server>();
    e2e_serve_config c{8, 256, 2, 8};
    if (cfg) {
        if (cfg->max_inflight < 1 || cfg->max_queue < 1 || cfg->n_streams < 1 ||
            cfg->n_streams > 8 || cfg->max_batch < 1)
            return fail(E2E_EINVAL, "serve config out of range");
        c = *cfg;
    }
    S->cfg = c;
    for (int i = 0; i < c.n_streams; ++i) {
        hipStream_t s;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto q : S->streams) hipStreamDestroy(q);
            return hip_fail(e, "serve stream");
        }
        S->streams.push_back(s);
        S->stream_busy.push_back(false);
    }
    hipError_t e = hipEventCreate(&S->ref);
    if (e == hipSuccess) e = hipEventRecord(S->ref, S->streams[0]);
    if (e != hipSuccess) {
        for (auto q : S->streams) hipStreamDestroy(q);
        return hip_fail(e, "serve reference event");
    }
    Server *raw = S.release();
    ctx->srv = raw;
    raw->th = std::thread(loop, ctx, raw);
    return E2E_OK;
}

extern "C" e2e_status e2e_serve_submit(e2e_ctx *ctx, const e2e_render_req *req, e2e_ticket *out)
{
    if (!ctx || !req || !out) return fail(E2E_EINVAL, "e2e_serve_submit: NULL argument");
    if (!ctx->srv) {
        e2e_status st = e2e_serve_start(ctx, nullptr);
        if (st != E2E_OK) return st;
    }
    Server *S = ctx->srv;
    auto *q = new SReq();
    q->r = *req;
    q->st.t_submit_us = now_us(ctx);
    hipSetDevice(ctx->dev);
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        e2e_status st = validate_req(ctx, req, &q->fmt, &q->psf);
        if (st != E2E_OK) {
            delete q;
            return st;
        }
        int ns = q->fmt->nslots;
        size_t esz = req->spectrum_dtype == E2E_F64 ? 8 : 4;
        q->specs.assign(req->spectra, req->spectra + ns);
        q->spec_bytes.assign(ns, 0);
        q->host_stage.assign(ns, nullptr);
        for (auto &T : q->fmt->host)
            q->spec_bytes[T.slot] = std::max(q->spec_bytes[T.slot], (size_t)T.n * esz);
        q->out_bytes = (size_t)q->fmt->nx * q->fmt->ny * (req->out_dtype == E2E_F64 ? 8 : 4);
        uint64_t fp = q->out_bytes;
        if (!req->spectra_on_device)
            for (size_t b : q->spec_bytes) fp += b;
        int tw = q->psf->kind == E2E_PSF_TABLE ? table_tw(q->psf->kw) : kSepTile;
        fp += (uint64_t)((q->fmt->nx + tw - 1) / tw) * q->fmt->ntr * sizeof(SegDev) +
              (uint64_t)q->fmt->ntr * sizeof(TraceFrameDev);
        q->footprint = fp;
        uint64_t avail = ctx->budget > ctx->used ? ctx->budget - ctx->used : 0;
        if (fp > avail) {
            delete q;
            return fail(E2E_ENOMEM, "request footprint %llu B exceeds the %llu B available",
                        (unsigned long long)fp, (unsigned long long)avail);
        }
        q->fmt->refs++;
        q->psf->refs++;
    }
    q->st.footprint_bytes = q->footprint;
    if (!req->out_on_device) q->user_out = req->out;
    if (!req->spectra_on_device) {
        for (size_t i = 0; i < q->specs.size(); ++i) {
            if (q->spec_bytes[i] == 0) continue;
            void *h = nullptr;
            if (hipHostMalloc(&h, q->spec_bytes[i]) != hipSuccess) {
                for (void *p : q->host_stage) hipHostFree(p);
                std::lock_guard<std::mutex> g(ctx->mu);
                q->fmt->refs--;
                q->psf->refs--;
                delete q;
                return fail(E2E_ENOMEM, "pinned staging for spectra failed");
            }
            memcpy(h, req->spectra[i], q->spec_bytes[i]);
            q->host_stage[i] = h;
        }
    }
    std::lock_guard<std::mutex> lk(S->m);
    if ((int)S->queue.size() >= S->cfg.max_queue) {
        for (void *p : q->host_stage) hipHostFree(p);
        std::lock_guard<std::mutex> g(ctx->mu);
        q->fmt->refs--;
        q->psf->refs--;
        delete q;
        return fail(E2E_EAGAIN, "serve queue full (%d)", S->cfg.max_queue);
    }
    q->id = S->next++;
    S->all[q->id] = q;
    S->queue.push_back(q);
    *out = q->id;
    S->cv.notify_all();
    return E2E_OK;
}

extern "C" e2e_status e2e_serve_poll(e2e_ctx *ctx, e2e_ticket t, int32_t timeout_ms,
                                     e2e_render_stats *stats)
{
    if (!ctx) return fail(E2E_EINVAL, "NULL context");
    if (!ctx->srv) return fail(E2E_ENOTFOUND, "ticket %llu not found", (unsigned long long)t);
    Server *S = ctx->srv;
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->all.find(t);
    if (it == S->all.end()) return fail(E2E_ENOTFOUND, "ticket %llu not found", (unsigned long long)t);
    SReq *q = it->second;
    if (!q->done && timeout_ms != 0) {
        if (timeout_ms < 0)
            S->cv_done.wait(lk, [&] { return q->done; });
        else
            S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return q->done; });
    }
    if (!q->done) return E2E_PENDING;
    if (stats) *stats = q->st;
    e2e_status st = q->status;
    std::string msg = q->msg;
    S->all.erase(it);
    delete q;
    if (st != E2E_OK) return fail(st, "%s", msg.c_str());
    return E2E_OK;
}

extern "C" e2e_status e2e_serve_stop(e2e_ctx *ctx)
{
    if (!ctx) return fail(E2E_EINVAL, "NULL context");
    std::unique_ptr<Server> S;
    {
        std::lock_guard<std::mutex> g(ctx->srv_mu);
        if (!ctx->srv) return E2E_OK;
        {
            std::lock_guard<std::mutex> lk(ctx->srv->m);
            ctx->srv->stop = true;
            ctx->srv->cv.notify_all();
        }
        if (ctx->srv->th.joinable()) ctx->srv->th.join();
        S.reset(ctx->srv);
        ctx->srv = nullptr;
    }
    for (auto &kv : S->all) delete kv.second;
    for (auto s : S->streams) {
        hipStreamSynchronize(s);
        hipStreamDestroy(s);
    }
    if (S->ref) hipEventDestroy(S->ref);
    return E2E_OK;
}
