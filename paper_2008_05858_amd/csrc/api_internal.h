// Host-side state behind the C ABI: context, resident tables, per-stream
// scratch, timing records, serve-loop hooks.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "e2e_impl.h"

namespace e2e {

struct FormatRes {
    int nx = 0, ny = 0, ntr = 0, nslots = 0, degx = 0, degy = 0;
    std::vector<TraceDev> host;
    TraceDev *dev = nullptr;
    size_t bytes = 0;
    int refs = 0;  // served requests holding it
};

struct PsfRes {
    int kind = 0;
    double sigma = 0;
    int H = 0, gx = 1, gy = 1, kw = 0, kh = 0, os = 0;
    uint16_t *tfrag = nullptr;  // table taps as fp16 hi/lo product fragments
    float *sxy = nullptr;   // separable sigma grid
    float *sfq = nullptr;   // SFI: quadrature nodes [R][3]
    int sfi_R = 0, sfi_S = 0, sfi_shape = 0;
    double rho = 0;
    size_t bytes = 0;
    int refs = 0;
};

struct GraphRec {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Device buffers reused by consecutive calls on one stream.
struct Scratch {
    FrameDev *frames_dev = nullptr;
    size_t frames_cap = 0;
    SegDev *segs = nullptr;
    size_t segs_cap = 0;
    int2 *work = nullptr;
    size_t work_cap = 0;
    const void **specptrs = nullptr;
    size_t specptrs_cap = 0;
    int *err = nullptr;
    int *counter = nullptr;
    int *err_host = nullptr;
    // pinned staging of the parameter uploads, reusable once `staged` fired
    void *stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t staged = nullptr;
    bool staged_valid = false;
    std::vector<void *> temps;   // device temporaries of the last call
    std::vector<FrameDev> h_frames;
    std::vector<void *> h_specptrs;
    std::vector<int2> h_work;
    std::map<std::string, GraphRec> graphs;
};

// Device memory of the allocation-free render (e2e_render_noalloc): the
// planner output, frame record, spectrum pointers, error word and queue
// counter of one frame, carved from a file-scope device array whose address
// e2e_create looks up once for its device.
constexpr size_t kNoAllocBytes = 16u << 20;
constexpr int kNoAllocSlots = 64;   // spectrum slots the parameter kernel carries
struct NoAlloc {
    char *base = nullptr;           // device address of the array on ctx->dev
    int err_host = 0;               // host copy of the error word
};

struct ProfRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};

struct Server;

}  // namespace e2e

namespace e2e {
// Launch choices of one workload shape, set by e2e_autotune.
struct TuneRec {
    int chunk = kTableChunk;  // table path: tiles per work unit
    int resident = 0;         // persistent launches: workgroups per CU (0 = default)
};
}  // namespace e2e

struct e2e_ctx {
    int dev = 0;
    uint64_t budget = 0;
    uint64_t used = 0;
    std::mutex mu;
    std::map<uint64_t, e2e::FormatRes *> fmts;
    std::map<uint64_t, e2e::PsfRes *> psfs;
    uint64_t next_id = 1;
    hipStream_t stream = nullptr;
    std::map<hipStream_t, e2e::Scratch *> scratch;
    bool prof = false;
    bool graphs = true;           // batches replay captured HIP graphs
    std::vector<e2e::ProfRec> prof_pending;
    std::map<std::string, std::pair<int64_t, double>> prof_acc;
    std::chrono::steady_clock::time_point t0;
    e2e::Server *srv = nullptr;  // owned by serve.cpp
    e2e::NoAlloc noalloc;        // the allocation-free render's device array
    std::map<std::string, e2e::TuneRec> tune;  // by workload shape (guarded by mu)
    std::mutex srv_mu;
};

namespace e2e {

e2e_status fail(e2e_status code, const char *fmt, ...);
e2e_status hip_fail(hipError_t e, const char *what);
double now_us(const e2e_ctx *ctx);
Scratch *scratch_for(e2e_ctx *ctx, hipStream_t s);
e2e_status validate_req(e2e_ctx *ctx, const e2e_render_req *r, FormatRes **pf, PsfRes **pp);
// Render n frames (batch: one persistent launch).  Caller must not hold mu.
e2e_status run_frames(e2e_ctx *ctx, const e2e_render_req *reqs, int n, bool batch,
                      bool noalloc = false);
e2e_status check_err_word(int w);
e2e_status take_err_word(Scratch *sc, hipStream_t s);
std::string tune_key(const FormatRes *f, const PsfRes *p, int precision, int spectrum_dtype);
void prof_begin(e2e_ctx *ctx, hipStream_t s, const char *name);
void prof_end(e2e_ctx *ctx, hipStream_t s);
void serve_shutdown(e2e_ctx *ctx);

}  // namespace e2e
