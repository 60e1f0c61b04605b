// Internal declarations of the MI355X echellogram renderer (device tables,
// per-frame launch parameters, launch wrappers).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/e2e.h"

namespace e2e {

constexpr int kNCoef = 8;        // polynomial coefficients stored per axis
constexpr int kOS = 4;           // PSF table cells per pixel on the GPU path
constexpr int kTableThreads = 256;
constexpr int kTableTH = 32;     // table-path tile height (rows)
constexpr int kTableChunk = 8;   // default run of table-path tiles one workgroup walks
constexpr int kSepTile = 16;     // VALU separable / erf tile edge
constexpr int kMfmaTW = 64;      // MFMA separable tile width (x)
constexpr int kMfmaTH = 32;      // MFMA separable tile height (y)
constexpr int kMaxTileTraces = 512;
constexpr int kSfiMaxR = 16;     // SFI: quadrature node pairs (32 nodes)
constexpr int kSfiMaxH = 7;      // SFI: footprint half width
constexpr int kSfiTW = 64;       // SFI tile width (x)
constexpr int kSfiTH = 32;       // SFI tile height (y)
constexpr int kTapShift = 8;     // table taps are stored times 2^8 in their fp16 fragments

// Table path: the stencil of one node layer over a band of 4 deposit rows is
// a product with k = (slot offset s, band row r), s padded to a multiple of 8
// so k runs in steps of 32 (v_mfma_f32_16x16x32_f16).
constexpr __host__ __device__ int table_dd(int kw) { return (kw + kOS - 2) / kOS + 1; }
constexpr __host__ __device__ int table_slots_padded(int kw) { return (kw + kOS - 1 + 7) / 8 * 8; }
constexpr __host__ __device__ int table_ksteps(int kw) { return table_slots_padded(kw) / 8; }
// halfs of one row (one output row j of one band phase) of a tap fragment table:
// [slot offset][band row]
constexpr __host__ __device__ int table_frag_row(int kw) { return 4 * table_slots_padded(kw); }
// rows per band phase: output rows 0 .. dd (dd + 1 of them), then a zero row
constexpr __host__ __device__ int table_frag_rows(int kw) { return table_dd(kw) + 2; }
// halfs of one node's fragments: [hi, lo][band phase][row][slot offset][band row]
constexpr __host__ __device__ int table_frag_node(int kw)
{
    return 2 * 4 * table_frag_rows(kw) * table_frag_row(kw);
}
// slots of one band row in LDS: 64 pixel columns x 4, plus the widest read
constexpr __host__ __device__ int table_band_slots(int kw) { return 4 * 64 + 8 * table_ksteps(kw); }

// Device-resident record of one trace (spectral-format database row).
struct TraceDev {
    double cx[kNCoef];
    double cy[kNCoef];
    double lmin, lmax;
    double thr;
    double y2max;      // bound on |d2y/dt2| over the trace (planner margin)
    int32_t n;
    int32_t degx, degy;
    int32_t slot;
};

// Planner output per (tile column, trace): the samples that can reach the
// column, the tile rows they can reach and the node cells they fall in.
struct SegDev {
    int32_t k0, k1;          // sample range [k0, k1)
    int16_t ty0, ty1;        // tile rows reached (inclusive); ty0 > ty1: none
    int8_t cx0, cx1, cy0, cy1;  // node cells spanned (table path)
};

static_assert(sizeof(SegDev) == 16, "SegDev is read as one 16-byte word");

// Per-frame constants of one trace, written by the planner: the affine
// wavelength map t = t0 + k dt of its samples (Doppler shift included), its
// flux scale (throughput x exposure) and its spectrum.
struct TraceFrameDev {
    double t0, dt, scale;
    const void *spec;
};
static_assert(sizeof(TraceFrameDev) == 32, "TraceFrameDev is 32 bytes");

// Everything one frame's kernels need; lives in device memory.
struct FrameDev {
    const TraceDev *tr;
    const void *const *spec;  // device array of device pointers, per slot
    void *out;
    const void *tfrag;        // table path: fp16 tap fragments per node (table_frag_node)
    const float *sxy;         // separable / SFI: [gy][gx][2]
    const float *sfq;         // SFI: quadrature nodes [R][3] (a_p, h_p, w_p)
    SegDev *segs;             // [ntx][ntr]
    TraceFrameDev *tf;        // [ntr]
    double beta, flux_scale;
    double sigma;             // erf
    double gsx, gsy;          // (g-1)/(n-1) node-grid scale
    int32_t ntr, nx, ny;
    int32_t psf_kind, H, gx, gy, kw;
    int32_t spec_f64, out_f64;
    int32_t precision;
    int32_t tw, th, ntx, nty;
    int32_t chunk;            // table path: tiles per work unit
    int32_t poisson;
    uint32_t frame_index;
    uint64_t seed;
    int32_t sfi_R, sfi_S, sfi_shape;  // SFI: node pairs, sub-pixels, fiber shape
};

// Device error word bits.
enum : int {
    kErrTileTraces = 1,   // more traces reach a tile than the list holds
    kErrRowWindow = 2,    // a column's rows left its 4-row window
    kErrSearch = 4,       // a column boundary search did not converge
    kErrCells = 8,        // a trace spans more node cells than supported
};

// Tile geometry of each path.
inline int table_tw(int kw) { return (kTableThreads - kw) / kOS; }
// Work units of the table path: runs of `chunk` tiles down one column.
inline int table_units(int ntx, int nty, int chunk) { return ntx * ((nty + chunk - 1) / chunk); }

// Compile-time choices of a render launch (shared by every frame of it).
struct KernelCfg {
    int kw;             // table cells per kernel side (table path)
    int degx, degy;     // largest polynomial degrees among the traces
    int spec_f64;       // spectra element type
    int plain_tiles;    // plain launch: tiles of frame 0 (one block each)
    int precision;      // E2E_PREC_*
    int mfma_tiles;     // separable MFMA path: tiles of frame 0
    int resident;       // persistent launches: workgroups per CU (0 = path default)
};

// Launch wrappers (each .hip file owns its kernels).  work == nullptr
// selects the plain launch over frame 0; otherwise a persistent launch pulls
// (frame, tile) items through *counter.
hipError_t launch_plan(const FrameDev *frames_dev, const FrameDev *frames_host, int n_frames,
                       int *err, hipStream_t s);
hipError_t launch_table(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                        int n_work, int *counter, int *err, hipStream_t s);
hipError_t launch_sep(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                      int n_work, int *counter, int *err, hipStream_t s);
hipError_t launch_sfi(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                      int n_work, int *counter, int *err, hipStream_t s);
hipError_t launch_sep_mfma(const FrameDev *frames_dev, const KernelCfg &cfg, const int2 *work,
                           int n_work, int *counter, int *err, hipStream_t s);
hipError_t launch_noise(void *frame, int f64, int64_t n, uint64_t seed, uint32_t frame_index,
                        hipStream_t s);
hipError_t launch_noise_frames(const FrameDev *frames_dev, const FrameDev *frames_host,
                               int n_frames, hipStream_t s);
hipError_t launch_philox(uint64_t seed, uint32_t frame, uint64_t pixel0, int64_t n,
                         uint32_t blocks, uint32_t *out, hipStream_t s);
hipError_t launch_fill_i32(int *p, int n, int v, hipStream_t s);
// Writes one frame record and up to kParamSlots spectrum pointers into device
// memory from a kernel argument (no host staging buffer).
constexpr int kParamSlots = 64;
struct FrameParams {
    FrameDev f;
    int32_t nslots;
    const void *spec[kParamSlots];
};
hipError_t launch_put_params(const FrameParams &p, FrameDev *frame_dst, const void **spec_dst,
                             hipStream_t s);
hipError_t launch_detector(const void *frame, int f64, const float *prnu, int nx, int ny,
                           double dark, int shot, const double *xtalk, double ron, double gain,
                           double bias, int bits, uint64_t seed, uint32_t fidx, uint16_t *adu,
                           hipStream_t s);

// XCD-aware block order: blocks are dispatched round robin over the 8 XCDs,
// so block b runs on XCD b % 8.  Give each XCD a contiguous run of tiles
// (neighbouring tiles share spectrum halos in that XCD's L2).  Bijective on
// [0, nblocks).
__host__ __device__ inline int xcd_remap(int b, int nblocks)
{
    const int nx = 8;
    int q = nblocks / nx, r = nblocks % nx;
    int x = b % nx;
    int start = x * q + (x < r ? x : r);
    return start + b / nx;
}

}  // namespace e2e
