// internal.hpp -- structures shared by the host planner/executor and the
// gfx950 kernels of liboocs. Not part of the public ABI (include/oocs.h).
#pragma once
#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime.h>

namespace oocs {

// A ring of FP32 planes in device memory. Plane z lives in slot z mod W.
// A dense field is the special case W >= nz (no wrap-around).
struct Ring {
    float* base;
    int64_t W;     // planes in the ring
    int64_t ld_z;  // elements from one plane to the next
};

// Planes and ring sizes stay below 2^31 (the planner caps grid dimensions at
// 2^20), so the slot is a 32-bit remainder.
__host__ __device__ inline float* ring_plane(const Ring& r, int64_t z)
{
    return r.base + (int64_t)((uint32_t)z % (uint32_t)r.W) * r.ld_z;
}

enum JobKind : int32_t {
    JOB_HEAT = 1,    // one heat time level over planes [z0, z1)
    JOB_WAVE = 2,    // one wave time level over planes [z0, z1)
    JOB_DECODE = 3,  // staging (compressed words) -> ring planes
    JOB_ENCODE = 4,  // ring planes -> staging (compressed words)
    JOB_COPY_IN = 5, // staging (raw planes) -> ring planes
    JOB_COPY_OUT = 6,// ring planes -> staging (raw planes)
    JOB_FETCH = 7,   // host store bytes -> staging slot
    JOB_STORE = 8,   // staging slot -> host store bytes
    JOB_HEAT_TB = 9  // `rate` heat steps over planes [z0, z1) in one temporally blocked pass
};

// One job of a fused launch. For stencil jobs src = level l-1, src2 = level
// l-2 (wave), ro = read-only field ring (wave), dst = level l. For codec
// and copy jobs `ring` is the level ring and `stage` the staging slot.
struct Job {
    int32_t kind;
    int32_t z0, z1;
    int32_t rate;      // codec jobs
    int32_t has_src;   // wave: add the source amplitude at the source cell
    float amp;         // the amplitude when LaunchParams::src_table is null
    int32_t src_off;   // else the amplitude is src_table[*step_ctr + src_off]
    int32_t wg_count;  // workgroups of this job
    int32_t mid;       // decode jobs: mid-point reconstruction of the digits the budget cut off
    int32_t f64;       // FP64 planes (rings hold doubles; codec jobs use the FP64 format)
    Ring src, src2, ro, dst;  // stencil jobs (dst doubles as `ring` for codec/copy jobs)
    void* stage;              // codec/copy/transfer jobs
    void* host;               // transfer jobs: device address of the host-store bytes
    int64_t bytes;            // transfer jobs: bytes to move (a multiple of 8)
};

constexpr int kMaxJobs = 24;
constexpr int kBlockThreads = 256;  // every job runs 256-thread workgroups (4 waves)
constexpr int kZChunk = 16;         // planes one stencil thread marches
constexpr int kHeatTileX = 256;     // heat xy tile: 4 waves, each a 256-wide row (4 x per lane)
constexpr int kHeatTileY = 4;
constexpr int kTbTileY = 16;        // temporally blocked heat: 64 x 16 cell tiles (k-cell halo included)
constexpr int kWaveTileY = 16;      // wave: 64 x 16 cell tiles, planes staged through LDS with a 4-cell halo
constexpr int kMaxTbSteps = 4;

struct LaunchParams {
    int32_t nx, ny, nz;
    float alpha;
    int32_t src_x, src_y, src_z;
    int32_t njobs;
    const float* src_table;    // wave source amplitudes of the current run chunk (device), or null
    const int32_t* step_ctr;   // device counter: steps done in the chunk before this residency
    // Workgroups of the jobs before the codec jobs, and of the codec jobs:
    // with both present, workgroup b of the launch runs the (b*ncodec /
    // (nfirst+ncodec))-th codec workgroup where that index steps up, so the
    // codec workgroups are spread evenly among the others (0: plain order).
    int32_t nfirst, ncodec;
    int32_t wg_begin[kMaxJobs + 1];  // prefix sums of wg_count
    Job jobs[kMaxJobs];
};

// Workgroups a job needs (host side).
int32_t job_workgroups(const Job& j, int nx, int ny);

// True for the decode and encode jobs.
bool is_codec_job(int kind);

// True for the host-link transfer jobs (FETCH / STORE).
inline bool is_xfer_job(int kind) { return kind == JOB_FETCH || kind == JOB_STORE; }

// Launch the fused kernel for the jobs in p (reorders p.jobs so that codec
// jobs come first; fills p.wg_begin).
hipError_t launch_jobs(LaunchParams& p, hipStream_t stream);

// The same launch as a kernel node of graph g after `deps` (node left in *node;
// no node and hipSuccess if there is no work).
hipError_t add_jobs_node(LaunchParams& p, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps, hipGraphNode_t* node);

// FP64 jobs (Job::f64; every job of the launch): the FP64 pipeline kernel,
// which runs wave levels, FP64-format codec jobs and raw copies. launch_jobs
// and add_jobs_node hand such launches to these.
// FP64 jobs: up to two kernels per tick (the stencil and copy jobs, then the
// codec jobs), returned in launch order; the count is the return value.
int prepare_jobs_f64(LaunchParams& p, const void* func[2], unsigned grid[2], size_t lds[2]);
hipError_t launch_jobs_f64(LaunchParams& p, hipStream_t stream);

// Device step counter of the wave source table: set to `value` (add = false)
// or advanced by `value` (add = true); as a launch or as a graph node.
hipError_t launch_step_ctr(int32_t* ctr, bool add, int32_t value, hipStream_t stream);
hipError_t add_step_ctr_node(int32_t* ctr, bool add, int32_t value, hipGraph_t g, const hipGraphNode_t* deps,
                             size_t ndeps, hipGraphNode_t* node);

// Standalone codec launches on dense (non-ring) fields; mid: mid-point
// reconstruction when decoding.
hipError_t launch_codec_field(bool encode, const float* in_f, float* out_f, const uint64_t* in_w, uint64_t* out_w,
                              int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                              hipStream_t stream, bool mid = false);

// Exchange the contents of two device arrays of n floats.
hipError_t launch_swap(float* a, float* b, int64_t n, hipStream_t stream);

// Adjoint helpers (in-core fields, nx*ny*nz floats, x fastest).
// lam(t) and w . lam(t) from lam(t+1), w . lam(t+1), lam(t+2); grad += lam(t+1) . L p(t).
hipError_t launch_adjoint_step(const float* l1, const float* wl1, const float* l2, const float* w, const float* p,
                               float* l0, float* wl0, float* grad, int64_t nx, int64_t ny, int64_t nz,
                               hipStream_t stream);
// Receivers outside [0, n) are skipped.
hipError_t launch_rcv_sample(const float* p, const int64_t* rcv, int nr, const float* obs, float* res, int64_t n,
                             hipStream_t s);
// lam += res at the receivers, and wl = w * lam at the cells touched.
hipError_t launch_rcv_inject(float* lam, float* wl, const float* w, const int64_t* rcv, int nr, const float* res,
                             int64_t n, hipStream_t s);
hipError_t launch_v_to_w(const float* v, float c, float* w, int64_t n, hipStream_t s);
hipError_t launch_grad_w_to_v(const float* gw, const float* v, float c, float* gv, int64_t n, hipStream_t s);
hipError_t launch_fill(float* x, float value, int64_t n, hipStream_t s);

// ---- batched heat domains ---------------------------------------------------
// Tile configurations the batch autotuner chooses from (TX x TY threads,
// ZC planes per thread).
struct TileCfg {
    int tx, ty, zc;  // threads per tile in x and y (k = 1) or tile size in cells (k > 1); planes per chunk
    int k;           // steps per launch (temporal-blocking depth)
};
// k = 1: threads per tile (tx * ty = 256) and planes marched per thread.
// k > 1: a 64 x ty cell tile (halo k cells on each side included) advanced k
// steps per launch over z chunks of zc planes (heat_tb). Three or more
// candidates per depth. (Taller tiles at k = 4 raise the register count of
// every blocked kernel: 20 rows took them from 67 to 82 VGPRs.)
constexpr int kNumTileCfgs = 12;
inline constexpr TileCfg kTileCfgs[kNumTileCfgs] = {
    {64, 4, 16, 1},  {64, 4, 32, 1},   {64, 4, 64, 1},  {32, 8, 16, 1},   {128, 2, 16, 1},
    {64, 4, 8, 1},   {64, 16, 64, 2},  {64, 16, 128, 2}, {64, 16, 32, 2}, {64, 16, 64, 4},
    {64, 16, 32, 4}, {64, 16, 128, 4}};

struct BatchDomain {   // one entry of the device work-list table
    float* a;          // field at even steps (the caller's u)
    float* b;          // field at odd steps (the caller's scratch)
    int32_t nx, ny, nz;
    int32_t cfg;         // index into kTileCfgs
    int32_t wg_begin;    // first workgroup of this domain in a launch
    int32_t item_begin;  // first item of this domain in a group of a persistent launch
};

// Workgroups one domain needs with tile configuration cfg.
int32_t batch_domain_workgroups(int nx, int ny, int nz, int cfg);

// Dynamic LDS bytes a tile configuration needs (0 for k = 1).
size_t tile_cfg_lds(int cfg);

// The persistent batched launch: one kernel runs groups of k steps of every
// domain, as items (domain, up to kBatchTilesPerItem consecutive tiles,
// group) taken in order from a device queue; an item of group g of domain d
// starts once every tile of group g-1 of d has finished (a per-domain count
// of finished tiles). A launch holds the groups of one work list; copy items
// after its last group move a result left in the scratch buffers back to u
// (depth-1 launches only). Each item costs a device-scope acquire and
// release (on gfx950 an L2 invalidate and write-back, since the dies' L2s
// are not coherent with each other), so items take several tiles.
struct BatchPersistArgs {
    const BatchDomain* tab;     // work list of this launch's groups
    const int32_t* copy_begin;  // nd + 1 prefix sums of each domain's copy items
    uint32_t* sync;             // [0] queue head, [1] workgroups exited, [2] status, [3] unused, [4 + d] tiles done
    int32_t nd;
    int32_t groups;             // groups of this launch
    int32_t parity0;            // parity of its first group (0: reads a, writes b)
    int32_t total;              // tiles of one group
    int32_t items;              // items of one group
    int32_t copy_items;
    int32_t force_wait;         // test hook: no wait is ever satisfied
    int64_t spin_limit;         // polls before a wait gives up and sets the status
    float alpha;
};
constexpr int kBatchSyncWords = 4;         // words of the sync area before the per-domain counts
constexpr int kBatchCopyFloats = 1 << 16;  // floats one copy item moves
// Tiles of one item: 64 heat cubes of sides 64..384 at depth 4 ran 186
// GCell/s with one tile per item, 508 / 611 / 680 / 360 with 8 / 16 / 32 /
// 128 (beyond 32 the items of the largest domain, done one after another
// by a workgroup, make each group's critical path the limit).
constexpr int kBatchTilesPerItem = 32;
// tb: the list's tiles are temporally blocked (no copy items then).
hipError_t launch_batch_persistent(const BatchPersistArgs& a, bool tb, int grid, size_t lds, hipStream_t stream);
hipError_t add_batch_persistent_node(const BatchPersistArgs& a, bool tb, int grid, size_t lds, hipGraph_t g,
                                     const hipGraphNode_t* deps, size_t ndeps, hipGraphNode_t* node);
// Workgroups of the persistent launch: those that fit the device at once.
hipError_t batch_persistent_grid(bool tb, size_t lds, int* grid);
// Zero n words of device memory (a fill kernel, so that it may be captured).
hipError_t launch_zero_words(uint32_t* p, int64_t n, hipStream_t stream);

// One step of every domain: parity 0 reads a and writes b, 1 the reverse.
hipError_t launch_batch_step(const BatchDomain* d_table, int nd, int32_t total_wg, size_t lds, int parity,
                             float alpha, hipStream_t stream);
hipError_t add_batch_step_node(const BatchDomain* d_table, int nd, int32_t total_wg, size_t lds, int parity,
                               float alpha, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                               hipGraphNode_t* node);
// One launch (the configuration's k steps) of one dense domain with tile
// configuration cfg (tuning and the per-domain baseline).
hipError_t launch_heat_dense(const float* src, float* dst, int nx, int ny, int nz, float alpha, int cfg,
                             hipStream_t stream);

// FP64 format (codec64.hip): whole fields, and per-block stages.
hipError_t launch_codec64_field(bool encode, const double* in_f, double* out_f, const uint64_t* in_w, uint64_t* out_w,
                                int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                                hipStream_t stream);
hipError_t launch_codec64_stages(bool encode, const double* blocks, const uint64_t* in_w, int64_t nblocks, int rate,
                                 int32_t* emax, int64_t* q, int64_t* t, uint64_t* u, uint64_t* planes,
                                 uint64_t* out_w, int32_t* bits, double* out, hipStream_t stream);
// One FP64 wave step on a dense field; p(n+1) is written over pm.
hipError_t launch_wave_f64(const double* p, double* pm, const double* w, int64_t nx, int64_t ny, int64_t nz,
                           int64_t src_cell, double amp, hipStream_t stream);

struct EncStages {
    int32_t* emax; int32_t* q; int32_t* t; uint32_t* u; uint64_t* planes; uint64_t* words; int32_t* bits;
};
struct DecStages {
    int32_t* emax; uint64_t* planes; uint32_t* u; int32_t* q; float* out;
};
hipError_t launch_encode_stages(const float* blocks, int64_t nblocks, int rate, EncStages s, hipStream_t stream);
hipError_t launch_decode_stages(const uint64_t* words, int64_t nblocks, int rate, bool mid, DecStages s,
                                hipStream_t stream);

}  // namespace oocs
