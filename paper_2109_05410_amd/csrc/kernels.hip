// kernels.hip -- the gfx950 kernels of liboocs and their host launchers.
//
// The out-of-core pipeline issues one launch per tick. A tick's jobs (decode
// of the next input group, one z-range of every time level, encode of the
// finished output group) are independent by construction of the schedule,
// so they share one launch: the workgroup index selects the job and the
// job's own workgroup. All jobs use 256-thread workgroups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adjoint_dev.hpp"
#include "codec_dev.hpp"
#include "internal.hpp"
#include "stencil_dev.hpp"

namespace oocs {

static_assert(sizeof(LaunchParams) <= 4096, "kernel arguments must stay within 4 KiB");

constexpr int kWavesPerWG = kBlockThreads / 64;
constexpr int kCopyFloat4PerThread = 4;
constexpr int kHeatBatch = 4;       // planes whose loads a heat lane issues together (shared kernels)
constexpr int kHeatBatchAlone = 8;  // the same in launches of heat levels only (more registers)

extern __shared__ uint64_t dyn_lds[];  // codec jobs: 64 * rate words per wave

// ---------------------------------------------------------------------------
// Codec and copy jobs on ring planes
// ---------------------------------------------------------------------------

// Each wave codes 64 blocks consecutive in x (one lane per block). Staging
// slot of compressed words: the 4-plane layers of [z0, z1) in z order, each
// layer's blocks x fastest then y; rate words per block.
template <bool MID>
__device__ inline void codec_job(const Job& j, int nx, int ny, int wg, bool encode)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int nbx = nx >> 2, nby = ny >> 2;
    const int chunks = (nbx + 63) / 64;
    const int c = wg * kWavesPerWG + wave;  // wave chunk within the job
    const int layer = c / (chunks * nby);
    const int rem = c % (chunks * nby);
    const int by = rem / chunks;
    const int bx0 = (rem % chunks) * 64;
    const int z = j.z0 + 4 * layer;
    const bool wave_active = z < j.z1;
    const int nblocks = wave_active ? min(64, nbx - bx0) : 0;
    const bool active = lane < nblocks;
    const int rate = j.rate;
    uint64_t* lds = dyn_lds + (size_t)wave * 64 * rate;
    uint64_t* words = static_cast<uint64_t*>(j.stage) + (((int64_t)layer * nby + by) * nbx + bx0) * rate;
    const int64_t row0 = (int64_t)(4 * by) * nx + 4 * (bx0 + lane);
    float x[64];
    if (encode) {
        if (active) {
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const float* pl = ring_plane(j.dst, z + l) + row0;
#pragma unroll
                for (int jy = 0; jy < 4; ++jy) {
                    const float4 v = *reinterpret_cast<const float4*>(pl + (int64_t)jy * nx);
                    x[16 * l + 4 * jy] = v.x; x[16 * l + 4 * jy + 1] = v.y;
                    x[16 * l + 4 * jy + 2] = v.z; x[16 * l + 4 * jy + 3] = v.w;
                }
            }
            codec::encode_lane<false>(x, rate, lds + lane);
        }
        __syncthreads();
        if (nblocks > 0) codec::lds_to_words(lds, words, rate, nblocks, lane);
    } else {
        if (nblocks > 0) codec::words_to_lds(words, lds, rate, nblocks, lane);
        __syncthreads();
        if (active) {
            codec::decode_lane<false, MID>(lds + lane, rate, x);
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                float* pl = ring_plane(j.dst, z + l) + row0;
#pragma unroll
                for (int jy = 0; jy < 4; ++jy)
                    *reinterpret_cast<float4*>(pl + (int64_t)jy * nx) =
                        make_float4(x[16 * l + 4 * jy], x[16 * l + 4 * jy + 1], x[16 * l + 4 * jy + 2], x[16 * l + 4 * jy + 3]);
            }
        }
    }
}

// Raw planes: staging holds planes [z0, z1) back to back.
__device__ inline void copy_job(const Job& j, int nx, int ny, int wg, bool in)
{
    const int64_t plane = (int64_t)nx * ny;
    const int64_t n4 = plane / 4;                            // nx % 4 == 0
    const int64_t per_wg = (int64_t)kBlockThreads * kCopyFloat4PerThread;
    const int64_t wg_per_plane = (n4 + per_wg - 1) / per_wg;
    const int pz = (int)(wg / wg_per_plane);
    const int z = j.z0 + pz;
    if (z >= j.z1) return;
    const int64_t base = (wg % wg_per_plane) * per_wg;
    float4* r = reinterpret_cast<float4*>(ring_plane(j.dst, z));
    float4* s = reinterpret_cast<float4*>(static_cast<float*>(j.stage) + (int64_t)pz * plane);
#pragma unroll
    for (int k = 0; k < kCopyFloat4PerThread; ++k) {
        const int64_t e = base + (int64_t)k * kBlockThreads + threadIdx.x;
        if (e < n4) {
            if (in) r[e] = s[e]; else s[e] = r[e];
        }
    }
}

// Temporally blocked heat job: planes [z0, z1) of the output ring, j.rate steps.
__device__ inline void heat_tb_job(const Job& j, int nx, int ny, int nz, float alpha, int wg)
{
    float* lds = reinterpret_cast<float*>(dyn_lds);
    switch (j.rate) {
    case 1: stencil::heat_tb<kTbTileY, 1>(j.src, j.dst, nx, ny, nz, alpha, j.z0, j.z1, wg, lds); break;
    case 2: stencil::heat_tb<kTbTileY, 2>(j.src, j.dst, nx, ny, nz, alpha, j.z0, j.z1, wg, lds); break;
    case 3: stencil::heat_tb<kTbTileY, 3>(j.src, j.dst, nx, ny, nz, alpha, j.z0, j.z1, wg, lds); break;
    default: stencil::heat_tb<kTbTileY, 4>(j.src, j.dst, nx, ny, nz, alpha, j.z0, j.z1, wg, lds); break;
    }
}

static size_t heat_tb_lds(int steps) { return (size_t)steps * 2 * 2 * 4 * 64 * sizeof(float); }

// Host-link transfer: `bytes` (a multiple of 8) between the staging slot and
// the host store, 16 KiB per workgroup in 8-byte words. Every thread issues
// all its loads before its stores, so a workgroup keeps 16 KiB in flight
// across the link.
constexpr int kXferWordsPerThread = 8;
constexpr int64_t kXferBytesPerWG = (int64_t)kBlockThreads * kXferWordsPerThread * 8;

__device__ inline void xfer_job(const Job& j, int wg)
{
    const bool fetch = j.kind == JOB_FETCH;
    const uint2* src = static_cast<const uint2*>(fetch ? j.host : j.stage);
    uint2* dst = static_cast<uint2*>(fetch ? j.stage : j.host);
    const int64_t n = j.bytes / 8;
    const int64_t base = (int64_t)wg * (kXferBytesPerWG / 8) + threadIdx.x;
    uint2 v[kXferWordsPerThread];
#pragma unroll
    for (int k = 0; k < kXferWordsPerThread; ++k) {
        const int64_t e = base + (int64_t)k * kBlockThreads;
        if (e < n) v[k] = src[e];
    }
#pragma unroll
    for (int k = 0; k < kXferWordsPerThread; ++k) {
        const int64_t e = base + (int64_t)k * kBlockThreads;
        if (e < n) dst[e] = v[k];
    }
}

// All jobs of a tick share one launch. Transfer jobs come first in the job
// list, so that their link-bound workgroups start at once and run for the
// whole tick; codec jobs come next
// so that their workgroups, whose lanes each run a whole block's serial bit
// coding, are dispatched first and the short stencil workgroups fill the
// machine around them. MID: the decode jobs reconstruct cut-off digits at
// mid-points (a separate kernel: the extra registers would make the common
// kernel spill).
// Launch-order workgroup index: with codec jobs and other jobs present,
// block b takes the next codec workgroup wherever floor(b*C/T) steps up
// (T = all workgroups, C = codec ones), else the next other workgroup; the
// codec jobs come last in the job list, so codec workgroup c is nfirst + c.
__device__ inline int spread_wg(const LaunchParams& p)
{
    const int b = (int)blockIdx.x;
    if (p.ncodec == 0 || p.nfirst == 0) return b;
    const int64_t T = (int64_t)p.nfirst + p.ncodec;
    const int c0 = (int)((int64_t)b * p.ncodec / T), c1 = (int)((int64_t)(b + 1) * p.ncodec / T);
    return c1 > c0 ? p.nfirst + c0 : b - c0;
}

template <bool MID>
__global__ void __launch_bounds__(kBlockThreads) fused_kernel(LaunchParams p)
{
    const int wg = spread_wg(p);
    int jdx = 0;
    while (jdx + 1 < p.njobs && wg >= p.wg_begin[jdx + 1]) ++jdx;
    const Job& j = p.jobs[jdx];
    const int local = wg - p.wg_begin[jdx];
    switch (j.kind) {
    case JOB_DECODE: codec_job<MID>(j, p.nx, p.ny, local, false); break;
    case JOB_ENCODE: codec_job<false>(j, p.nx, p.ny, local, true); break;
    case JOB_HEAT: stencil::heat_level<kHeatBatch>(j, p.nx, p.ny, p.nz, p.alpha, local); break;
    case JOB_WAVE:
        stencil::wave_tile(j, p.nx, p.ny, p.nz, p.src_x, p.src_y, p.src_z, p.src_table, p.step_ctr, local,
                           reinterpret_cast<float*>(dyn_lds));
        break;
    case JOB_COPY_IN: copy_job(j, p.nx, p.ny, local, true); break;
    case JOB_COPY_OUT: copy_job(j, p.nx, p.ny, local, false); break;
    case JOB_FETCH:
    case JOB_STORE: xfer_job(j, local); break;
    case JOB_HEAT_TB: heat_tb_job(j, p.nx, p.ny, p.nz, p.alpha, local); break;
    default: break;
    }
}

// Launches without codec jobs use this kernel: a stencil thread needs about
// 40 VGPRs, and the codec path of the fused kernel would cap it at the
// codec's occupancy.
// Variants: kStencilWave can run wave jobs (launches holding one);
// kStencilPlain leaves the wave's register queues and staging out, so heat
// and copy launches keep their occupancy; kStencilHeat runs heat levels only
// (in-core steps, level-by-level ticks) with a deeper load batch.
constexpr int kStencilPlain = 0, kStencilWave = 1, kStencilHeat = 2;

template <int V>
__global__ void __launch_bounds__(kBlockThreads) stencil_kernel(LaunchParams p)
{
    const int wg = (int)blockIdx.x;
    int jdx = 0;
    while (jdx + 1 < p.njobs && wg >= p.wg_begin[jdx + 1]) ++jdx;
    const Job& j = p.jobs[jdx];
    const int local = wg - p.wg_begin[jdx];
    if (V == kStencilHeat) {
        stencil::heat_level<kHeatBatchAlone>(j, p.nx, p.ny, p.nz, p.alpha, local);
        return;
    }
    switch (j.kind) {
    case JOB_HEAT: stencil::heat_level<kHeatBatch>(j, p.nx, p.ny, p.nz, p.alpha, local); break;
    case JOB_WAVE:
        if (V == kStencilWave)
            stencil::wave_tile(j, p.nx, p.ny, p.nz, p.src_x, p.src_y, p.src_z, p.src_table, p.step_ctr, local,
                               reinterpret_cast<float*>(dyn_lds));
        break;
    case JOB_COPY_IN: copy_job(j, p.nx, p.ny, local, true); break;
    case JOB_COPY_OUT: copy_job(j, p.nx, p.ny, local, false); break;
    case JOB_FETCH:
    case JOB_STORE: xfer_job(j, local); break;
    case JOB_HEAT_TB: heat_tb_job(j, p.nx, p.ny, p.nz, p.alpha, local); break;
    default: break;
    }
}

bool is_codec_job(int kind) { return kind == JOB_DECODE || kind == JOB_ENCODE; }

int32_t job_workgroups(const Job& j, int nx, int ny)
{
    const int planes = j.z1 - j.z0;
    if (planes <= 0) return 0;
    switch (j.kind) {
    case JOB_HEAT: {
        const int tiles = ((nx + kHeatTileX - 1) / kHeatTileX) * ((ny + kHeatTileY - 1) / kHeatTileY);
        return tiles * ((planes + kZChunk - 1) / kZChunk);
    }
    case JOB_WAVE: {
        const int tiles = ((nx + 63) / 64) * ((ny + kWaveTileY - 1) / kWaveTileY);
        return tiles * ((planes + kZChunk - 1) / kZChunk);
    }
    case JOB_HEAT_TB: {
        const int ox = 64 - 2 * j.rate, oy = kTbTileY - 2 * j.rate;
        return ((nx + ox - 1) / ox) * ((ny + oy - 1) / oy);
    }
    case JOB_DECODE:
    case JOB_ENCODE: {
        const int nbx = nx / 4, nby = ny / 4;
        const int waves = ((nbx + 63) / 64) * nby * ((planes + 3) / 4);
        return (waves + kWavesPerWG - 1) / kWavesPerWG;
    }
    case JOB_COPY_IN:
    case JOB_COPY_OUT: {
        const int64_t n4 = (int64_t)nx * ny / 4;
        const int64_t per_wg = (int64_t)kBlockThreads * kCopyFloat4PerThread;
        return (int32_t)(((n4 + per_wg - 1) / per_wg) * planes);
    }
    case JOB_FETCH:
    case JOB_STORE: return (int32_t)((j.bytes + kXferBytesPerWG - 1) / kXferBytesPerWG);
    default: return 0;
    }
}

// Orders the jobs, fills the workgroup prefix sums and picks the kernel.
// Returns false if there is no work. Workgroups are dispatched in index
// order and a tick has more of them than the chip holds at once, so the
// longest-running ones go first: transfers (on the pipeline's critical
// path), then the stencil jobs (a temporally blocked workgroup marches its
// whole z-range), then the codec jobs, which fill the slots the others
// leave (a 512^2 x 20-plane tick at 8 bits: 76 -> 62 us against codec first).
static int dispatch_class(int kind) { return is_xfer_job(kind) ? 0 : (is_codec_job(kind) ? 2 : 1); }

static bool prepare_jobs(LaunchParams& p, const void** func, unsigned* grid, size_t* lds)
{
    Job sorted[kMaxJobs];
    int n = 0;
    for (int pass = 0; pass < 3; ++pass)
        for (int i = 0; i < p.njobs; ++i)
            if (dispatch_class(p.jobs[i].kind) == pass) sorted[n++] = p.jobs[i];
    int32_t total = 0;
    int max_rate = 0;
    for (int i = 0; i < n; ++i) {
        p.jobs[i] = sorted[i];
        p.wg_begin[i] = total;
        p.jobs[i].wg_count = job_workgroups(p.jobs[i], p.nx, p.ny);
        total += p.jobs[i].wg_count;
        if (is_codec_job(p.jobs[i].kind)) max_rate = max(max_rate, p.jobs[i].rate);
    }
    p.wg_begin[p.njobs] = total;
    if (total == 0) return false;
    *grid = (unsigned)total;
    p.nfirst = p.ncodec = 0;
    for (int i = 0; i < n; ++i) (is_codec_job(p.jobs[i].kind) ? p.ncodec : p.nfirst) += p.jobs[i].wg_count;
    size_t tb_lds = 0;  // stencil jobs' LDS: blocked heat edge rows, staged wave planes
    bool wave = false, heat_only = true;
    for (int i = 0; i < n; ++i) {
        wave = wave || p.jobs[i].kind == JOB_WAVE;
        heat_only = heat_only && p.jobs[i].kind == JOB_HEAT;
        if (p.jobs[i].kind == JOB_HEAT_TB && heat_tb_lds(p.jobs[i].rate) > tb_lds) tb_lds = heat_tb_lds(p.jobs[i].rate);
        if (p.jobs[i].kind == JOB_WAVE && stencil::wave_tile_lds() > tb_lds) tb_lds = stencil::wave_tile_lds();
    }
    bool mid = false;
    for (int i = 0; i < n; ++i) mid = mid || (p.jobs[i].kind == JOB_DECODE && p.jobs[i].mid);
    if (max_rate > 0) {
        *func = mid ? reinterpret_cast<const void*>(&fused_kernel<true>) : reinterpret_cast<const void*>(&fused_kernel<false>);
        const size_t codec_lds = (size_t)kWavesPerWG * 64 * max_rate * sizeof(uint64_t);
        *lds = codec_lds > tb_lds ? codec_lds : tb_lds;
    } else {
        *func = wave        ? reinterpret_cast<const void*>(&stencil_kernel<kStencilWave>)
                : heat_only ? reinterpret_cast<const void*>(&stencil_kernel<kStencilHeat>)
                            : reinterpret_cast<const void*>(&stencil_kernel<kStencilPlain>);
        *lds = tb_lds;
    }
    return true;
}

hipError_t launch_jobs(LaunchParams& p, hipStream_t stream)
{
    if (p.njobs > 0 && p.jobs[0].f64) return launch_jobs_f64(p, stream);
    const void* func;
    unsigned grid;
    size_t lds;
    if (!prepare_jobs(p, &func, &grid, &lds)) return hipSuccess;
    if (func == reinterpret_cast<const void*>(&fused_kernel<false>))
        hipLaunchKernelGGL(fused_kernel<false>, dim3(grid), dim3(kBlockThreads), lds, stream, p);
    else if (func == reinterpret_cast<const void*>(&fused_kernel<true>))
        hipLaunchKernelGGL(fused_kernel<true>, dim3(grid), dim3(kBlockThreads), lds, stream, p);
    else if (func == reinterpret_cast<const void*>(&stencil_kernel<kStencilWave>))
        hipLaunchKernelGGL(stencil_kernel<kStencilWave>, dim3(grid), dim3(kBlockThreads), lds, stream, p);
    else if (func == reinterpret_cast<const void*>(&stencil_kernel<kStencilHeat>))
        hipLaunchKernelGGL(stencil_kernel<kStencilHeat>, dim3(grid), dim3(kBlockThreads), lds, stream, p);
    else
        hipLaunchKernelGGL(stencil_kernel<kStencilPlain>, dim3(grid), dim3(kBlockThreads), lds, stream, p);
    return hipGetLastError();
}

hipError_t add_jobs_node(LaunchParams& p, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps, hipGraphNode_t* node)
{
    const void* func[2];
    unsigned grid[2];
    size_t lds[2];
    int nk;
    *node = nullptr;
    if (p.njobs > 0 && p.jobs[0].f64) {
        nk = prepare_jobs_f64(p, func, grid, lds);
    } else {
        nk = prepare_jobs(p, &func[0], &grid[0], &lds[0]) ? 1 : 0;
    }
    // the kernels of a tick in a chain; *node is the last one
    for (int i = 0; i < nk; ++i) {
        void* args[] = {&p};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(func[i]);
        kp.gridDim = dim3(grid[i]);
        kp.blockDim = dim3(kBlockThreads);
        kp.sharedMemBytes = (unsigned)lds[i];
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t prev = *node;
        const hipError_t e = i == 0 ? hipGraphAddKernelNode(node, g, deps, ndeps, &kp)
                                    : hipGraphAddKernelNode(node, g, &prev, 1, &kp);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ void step_ctr_kernel(int32_t* ctr, int add, int32_t value)
{
    if (threadIdx.x == 0) *ctr = add ? *ctr + value : value;
}

hipError_t launch_step_ctr(int32_t* ctr, bool add, int32_t value, hipStream_t stream)
{
    hipLaunchKernelGGL(step_ctr_kernel, dim3(1), dim3(64), 0, stream, ctr, add ? 1 : 0, value);
    return hipGetLastError();
}

hipError_t add_step_ctr_node(int32_t* ctr, bool add, int32_t value, hipGraph_t g, const hipGraphNode_t* deps,
                             size_t ndeps, hipGraphNode_t* node)
{
    int a = add ? 1 : 0;
    void* args[] = {&ctr, &a, &value};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(&step_ctr_kernel);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, deps, ndeps, &kp);
}

// ---------------------------------------------------------------------------
// Standalone codec on dense fields
// ---------------------------------------------------------------------------

// MID: decode with mid-point reconstruction (its own kernel, for the
// registers).
template <bool MID>
__global__ void __launch_bounds__(kBlockThreads)
codec_field_kernel(bool encode, const float* in_f, float* out_f, const uint64_t* in_w, uint64_t* out_w, int nbx,
                   int nby, int nbz, int64_t ld_y, int64_t ld_z, int rate)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int chunks = (nbx + 63) / 64;
    const int64_t c = (int64_t)blockIdx.x * kWavesPerWG + wave;
    const int bz = (int)(c / ((int64_t)chunks * nby));
    const int rem = (int)(c % ((int64_t)chunks * nby));
    const int by = rem / chunks;
    const int bx0 = (rem % chunks) * 64;
    const int nblocks = bz < nbz ? min(64, nbx - bx0) : 0;
    const bool active = lane < nblocks;
    uint64_t* lds = dyn_lds + (size_t)wave * 64 * rate;
    const int64_t blk0 = ((int64_t)bz * nby + by) * nbx + bx0;
    const int64_t base = (int64_t)(4 * bz) * ld_z + (int64_t)(4 * by) * ld_y + 4 * (bx0 + lane);
    float x[64];
    if (encode) {
        if (active) {
#pragma unroll
            for (int l = 0; l < 4; ++l)
#pragma unroll
                for (int jy = 0; jy < 4; ++jy) {
                    const float4 v = *reinterpret_cast<const float4*>(in_f + base + l * ld_z + jy * ld_y);
                    x[16 * l + 4 * jy] = v.x; x[16 * l + 4 * jy + 1] = v.y;
                    x[16 * l + 4 * jy + 2] = v.z; x[16 * l + 4 * jy + 3] = v.w;
                }
            codec::encode_lane<false>(x, rate, lds + lane);
        }
        __syncthreads();
        if (nblocks > 0) codec::lds_to_words(lds, out_w + blk0 * rate, rate, nblocks, lane);
    } else {
        if (nblocks > 0) codec::words_to_lds(in_w + blk0 * rate, lds, rate, nblocks, lane);
        __syncthreads();
        if (active) {
            codec::decode_lane<false, MID>(lds + lane, rate, x);
#pragma unroll
            for (int l = 0; l < 4; ++l)
#pragma unroll
                for (int jy = 0; jy < 4; ++jy)
                    *reinterpret_cast<float4*>(out_f + base + l * ld_z + jy * ld_y) =
                        make_float4(x[16 * l + 4 * jy], x[16 * l + 4 * jy + 1], x[16 * l + 4 * jy + 2], x[16 * l + 4 * jy + 3]);
        }
    }
}

hipError_t launch_codec_field(bool encode, const float* in_f, float* out_f, const uint64_t* in_w, uint64_t* out_w,
                              int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                              hipStream_t stream, bool mid)
{
    const int nbx = (int)(nx / 4), nby = (int)(ny / 4), nbz = (int)(nz / 4);
    const int64_t waves = (int64_t)((nbx + 63) / 64) * nby * nbz;
    const int64_t groups = (waves + kWavesPerWG - 1) / kWavesPerWG;
    if (groups == 0) return hipSuccess;
    const size_t lds = (size_t)kWavesPerWG * 64 * rate * sizeof(uint64_t);
    if (mid && !encode)
        hipLaunchKernelGGL(codec_field_kernel<true>, dim3((unsigned)groups), dim3(kBlockThreads), lds, stream, false,
                           in_f, out_f, in_w, out_w, nbx, nby, nbz, ld_y, ld_z, rate);
    else
        hipLaunchKernelGGL(codec_field_kernel<false>, dim3((unsigned)groups), dim3(kBlockThreads), lds, stream, encode,
                           in_f, out_f, in_w, out_w, nbx, nby, nbz, ld_y, ld_z, rate);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlockThreads) swap_kernel(float* a, float* b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x;
    if (i < n) {
        const float t = a[i];
        a[i] = b[i];
        b[i] = t;
    }
}

hipError_t launch_swap(float* a, float* b, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(swap_kernel, dim3((unsigned)((n + kBlockThreads - 1) / kBlockThreads)), dim3(kBlockThreads), 0,
                       stream, a, b, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched heat domains: one launch advances every domain one step
// ---------------------------------------------------------------------------

size_t tile_cfg_lds(int cfg)
{
    const TileCfg& t = kTileCfgs[cfg];
    return t.k > 1 ? (size_t)t.k * 2 * 2 * 4 * 64 * sizeof(float) : 0;
}

template <int C>
__device__ __attribute__((always_inline)) inline void heat_dense_cfg(const float* src, float* dst, int nx, int ny, int nz, float alpha, int wg,
                                      float* lds)
{
    constexpr TileCfg t = kTileCfgs[C];
    if constexpr (t.k > 1) {
        const Ring rs{const_cast<float*>(src), nz, (int64_t)nx * ny}, rd{dst, nz, (int64_t)nx * ny};
        const int tiles = stencil::heat_tb_tiles<t.ty, t.k>(nx, ny);
        const int z0 = (wg / tiles) * t.zc;
        stencil::heat_tb<t.ty, t.k>(rs, rd, nx, ny, nz, alpha, z0, min(nz, z0 + t.zc), wg % tiles, lds);
    } else {
        stencil::heat_dense<t.tx, t.ty, t.zc>(src, dst, nx, ny, nz, alpha, wg);
    }
}

// TB = false: the depth-1 configurations only; TB = true: the temporally
// blocked ones. Separate kernels keep the depth-1 code at its own register
// count (a kernel's occupancy follows its costliest path).
template <bool TB>
__device__ __attribute__((always_inline)) inline void heat_dense_any(int cfg, const float* src, float* dst, int nx, int ny, int nz, float alpha, int wg,
                                      float* lds)
{
    if constexpr (TB) {
        switch (cfg) {
        case 6: heat_dense_cfg<6>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 7: heat_dense_cfg<7>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 8: heat_dense_cfg<8>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 10: heat_dense_cfg<10>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 11: heat_dense_cfg<11>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        default: heat_dense_cfg<9>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        }
    } else {
        switch (cfg) {
        case 0: heat_dense_cfg<0>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 1: heat_dense_cfg<1>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 2: heat_dense_cfg<2>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 3: heat_dense_cfg<3>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        case 4: heat_dense_cfg<4>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        default: heat_dense_cfg<5>(src, dst, nx, ny, nz, alpha, wg, lds); break;
        }
    }
}

int32_t batch_domain_workgroups(int nx, int ny, int nz, int cfg)
{
    const TileCfg& t = kTileCfgs[cfg];
    if (t.k > 1) {
        const int ox = t.tx - 2 * t.k, oy = t.ty - 2 * t.k;
        return ((nx + ox - 1) / ox) * ((ny + oy - 1) / oy) * ((nz + t.zc - 1) / t.zc);
    }
    return ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty) * ((nz + t.zc - 1) / t.zc);
}

// One launch advances every domain of the table by its configuration's k
// steps (the table holds one depth). Workgroup -> domain by binary search.
template <bool TB>
__global__ void __launch_bounds__(kBlockThreads)
batch_step_kernel(const BatchDomain* __restrict__ table, int nd, int parity, float alpha)
{
    const int wg = (int)blockIdx.x;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (table[mid].wg_begin <= wg) lo = mid; else hi = mid - 1;
    }
    const BatchDomain& d = table[lo];
    const float* src = parity ? d.b : d.a;
    float* dst = parity ? d.a : d.b;
    heat_dense_any<TB>(d.cfg, src, dst, d.nx, d.ny, d.nz, alpha, wg - d.wg_begin, reinterpret_cast<float*>(dyn_lds));
}

template <bool TB>
__global__ void __launch_bounds__(kBlockThreads)
heat_dense_kernel(const float* src, float* dst, int nx, int ny, int nz, float alpha, int cfg)
{
    heat_dense_any<TB>(cfg, src, dst, nx, ny, nz, alpha, (int)blockIdx.x, reinterpret_cast<float*>(dyn_lds));
}

// ---- persistent batched launch ----------------------------------------------

// Item i of the queue: a tile of one group of one domain, or a copy item.
struct BatchItem {
    const BatchDomain* e;  // the domain's work-list entry
    int32_t d;             // domain
    int32_t wg;            // first tile (workgroup index within the domain) or copy item of the domain
    int32_t nt;            // tiles of the item (1 for a copy item)
    int32_t g;             // group of this launch, or -1 for a copy item
    uint32_t need;         // finished tiles of d this item waits for
};

__device__ inline BatchItem batch_item(const BatchPersistArgs& a, uint32_t i)
{
    BatchItem it;
    const uint32_t n = (uint32_t)a.groups * (uint32_t)a.items;
    int32_t r;
    const int32_t* begin;  // per domain: first item (tiles or copy) of the domain
    int stride;            // in int32 words
    if (i < n) {
        it.g = (int32_t)(i / (uint32_t)a.items);
        r = (int32_t)(i % (uint32_t)a.items);
        begin = &a.tab->item_begin;
        stride = (int)(sizeof(BatchDomain) / sizeof(int32_t));
    } else {
        it.g = -1;
        r = (int32_t)(i - n);
        begin = a.copy_begin;
        stride = 1;
    }
    int lo = 0, hi = a.nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (begin[mid * stride] <= r) lo = mid; else hi = mid - 1;
    }
    it.d = lo;
    it.e = a.tab + lo;
    const int32_t tiles = (lo + 1 < a.nd ? a.tab[lo + 1].wg_begin : a.total) - a.tab[lo].wg_begin;
    if (it.g >= 0) {
        it.wg = (r - begin[lo * stride]) * kBatchTilesPerItem;
        it.nt = min(kBatchTilesPerItem, tiles - it.wg);
    } else {
        it.wg = r - begin[lo * stride];
        it.nt = 1;
    }
    it.need = (uint32_t)(it.g < 0 ? a.groups : it.g) * (uint32_t)tiles;
    return it;
}

// Queue accesses of the persistent kernel. Only lane 0 of wave 0 touches
// the counters, but the whole of wave 0 runs the grab and the waits, with
// every value made uniform by readfirstlane, so no loop sits inside a
// region that only some lanes of a wave enter. (With the poll loop inside
// `if (threadIdx.x == 0)`, the compiler kept the other lanes in an inner
// loop around the barrier that re-read the old item and never left it:
// the launch never ended.)
__device__ inline uint32_t lane0_load(uint32_t* p)
{
    uint32_t v = 0;
    if ((threadIdx.x & 63) == 0) v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ inline uint32_t lane0_fetch_add(uint32_t* p, uint32_t v)
{
    uint32_t old = 0;
    if ((threadIdx.x & 63) == 0) old = __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)old);
}

// Wave 0: wait until *ctr >= need. Gives up (false) when another wait has
// given up (status set) or after spin_limit polls, then setting the status.
__device__ inline bool batch_wait(uint32_t* ctr, uint32_t need, uint32_t* status, int64_t spin_limit, bool force)
{
    for (int64_t spins = 0;; ++spins) {
        if (!force && lane0_load(ctr) >= need) return true;
        if (lane0_load(status) != 0u) return false;
        if (spins >= spin_limit) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// A work-list entry in scalar registers. The entry is the same for the whole
// workgroup, but the compiler cannot tell (the list is read through a
// structure field, so its loads are vector loads): every field goes through
// readfirstlane, which keeps the tile code's addresses and its switch on the
// configuration uniform.
__device__ inline int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float* uni(float* p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint64_t lo = (uint32_t)uni((int32_t)(uint32_t)v), hi = (uint32_t)uni((int32_t)(uint32_t)(v >> 32));
    return reinterpret_cast<float*>(lo | (hi << 32));
}
__device__ inline BatchDomain uniform_entry(const BatchDomain* p)
{
    BatchDomain e;
    e.a = uni(p->a);
    e.b = uni(p->b);
    e.nx = uni(p->nx);
    e.ny = uni(p->ny);
    e.nz = uni(p->nz);
    e.cfg = uni(p->cfg);
    e.wg_begin = uni(p->wg_begin);
    e.item_begin = uni(p->item_begin);
    return e;
}

// Every workgroup takes items from the queue in order until it is empty (or a
// wait gave up). An item only waits for items earlier in the queue, which
// running workgroups already hold, so the launch drains whatever number of
// workgroups the device runs at once. Every wave releases its outputs at
// device scope before the domain's count is raised, and acquires at device
// scope before reading its inputs, so halo cells written by workgroups on
// other dies (each with its own L2) are seen. The last workgroup to leave
// resets the queue and the counts for the next launch; the status stays for
// the host to read. TB: temporally blocked tiles only (a separate kernel, so
// that the depth-1 path and the copy items do not raise its register count;
// at 7 waves per SIMD it needs no spill).
template <bool TB>
__global__ void __launch_bounds__(kBlockThreads, TB ? 7 : 8) batch_persistent_kernel(BatchPersistArgs a)
{
    __shared__ uint32_t s_item;
    uint32_t* head = a.sync;
    uint32_t* exited = a.sync + 1;
    uint32_t* status = a.sync + 2;
    uint32_t* done = a.sync + kBatchSyncWords;
    const uint32_t total = (uint32_t)a.groups * (uint32_t)a.items + (TB ? 0u : (uint32_t)a.copy_items);
    float* lds = reinterpret_cast<float*>(dyn_lds);
    for (;;) {
        if (threadIdx.x < 64) {  // wave 0, all lanes (a wave-uniform branch)
            uint32_t item = 0xffffffffu;
            if (lane0_load(status) == 0u) {
                const uint32_t i = lane0_fetch_add(head, 1u);
                if (i < total) {
                    const BatchItem it = batch_item(a, i);
                    if (batch_wait(done + it.d, it.need, status, a.spin_limit, a.force_wait != 0)) item = i;
                }
            }
            if (threadIdx.x == 0) s_item = item;
        }
        __syncthreads();
        // the same for every lane: kept in scalar registers
        const uint32_t i = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
        if (i == 0xffffffffu) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const BatchItem it = batch_item(a, i);
        const BatchDomain e = uniform_entry(it.e);
        const int nt = uni(it.nt);
        if (TB || it.g >= 0) {
            const bool odd = ((it.g + a.parity0) & 1) != 0;
            const float* src = odd ? e.b : e.a;
            float* dst = odd ? e.a : e.b;
            const int wg0 = uni(it.wg);
            for (int t = 0; t < nt; ++t) {
                if (t) __syncthreads();  // the tiles share the workgroup's LDS
                heat_dense_any<TB>(e.cfg, src, dst, e.nx, e.ny, e.nz, a.alpha, wg0 + t, lds);
            }
        } else {
            // the last group left the state in b: move kBatchCopyFloats of it
            const int64_t n = (int64_t)e.nx * e.ny * e.nz;
            const int64_t off = (int64_t)it.wg * kBatchCopyFloats;
            const int m = (int)min((int64_t)kBatchCopyFloats, n - off);
            const float* src = e.b + off;
            float* dst = e.a + off;
            for (int q = (int)threadIdx.x; q < m; q += kBlockThreads) dst[q] = src[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0 && (TB || it.g >= 0))  // a single atomic, no loop: safe for one lane
            __hip_atomic_fetch_add(done + it.d, (uint32_t)nt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
        const uint32_t n = __hip_atomic_fetch_add(exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (n + 1u == gridDim.x) {
            for (int d = 0; d < a.nd; ++d) __hip_atomic_store(done + d, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(exited, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

static const void* persistent_fn(bool tb)
{
    return tb ? reinterpret_cast<const void*>(&batch_persistent_kernel<true>)
              : reinterpret_cast<const void*>(&batch_persistent_kernel<false>);
}

hipError_t launch_batch_persistent(const BatchPersistArgs& a, bool tb, int grid, size_t lds, hipStream_t stream)
{
    if (grid <= 0) return hipSuccess;
    if (tb)
        hipLaunchKernelGGL(batch_persistent_kernel<true>, dim3((unsigned)grid), dim3(kBlockThreads), lds, stream, a);
    else
        hipLaunchKernelGGL(batch_persistent_kernel<false>, dim3((unsigned)grid), dim3(kBlockThreads), lds, stream, a);
    return hipGetLastError();
}

hipError_t add_batch_persistent_node(const BatchPersistArgs& a, bool tb, int grid, size_t lds, hipGraph_t g,
                                     const hipGraphNode_t* deps, size_t ndeps, hipGraphNode_t* node)
{
    BatchPersistArgs copy = a;
    void* args[] = {&copy};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(persistent_fn(tb));
    kp.gridDim = dim3((unsigned)grid);
    kp.blockDim = dim3(kBlockThreads);
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, deps, ndeps, &kp);
}

hipError_t batch_persistent_grid(bool tb, size_t lds, int* grid)
{
    int dev = 0, per_cu = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_fn(tb), kBlockThreads, lds);
    if (e != hipSuccess) return e;
    *grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    return hipSuccess;
}

__global__ void zero_words_kernel(uint32_t* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero_words(uint32_t* p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((n + kBlockThreads - 1) / kBlockThreads)),
                       dim3(kBlockThreads), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_batch_step(const BatchDomain* d_table, int nd, int32_t total_wg, size_t lds, int parity,
                             float alpha, hipStream_t stream)
{
    if (total_wg <= 0 || nd <= 0) return hipSuccess;
    if (lds > 0)
        hipLaunchKernelGGL(batch_step_kernel<true>, dim3((unsigned)total_wg), dim3(kBlockThreads), lds, stream, d_table,
                           nd, parity, alpha);
    else
        hipLaunchKernelGGL(batch_step_kernel<false>, dim3((unsigned)total_wg), dim3(kBlockThreads), 0, stream, d_table,
                           nd, parity, alpha);
    return hipGetLastError();
}

hipError_t add_batch_step_node(const BatchDomain* d_table, int nd, int32_t total_wg, size_t lds, int parity,
                               float alpha, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                               hipGraphNode_t* node)
{
    void* args[] = {&d_table, &nd, &parity, &alpha};
    hipKernelNodeParams kp{};
    kp.func = lds > 0 ? reinterpret_cast<void*>(&batch_step_kernel<true>) : reinterpret_cast<void*>(&batch_step_kernel<false>);
    kp.gridDim = dim3((unsigned)total_wg);
    kp.blockDim = dim3(kBlockThreads);
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, deps, ndeps, &kp);
}

hipError_t launch_heat_dense(const float* src, float* dst, int nx, int ny, int nz, float alpha, int cfg,
                             hipStream_t stream)
{
    const int32_t wgs = batch_domain_workgroups(nx, ny, nz, cfg);
    if (wgs <= 0) return hipSuccess;
    if (kTileCfgs[cfg].k > 1)
        hipLaunchKernelGGL(heat_dense_kernel<true>, dim3((unsigned)wgs), dim3(kBlockThreads), tile_cfg_lds(cfg), stream,
                           src, dst, nx, ny, nz, alpha, cfg);
    else
        hipLaunchKernelGGL(heat_dense_kernel<false>, dim3((unsigned)wgs), dim3(kBlockThreads), 0, stream, src, dst, nx,
                           ny, nz, alpha, cfg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the wave propagator and its small helpers
// ---------------------------------------------------------------------------

constexpr int kAdjTileY = 8;  // adjoint step tile: 64 x 8 cells

__global__ void __launch_bounds__(kBlockThreads) adjoint_step_kernel(adjoint::StepArgs a)
{
    adjoint::adjoint_step<kAdjTileY>(a, (int)blockIdx.x, reinterpret_cast<float*>(dyn_lds));
}

hipError_t launch_adjoint_step(const float* l1, const float* wl1, const float* l2, const float* w, const float* p,
                               float* l0, float* wl0, float* grad, int64_t nx, int64_t ny, int64_t nz,
                               hipStream_t stream)
{
    adjoint::StepArgs a{l1, wl1, l2, w, p, l0, wl0, grad, (int)nx, (int)ny, (int)nz};
    const int64_t tiles = ((nx + 63) / 64) * ((ny + kAdjTileY - 1) / kAdjTileY);
    const int64_t wgs = tiles * ((nz + kZChunk - 1) / kZChunk);
    if (wgs == 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_step_kernel, dim3((unsigned)wgs), dim3(kBlockThreads),
                       adjoint::StepTile<kAdjTileY>::lds_bytes(), stream, a);
    return hipGetLastError();
}

// res[i] = p[rcv[i]] - obs[i]; receivers outside [0, n) are skipped
__global__ void rcv_sample_kernel(const float* p, const int64_t* rcv, int nr, const float* obs, float* res, int64_t n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < nr) {
        const int64_t r = rcv[i];
        res[i] = (r >= 0 && r < n) ? p[r] - obs[i] : 0.0f;
    }
}

// lam[rcv[i]] += res[i] for i = 0, 1, ... in order, and wl = w * lam at each
// touched cell. Receivers may share a cell: one thread per receiver, and the
// first receiver at a cell owns it and adds the residuals of every receiver
// there in index order (the same FP32 sums as the sequential loop); the
// others return. Each scan is over nr indexes, read from cache.
__global__ void rcv_inject_kernel(float* lam, float* wl, const float* w, const int64_t* rcv, int nr, const float* res,
                                  int64_t n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nr) return;
    const int64_t r = rcv[i];
    if (r < 0 || r >= n) return;
    for (int j = 0; j < i; ++j)
        if (rcv[j] == r) return;
    float l = lam[r];
    for (int j = i; j < nr; ++j)
        if (rcv[j] == r) l = l + res[j];
    lam[r] = l;
    wl[r] = w[r] * l;
}

hipError_t launch_rcv_sample(const float* p, const int64_t* rcv, int nr, const float* obs, float* res, int64_t n,
                             hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(rcv_sample_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, p, rcv, nr, obs, res, n);
    return hipGetLastError();
}

hipError_t launch_rcv_inject(float* lam, float* wl, const float* w, const int64_t* rcv, int nr, const float* res,
                             int64_t n, hipStream_t s)
{
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(rcv_inject_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, lam, wl, w, rcv, nr,
                       res, n);
    return hipGetLastError();
}

// w = (v*c)*(v*c);  gv = gw*((2*v)*(c*c));  x = 0
__global__ void v_to_w_kernel(const float* v, float c, float* w, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x;
    if (i < n) {
        const float t = v[i] * c;
        w[i] = t * t;
    }
}

__global__ void grad_w_to_v_kernel(const float* gw, const float* v, float c, float* gv, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x;
    if (i < n) gv[i] = gw[i] * ((2.0f * v[i]) * (c * c));
}

__global__ void fill_kernel(float* x, float value, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlockThreads + threadIdx.x;
    if (i < n) x[i] = value;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlockThreads - 1) / kBlockThreads); }

hipError_t launch_v_to_w(const float* v, float c, float* w, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(v_to_w_kernel, dim3(blocks_for(n)), dim3(kBlockThreads), 0, s, v, c, w, n);
    return hipGetLastError();
}

hipError_t launch_grad_w_to_v(const float* gw, const float* v, float c, float* gv, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(grad_w_to_v_kernel, dim3(blocks_for(n)), dim3(kBlockThreads), 0, s, gw, v, c, gv, n);
    return hipGetLastError();
}

hipError_t launch_fill(float* x, float value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(kBlockThreads), 0, s, x, value, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Diagnostic stage kernels (same device code, stage outputs switched on)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlockThreads)
encode_stages_kernel(const float* blocks, int64_t nblocks, int rate, EncStages s)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t b0 = ((int64_t)blockIdx.x * kWavesPerWG + wave) * 64;
    const int nb = (int)max<int64_t>(0, min<int64_t>(64, nblocks - b0));
    const int64_t b = b0 + lane;
    uint64_t* lds = dyn_lds + (size_t)wave * 64 * rate;
    if (lane < nb) {
        float x[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) x[i] = blocks[64 * b + i];
        codec::EncStageOut st{s.emax, s.q, s.t, s.u, s.planes, s.bits};
        codec::encode_lane<true>(x, rate, lds + lane, st, b);
    }
    __syncthreads();
    if (nb > 0 && s.words) codec::lds_to_words(lds, s.words + b0 * rate, rate, nb, lane);
}

__global__ void __launch_bounds__(kBlockThreads)
decode_stages_kernel(const uint64_t* words, int64_t nblocks, int rate, bool mid, DecStages s)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t b0 = ((int64_t)blockIdx.x * kWavesPerWG + wave) * 64;
    const int nb = (int)max<int64_t>(0, min<int64_t>(64, nblocks - b0));
    const int64_t b = b0 + lane;
    uint64_t* lds = dyn_lds + (size_t)wave * 64 * rate;
    if (nb > 0) codec::words_to_lds(words + b0 * rate, lds, rate, nb, lane);
    __syncthreads();
    if (lane < nb) {
        float x[64];
        codec::DecStageOut st{s.emax, s.planes, s.u, s.q};
        if (mid) codec::decode_lane<true, true>(lds + lane, rate, x, st, b);
        else codec::decode_lane<true, false>(lds + lane, rate, x, st, b);
        if (s.out) {
#pragma unroll
            for (int i = 0; i < 64; ++i) s.out[64 * b + i] = x[i];
        }
    }
}

hipError_t launch_encode_stages(const float* blocks, int64_t nblocks, int rate, EncStages s, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const unsigned g = (unsigned)((nblocks + 64 * kWavesPerWG - 1) / (64 * kWavesPerWG));
    const size_t lds = (size_t)kWavesPerWG * 64 * rate * sizeof(uint64_t);
    hipLaunchKernelGGL(encode_stages_kernel, dim3(g), dim3(kBlockThreads), lds, stream, blocks, nblocks, rate, s);
    return hipGetLastError();
}

hipError_t launch_decode_stages(const uint64_t* words, int64_t nblocks, int rate, bool mid, DecStages s,
                                hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const unsigned g = (unsigned)((nblocks + 64 * kWavesPerWG - 1) / (64 * kWavesPerWG));
    const size_t lds = (size_t)kWavesPerWG * 64 * rate * sizeof(uint64_t);
    hipLaunchKernelGGL(decode_stages_kernel, dim3(g), dim3(kBlockThreads), lds, stream, words, nblocks, rate, mid, s);
    return hipGetLastError();
}

}  // namespace oocs
