// kernels.hip -- the gfx950 kernels of liboocs and their host launchers.
//
// The out-of-core pipeline issues one launch per tick. A tick's jobs
// (decode of the next input group, one z-range of every time level, encode
// of the finished output group) are independent by construction of the
// schedule, so they share one launch: the workgroup index selects the job
// and the job's own workgroup. All jobs use 256-thread workgroups.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec_dev.hpp"
#include "internal.hpp"
#include "stencil_dev.hpp"

namespace oocs {

static_assert(sizeof(LaunchParams) <= 4096, "kernel arguments must stay within 4 KiB");

constexpr int kWavesPerWG = kBlockThreads / 64;  // codec: one 4^3 block per wave
constexpr int kCopyFloat4PerThread = 4;

// ---------------------------------------------------------------------------
// Codec and copy jobs on ring planes
// ---------------------------------------------------------------------------

// Staging slot of compressed words: the 4-plane layers of [z0, z1) in z
// order, each layer's blocks x fastest then y; rate words per block.
__device__ inline void codec_job(const Job& j, int nx, int ny, int wg, bool encode)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int nbx = nx >> 2, nby = ny >> 2;
    const int groups_x = (nbx + kWavesPerWG - 1) / kWavesPerWG;
    const int per_layer = groups_x * nby;
    const int layer = wg / per_layer;
    const int rem = wg % per_layer;
    const int by = rem / groups_x;
    const int bx = (rem % groups_x) * kWavesPerWG + wave;
    const int z = j.z0 + 4 * layer;
    if (bx >= nbx || z >= j.z1) return;  // whole wave leaves together
    const int rate = j.rate;
    const int64_t blk = ((int64_t)layer * nby + by) * nbx + bx;
    uint64_t* words = static_cast<uint64_t*>(j.stage) + blk * rate;
    const int i = lane & 3, jy = (lane >> 2) & 3, l = lane >> 4;
    float* cell = ring_plane(j.dst, z + l) + (int64_t)(4 * by + jy) * nx + 4 * bx + i;
    if (encode) {
        const uint64_t w = codec::encode_block<false>(*cell, lane, rate);
        if (lane < rate) words[lane] = w;
    } else {
        const uint64_t w = lane < rate ? words[lane] : 0;
        *cell = codec::decode_block<false>(w, lane, rate);
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

__global__ void __launch_bounds__(kBlockThreads) fused_kernel(LaunchParams p)
{
    const int wg = (int)blockIdx.x;
    int jdx = 0;
    while (jdx + 1 < p.njobs && wg >= p.wg_begin[jdx + 1]) ++jdx;
    const Job& j = p.jobs[jdx];
    const int local = wg - p.wg_begin[jdx];
    switch (j.kind) {
    case JOB_HEAT: stencil::heat_level(j, p.nx, p.ny, p.nz, p.alpha, local); break;
    case JOB_WAVE: stencil::wave_level(j, p.nx, p.ny, p.nz, p.src_x, p.src_y, p.src_z, local); break;
    case JOB_DECODE: codec_job(j, p.nx, p.ny, local, false); break;
    case JOB_ENCODE: codec_job(j, p.nx, p.ny, local, true); break;
    case JOB_COPY_IN: copy_job(j, p.nx, p.ny, local, true); break;
    case JOB_COPY_OUT: copy_job(j, p.nx, p.ny, local, false); break;
    default: break;
    }
}

int32_t job_workgroups(const Job& j, int nx, int ny)
{
    const int planes = j.z1 - j.z0;
    if (planes <= 0) return 0;
    switch (j.kind) {
    case JOB_HEAT:
    case JOB_WAVE: {
        const int tiles = ((nx + kTileX - 1) / kTileX) * ((ny + kTileY - 1) / kTileY);
        return tiles * ((planes + kZChunk - 1) / kZChunk);
    }
    case JOB_DECODE:
    case JOB_ENCODE: {
        const int nbx = nx / 4, nby = ny / 4;
        return ((nbx + kWavesPerWG - 1) / kWavesPerWG) * nby * ((planes + 3) / 4);
    }
    case JOB_COPY_IN:
    case JOB_COPY_OUT: {
        const int64_t n4 = (int64_t)nx * ny / 4;
        const int64_t per_wg = (int64_t)kBlockThreads * kCopyFloat4PerThread;
        return (int32_t)(((n4 + per_wg - 1) / per_wg) * planes);
    }
    default: return 0;
    }
}

hipError_t launch_jobs(LaunchParams& p, hipStream_t stream)
{
    int32_t total = 0;
    for (int i = 0; i < p.njobs; ++i) {
        p.wg_begin[i] = total;
        p.jobs[i].wg_count = job_workgroups(p.jobs[i], p.nx, p.ny);
        total += p.jobs[i].wg_count;
    }
    p.wg_begin[p.njobs] = total;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(fused_kernel, dim3((unsigned)total), dim3(kBlockThreads), 0, stream, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Standalone codec on dense fields
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlockThreads)
codec_field_kernel(bool encode, const float* in_f, float* out_f, const uint64_t* in_w, uint64_t* out_w, int nbx,
                   int nby, int nbz, int64_t ld_y, int64_t ld_z, int rate)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int groups_x = (nbx + kWavesPerWG - 1) / kWavesPerWG;
    const int64_t wg = blockIdx.x;
    const int64_t per_layer = (int64_t)groups_x * nby;
    const int bz = (int)(wg / per_layer);
    const int rem = (int)(wg % per_layer);
    const int by = rem / groups_x;
    const int bx = (rem % groups_x) * kWavesPerWG + wave;
    if (bx >= nbx || bz >= nbz) return;
    const int64_t blk = ((int64_t)bz * nby + by) * nbx + bx;
    const int i = lane & 3, jy = (lane >> 2) & 3, l = lane >> 4;
    const int64_t cell = (int64_t)(4 * bz + l) * ld_z + (int64_t)(4 * by + jy) * ld_y + 4 * bx + i;
    if (encode) {
        const uint64_t w = codec::encode_block<false>(in_f[cell], lane, rate);
        if (lane < rate) out_w[blk * rate + lane] = w;
    } else {
        const uint64_t w = lane < rate ? in_w[blk * rate + lane] : 0;
        out_f[cell] = codec::decode_block<false>(w, lane, rate);
    }
}

hipError_t launch_codec_field(bool encode, const float* in_f, float* out_f, const uint64_t* in_w, uint64_t* out_w,
                              int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                              hipStream_t stream)
{
    const int nbx = (int)(nx / 4), nby = (int)(ny / 4), nbz = (int)(nz / 4);
    const int64_t groups = (int64_t)((nbx + kWavesPerWG - 1) / kWavesPerWG) * nby * nbz;
    if (groups == 0) return hipSuccess;
    hipLaunchKernelGGL(codec_field_kernel, dim3((unsigned)groups), dim3(kBlockThreads), 0, stream, encode, in_f,
                       out_f, in_w, out_w, nbx, nby, nbz, ld_y, ld_z, rate);
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
// Diagnostic stage kernels (same device code, stage outputs switched on)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlockThreads)
encode_stages_kernel(const float* blocks, int64_t nblocks, int rate, EncStages s)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t b = (int64_t)blockIdx.x * kWavesPerWG + (threadIdx.x >> 6);
    if (b >= nblocks) return;
    codec::EncStageOut st{s.emax, s.q, s.t, s.u, s.planes, s.bits};
    const uint64_t w = codec::encode_block<true>(blocks[64 * b + lane], lane, rate, st, b);
    if (s.words && lane < rate) s.words[b * rate + lane] = w;
}

__global__ void __launch_bounds__(kBlockThreads)
decode_stages_kernel(const uint64_t* words, int64_t nblocks, int rate, DecStages s)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t b = (int64_t)blockIdx.x * kWavesPerWG + (threadIdx.x >> 6);
    if (b >= nblocks) return;
    codec::DecStageOut st{s.emax, s.planes, s.u, s.q};
    const uint64_t w = lane < rate ? words[b * rate + lane] : 0;
    const float v = codec::decode_block<true>(w, lane, rate, st, b);
    if (s.out) s.out[64 * b + lane] = v;
}

hipError_t launch_encode_stages(const float* blocks, int64_t nblocks, int rate, EncStages s, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const unsigned g = (unsigned)((nblocks + kWavesPerWG - 1) / kWavesPerWG);
    hipLaunchKernelGGL(encode_stages_kernel, dim3(g), dim3(kBlockThreads), 0, stream, blocks, nblocks, rate, s);
    return hipGetLastError();
}

hipError_t launch_decode_stages(const uint64_t* words, int64_t nblocks, int rate, DecStages s, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const unsigned g = (unsigned)((nblocks + kWavesPerWG - 1) / kWavesPerWG);
    hipLaunchKernelGGL(decode_stages_kernel, dim3(g), dim3(kBlockThreads), 0, stream, words, nblocks, rate, s);
    return hipGetLastError();
}

}  // namespace oocs
