// codec64.hip -- the fixed-rate 4^3 block format for FP64 values, the
// precision of the paper's experiments (Sec. VI): the method of the FP32
// codec (Sec. IV; Lindstrom, IEEE TVCG 20(12), 2014) with 64-bit integers,
// an 11-bit exponent field (12-bit header) and 64 bit planes; the FP64 wave
// step; and the FP64 pipeline kernel.
//
// Codec mapping: one lane per block (codec64_lane.hpp), 64 blocks per wave
// that are consecutive in x, so a row load or store of the field is one
// 2 KiB contiguous access per wave instruction and the wave's blocks are one
// contiguous run of the compressed stream, moved through LDS (word w of
// lane L at w*64 + L). (A first version coded one block per wave, one lane
// per value, with the group tests as wave-uniform scalar code; it was bound
// by the CU's scalar unit at 34-41 G values/s.)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "codec64_lane.hpp"
#include "codec_dev.hpp"
#include "internal.hpp"
#include "stencil_dev.hpp"

namespace oocs {
namespace codec64 {

constexpr int kWaves = kBlockThreads / 64;

// One dynamic LDS buffer per launch: the codec's words (64 * rate per wave)
// or, in the pipeline kernel, also a wave tile's two staged planes.
extern __shared__ uint64_t dyn_lds64[];

// A block's 64 values (natural order i + 4j + 16l), rows of 4 doubles.
__device__ inline void load_block(const double* f, int64_t base, int64_t ld_y, int64_t ld_z, double (&x)[64])
{
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int jy = 0; jy < 4; ++jy) {
            const double2* row = reinterpret_cast<const double2*>(f + base + l * ld_z + jy * ld_y);
            const double2 a = row[0], c = row[1];
            x[16 * l + 4 * jy] = a.x; x[16 * l + 4 * jy + 1] = a.y;
            x[16 * l + 4 * jy + 2] = c.x; x[16 * l + 4 * jy + 3] = c.y;
        }
}

__device__ inline void store_block(double* f, int64_t base, int64_t ld_y, int64_t ld_z, const double (&x)[64])
{
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int jy = 0; jy < 4; ++jy) {
            double2* row = reinterpret_cast<double2*>(f + base + l * ld_z + jy * ld_y);
            row[0] = make_double2(x[16 * l + 4 * jy], x[16 * l + 4 * jy + 1]);
            row[1] = make_double2(x[16 * l + 4 * jy + 2], x[16 * l + 4 * jy + 3]);
        }
}

// Whole fields: wave c codes the 64 blocks from bx0 of block row (by, bz).
__global__ void __launch_bounds__(kBlockThreads)
field_kernel(bool encode, const double* in_f, double* out_f, const uint64_t* in_w, uint64_t* out_w, int nbx, int nby,
             int nbz, int64_t ld_y, int64_t ld_z, int rate)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int chunks = (nbx + 63) / 64;
    const int64_t c = (int64_t)blockIdx.x * kWaves + wave;
    const int bz = (int)(c / ((int64_t)chunks * nby));
    const int rem = (int)(c % ((int64_t)chunks * nby));
    const int by = rem / chunks;
    const int bx0 = (rem % chunks) * 64;
    const int nblocks = bz < nbz ? min(64, nbx - bx0) : 0;
    const bool active = lane < nblocks;
    uint64_t* lds = dyn_lds64 + (size_t)wave * 64 * rate;
    const int64_t blk0 = ((int64_t)bz * nby + by) * nbx + bx0;
    const int64_t base = (int64_t)(4 * bz) * ld_z + (int64_t)(4 * by) * ld_y + 4 * (bx0 + lane);
    double x[64];
    if (encode) {
        if (active) {
            load_block(in_f, base, ld_y, ld_z, x);
            encode_lane64<false>(x, rate, lds + lane);
        }
        __syncthreads();
        if (nblocks > 0) codec::lds_to_words(lds, out_w + blk0 * rate, rate, nblocks, lane);
    } else {
        if (nblocks > 0) codec::words_to_lds(in_w + blk0 * rate, lds, rate, nblocks, lane);
        __syncthreads();
        if (active) {
            decode_lane64<false>(lds + lane, rate, x);
            store_block(out_f, base, ld_y, ld_z, x);
        }
    }
}

// Blocks given as (N, 64) rows, every intermediate stage written out.
__global__ void __launch_bounds__(kBlockThreads)
encode_stages_kernel(const double* blocks, int64_t nblocks, int rate, LaneEncOut st, uint64_t* out_w)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t b0 = ((int64_t)blockIdx.x * kWaves + wave) * 64;
    const int nb = (int)min<int64_t>(64, max<int64_t>(0, nblocks - b0));
    uint64_t* lds = dyn_lds64 + (size_t)wave * 64 * rate;
    if (lane < nb) {
        double x[64];
        for (int i = 0; i < 64; ++i) x[i] = blocks[64 * (b0 + lane) + i];
        encode_lane64<true>(x, rate, lds + lane, st, b0 + lane);
    }
    __syncthreads();
    if (nb > 0) codec::lds_to_words(lds, out_w + b0 * rate, rate, nb, lane);
}

__global__ void __launch_bounds__(kBlockThreads)
decode_stages_kernel(const uint64_t* in_w, int64_t nblocks, int rate, LaneDecOut st, double* out)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int64_t b0 = ((int64_t)blockIdx.x * kWaves + wave) * 64;
    const int nb = (int)min<int64_t>(64, max<int64_t>(0, nblocks - b0));
    uint64_t* lds = dyn_lds64 + (size_t)wave * 64 * rate;
    if (nb > 0) codec::words_to_lds(in_w + b0 * rate, lds, rate, nb, lane);
    __syncthreads();
    if (lane < nb) {
        double x[64];
        decode_lane64<true>(lds + lane, rate, x, st, b0 + lane);
        if (out)
            for (int i = 0; i < 64; ++i) out[64 * (b0 + lane) + i] = x[i];
    }
}

}  // namespace codec64

hipError_t launch_codec64_field(bool encode, const double* in_f, double* out_f, const uint64_t* in_w, uint64_t* out_w,
                                int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                                hipStream_t stream)
{
    const int nbx = (int)(nx / 4), nby = (int)(ny / 4), nbz = (int)(nz / 4);
    const int64_t waves = (int64_t)((nbx + 63) / 64) * nby * nbz;
    const int64_t groups = (waves + codec64::kWaves - 1) / codec64::kWaves;
    if (groups == 0) return hipSuccess;
    const size_t lds = (size_t)codec64::kWaves * 64 * rate * sizeof(uint64_t);
    hipLaunchKernelGGL(codec64::field_kernel, dim3((unsigned)groups), dim3(kBlockThreads), lds, stream, encode, in_f,
                       out_f, in_w, out_w, nbx, nby, nbz, ld_y, ld_z, rate);
    return hipGetLastError();
}

hipError_t launch_codec64_stages(bool encode, const double* blocks, const uint64_t* in_w, int64_t nblocks, int rate,
                                 int32_t* emax, int64_t* q, int64_t* t, uint64_t* u, uint64_t* planes,
                                 uint64_t* out_w, int32_t* bits, double* out, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const int64_t waves = (nblocks + 63) / 64;
    const unsigned g = (unsigned)((waves + codec64::kWaves - 1) / codec64::kWaves);
    const size_t lds = (size_t)codec64::kWaves * 64 * rate * sizeof(uint64_t);
    if (encode)
        hipLaunchKernelGGL(codec64::encode_stages_kernel, dim3(g), dim3(kBlockThreads), lds, stream, blocks, nblocks,
                           rate, codec64::LaneEncOut{emax, q, t, u, planes, bits}, out_w);
    else
        hipLaunchKernelGGL(codec64::decode_stages_kernel, dim3(g), dim3(kBlockThreads), lds, stream, in_w, nblocks,
                           rate, codec64::LaneDecOut{emax, planes, u, q}, out);
    return hipGetLastError();
}

}  // namespace oocs

// ---------------------------------------------------------------------------
// FP64 wave step (the paper's precision) on dense fields: the pipeline's
// LDS-staged wave tile in double, over the whole grid as one job whose
// "rings" are the dense fields (ring size nz: no wrap-around). The formula
// and operation order are the FP32 level's, in double:
//   acc = 3 c0 p;  acc = acc + c_m * (((x+m + x-m) + (y+m + y-m)) + (z+m + z-m)),  m = 1..4
//   p(n+1) = (2 p - p(n-1)) + w * acc   (+ the source amplitude at its cell)
// p(n+1) is written over p(n-1): a thread reads p(n-1) only at its own
// cells, just before writing them. The source amplitude (a double) is added
// by a one-thread launch after the step: the same single addition.
// ---------------------------------------------------------------------------
namespace oocs {
namespace codec64 {

// FP64 tiles are 64 x 8 cells (2 cells per thread). With the FP32 tile's
// 16 rows a thread keeps 4 cells' 9-plane columns of doubles and the kernel
// needs 186 VGPRs (2 waves per SIMD); 8 rows: 116 (4 waves per SIMD).
constexpr int kTileY64 = 8;

__global__ void __launch_bounds__(kBlockThreads) wave_f64_kernel(Job j, int nx, int ny, int nz)
{
    stencil::wave_tile<double, kTileY64>(j, nx, ny, nz, -1, -1, -1, nullptr, nullptr, (int)blockIdx.x,
                                         reinterpret_cast<double*>(dyn_lds64));
}

__global__ void add_at_kernel(double* f, int64_t cell, double v)
{
    if (threadIdx.x == 0) f[cell] = f[cell] + v;
}

}  // namespace codec64

hipError_t launch_wave_f64(const double* p, double* pm, const double* w, int64_t nx, int64_t ny, int64_t nz,
                           int64_t src_cell, double amp, hipStream_t stream)
{
    if (nx * ny * nz == 0) return hipSuccess;
    Job j;
    memset(&j, 0, sizeof j);
    j.kind = JOB_WAVE;
    j.z0 = 0;
    j.z1 = (int32_t)nz;
    j.f64 = 1;
    const int64_t ld = 2 * nx * ny;  // a plane of doubles, in floats
    j.src = Ring{reinterpret_cast<float*>(const_cast<double*>(p)), nz, ld};
    j.src2 = Ring{reinterpret_cast<float*>(pm), nz, ld};
    j.ro = Ring{reinterpret_cast<float*>(const_cast<double*>(w)), nz, ld};
    j.dst = j.src2;
    const int64_t tiles = ((nx + 63) / 64) * ((ny + codec64::kTileY64 - 1) / codec64::kTileY64);
    const int64_t grid = tiles * ((nz + kZChunk - 1) / kZChunk);
    const size_t lds = stencil::wave_tile_lds<double, codec64::kTileY64>();
    hipLaunchKernelGGL(codec64::wave_f64_kernel, dim3((unsigned)grid), dim3(kBlockThreads), lds, stream, j, (int)nx,
                       (int)ny, (int)nz);
    if (src_cell >= 0) hipLaunchKernelGGL(codec64::add_at_kernel, dim3(1), dim3(64), 0, stream, pm, src_cell, amp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pipeline jobs on FP64 ring planes. A ring slot holds one plane of doubles
// (the ring's plane stride counts floats, two per double). The jobs and the
// staging layouts are those of the FP32 pipeline kernel: a tick's jobs share
// one launch and the workgroup index selects the job; compressed staging
// holds the 4-plane layers of [z0, z1) in z order, each layer's blocks x
// fastest then y, `rate` words per block; raw staging holds the planes back
// to back.
// ---------------------------------------------------------------------------
namespace codec64 {

constexpr int kCopy4PerThread = 4;

__device__ inline double* plane64(const Ring& r, int64_t z) { return reinterpret_cast<double*>(ring_plane(r, z)); }

// Codec job on ring planes: wave c of the job codes the 64 blocks from bx0
// of block row by of 4-plane layer `layer` (the field kernel's mapping).
__device__ inline void ring_codec_job(const Job& j, int nx, int ny, int wg, bool encode)
{
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int nbx = nx >> 2, nby = ny >> 2;
    const int chunks = (nbx + 63) / 64;
    const int c = wg * kWaves + wave;
    const int layer = c / (chunks * nby);
    const int rem = c % (chunks * nby);
    const int by = rem / chunks;
    const int bx0 = (rem % chunks) * 64;
    const int z = j.z0 + 4 * layer;
    const int nblocks = z < j.z1 ? min(64, nbx - bx0) : 0;
    const bool active = lane < nblocks;
    const int rate = j.rate;
    uint64_t* lds = dyn_lds64 + (size_t)wave * 64 * rate;
    uint64_t* words = static_cast<uint64_t*>(j.stage) + (((int64_t)layer * nby + by) * nbx + bx0) * rate;
    const int64_t row0 = (int64_t)(4 * by) * nx + 4 * (bx0 + lane);
    double x[64];
    if (encode) {
        if (active) {
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const double* pl = plane64(j.dst, z + l) + row0;
#pragma unroll
                for (int jy = 0; jy < 4; ++jy) {
                    const double2* row = reinterpret_cast<const double2*>(pl + (int64_t)jy * nx);
                    const double2 a = row[0], b = row[1];
                    x[16 * l + 4 * jy] = a.x; x[16 * l + 4 * jy + 1] = a.y;
                    x[16 * l + 4 * jy + 2] = b.x; x[16 * l + 4 * jy + 3] = b.y;
                }
            }
            encode_lane64<false>(x, rate, lds + lane);
        }
        __syncthreads();
        if (nblocks > 0) codec::lds_to_words(lds, words, rate, nblocks, lane);
    } else {
        if (nblocks > 0) codec::words_to_lds(words, lds, rate, nblocks, lane);
        __syncthreads();
        if (active) {
            decode_lane64<false>(lds + lane, rate, x);
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                double* pl = plane64(j.dst, z + l) + row0;
#pragma unroll
                for (int jy = 0; jy < 4; ++jy) {
                    double2* row = reinterpret_cast<double2*>(pl + (int64_t)jy * nx);
                    row[0] = make_double2(x[16 * l + 4 * jy], x[16 * l + 4 * jy + 1]);
                    row[1] = make_double2(x[16 * l + 4 * jy + 2], x[16 * l + 4 * jy + 3]);
                }
            }
        }
    }
}

// Raw planes of doubles between staging and ring, as float4 moves.
__device__ inline void ring_copy_job(const Job& j, int nx, int ny, int wg, bool in)
{
    const int64_t plane_f = 2 * (int64_t)nx * ny;  // floats per plane
    const int64_t n4 = plane_f / 4;
    const int64_t per_wg = (int64_t)kBlockThreads * kCopy4PerThread;
    const int64_t wg_per_plane = (n4 + per_wg - 1) / per_wg;
    const int pz = (int)(wg / wg_per_plane);
    const int z = j.z0 + pz;
    if (z >= j.z1) return;
    const int64_t base = (wg % wg_per_plane) * per_wg;
    float4* r = reinterpret_cast<float4*>(ring_plane(j.dst, z));
    float4* st = reinterpret_cast<float4*>(static_cast<float*>(j.stage) + (int64_t)pz * plane_f);
#pragma unroll
    for (int k = 0; k < kCopy4PerThread; ++k) {
        const int64_t e = base + (int64_t)k * kBlockThreads + threadIdx.x;
        if (e < n4) {
            if (in) r[e] = st[e]; else st[e] = r[e];
        }
    }
}

// Wave levels are the FP32 pipeline's LDS-staged tile in double (the same
// operation order as the FP64 step above). The jobs of a tick run as two
// kernels, the stencil and copy jobs (the first workgroups of the list),
// then the codec jobs (the last ones): the FP64 codec needs about 215 VGPRs
// per lane and the wave tile 116, and one kernel holding both ran every job
// at two waves per SIMD (with spills), where the stencil kernel alone keeps
// four. PART 1: workgroup b runs workgroup b of the list; PART 2: workgroup
// nfirst + b.
template <int PART>
__global__ void __launch_bounds__(kBlockThreads) fused64_kernel(LaunchParams p)
{
    const int wg = PART == 1 ? (int)blockIdx.x : p.nfirst + (int)blockIdx.x;
    int jdx = 0;
    while (jdx + 1 < p.njobs && wg >= p.wg_begin[jdx + 1]) ++jdx;
    const Job& j = p.jobs[jdx];
    const int local = wg - p.wg_begin[jdx];
    if constexpr (PART == 1) {
        switch (j.kind) {
        case JOB_WAVE:
            stencil::wave_tile<double, kTileY64>(j, p.nx, p.ny, p.nz, p.src_x, p.src_y, p.src_z, p.src_table,
                                                 p.step_ctr, local, reinterpret_cast<double*>(dyn_lds64));
            break;
        case JOB_COPY_IN: ring_copy_job(j, p.nx, p.ny, local, true); break;
        case JOB_COPY_OUT: ring_copy_job(j, p.nx, p.ny, local, false); break;
        default: break;
        }
    } else if (j.kind == JOB_DECODE || j.kind == JOB_ENCODE) {
        // one call with the direction as a value: two inlined copies, one per
        // direction, made the kernel spill 400 bytes per lane
        ring_codec_job(j, p.nx, p.ny, local, j.kind == JOB_ENCODE);
    }
}

static int32_t job_workgroups64(const Job& j, int nx, int ny)
{
    const int64_t planes = j.z1 - j.z0;
    if (planes <= 0) return 0;
    const int64_t plane = (int64_t)nx * ny;
    switch (j.kind) {
    case JOB_WAVE: {
        const int64_t tiles = (int64_t)((nx + 63) / 64) * ((ny + kTileY64 - 1) / kTileY64);
        return (int32_t)(tiles * ((planes + kZChunk - 1) / kZChunk));
    }
    case JOB_DECODE:
    case JOB_ENCODE: {
        const int64_t waves = (int64_t)((nx / 4 + 63) / 64) * (ny / 4) * ((planes + 3) / 4);
        return (int32_t)((waves + kWaves - 1) / kWaves);
    }
    case JOB_COPY_IN:
    case JOB_COPY_OUT: {
        const int64_t per_wg = (int64_t)kBlockThreads * kCopy4PerThread;
        return (int32_t)(((2 * plane / 4 + per_wg - 1) / per_wg) * planes);
    }
    default: return 0;
    }
}

}  // namespace codec64

// Stencil and copy jobs first, codec jobs last; up to two kernels in launch
// order (the first part, then the codec part), each with its grid and LDS.
int prepare_jobs_f64(LaunchParams& p, const void* func[2], unsigned grid[2], size_t lds[2])
{
    Job sorted[kMaxJobs];
    int n = 0;
    auto codec = [](int kind) { return kind == JOB_DECODE || kind == JOB_ENCODE; };
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < p.njobs; ++i)
            if (codec(p.jobs[i].kind) == (pass == 1)) sorted[n++] = p.jobs[i];
    int32_t total = 0;
    for (int i = 0; i < n; ++i) {
        p.jobs[i] = sorted[i];
        p.wg_begin[i] = total;
        p.jobs[i].wg_count = codec64::job_workgroups64(p.jobs[i], p.nx, p.ny);
        total += p.jobs[i].wg_count;
    }
    p.wg_begin[p.njobs] = total;
    p.nfirst = p.ncodec = 0;
    size_t lds_first = 0, lds_codec = 0;
    for (int i = 0; i < n; ++i) {
        if (codec(p.jobs[i].kind)) {
            p.ncodec += p.jobs[i].wg_count;
            lds_codec = std::max(lds_codec, (size_t)codec64::kWaves * 64 * p.jobs[i].rate * sizeof(uint64_t));
        } else {
            p.nfirst += p.jobs[i].wg_count;
            if (p.jobs[i].kind == JOB_WAVE)
                lds_first = std::max(lds_first, stencil::wave_tile_lds<double, codec64::kTileY64>());
        }
    }
    int k = 0;
    if (p.nfirst > 0) {
        func[k] = reinterpret_cast<const void*>(&codec64::fused64_kernel<1>);
        grid[k] = (unsigned)p.nfirst;
        lds[k++] = lds_first;
    }
    if (p.ncodec > 0) {
        func[k] = reinterpret_cast<const void*>(&codec64::fused64_kernel<2>);
        grid[k] = (unsigned)p.ncodec;
        lds[k++] = lds_codec;
    }
    return k;
}

hipError_t launch_jobs_f64(LaunchParams& p, hipStream_t stream)
{
    const void* func[2];
    unsigned grid[2];
    size_t lds[2];
    const int nk = prepare_jobs_f64(p, func, grid, lds);
    for (int i = 0; i < nk; ++i) {
        if (func[i] == reinterpret_cast<const void*>(&codec64::fused64_kernel<1>))
            hipLaunchKernelGGL(codec64::fused64_kernel<1>, dim3(grid[i]), dim3(kBlockThreads), lds[i], stream, p);
        else
            hipLaunchKernelGGL(codec64::fused64_kernel<2>, dim3(grid[i]), dim3(kBlockThreads), lds[i], stream, p);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace oocs
