// codec64.hip -- the fixed-rate 4^3 block format for FP64 values, the
// precision of the paper's experiments (Sec. VI): the method of the FP32
// codec (Sec. IV; Lindstrom, IEEE TVCG 20(12), 2014) with 64-bit integers,
// an 11-bit exponent field (12-bit header) and 64 bit planes.
//
// Mapping: one wavefront codes one block, one lane per value. The value's
// lane k is its in-block index i + 4j + 16l; the lifting along x, y and z
// exchanges the four values of a line with ds_bpermute (each lane runs its
// line's 4-point step and keeps its own output); the block exponent is a
// wave reduction; after the sequency reorder (another permute) lane s holds
// the s-th coefficient, so the word of bit plane p is one ballot. The
// group-test coding then runs on those plane words as wave-uniform (scalar)
// code with a bit writer / reader over the block's words in LDS, and the
// decoder hands every lane its digits back from the plane words.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "codec_dev.hpp"
#include "internal.hpp"
#include "stencil_dev.hpp"

namespace oocs {
namespace codec64 {

constexpr uint64_t kNB = 0xAAAAAAAAAAAAAAAAull;
constexpr int kMaxRate = 68;

struct PermTables {
    int fwd[64];   // fwd[s] = in-block index of the s-th coefficient (sequency order)
    int rank[64];  // rank[k] = sequency position of in-block index k
};

constexpr PermTables make_perm()
{
    PermTables t{};
    for (int k = 0; k < 64; ++k) {
        t.rank[k] = codec::seq_rank(k);
        t.fwd[codec::seq_rank(k)] = k;
    }
    return t;
}
__constant__ constexpr PermTables kPerm = make_perm();

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

__device__ inline uint64_t shfl64(uint64_t v, int src)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(v >> 32));
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ inline uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ---- lifting on int64 (wrap-around adds, arithmetic shifts) ------------------
__device__ inline int64_t add_(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
__device__ inline int64_t sub_(int64_t a, int64_t b) { return (int64_t)((uint64_t)a - (uint64_t)b); }

__device__ inline void fwd_lift(int64_t& a, int64_t& b, int64_t& c, int64_t& d)
{
    a = add_(a, d) >> 1; d = sub_(d, a);
    c = add_(c, b) >> 1; b = sub_(b, c);
    a = add_(a, c) >> 1; c = sub_(c, a);
    d = add_(d, b) >> 1; b = sub_(b, d);
    d = add_(d, b >> 1); b = sub_(b, d >> 1);
}

__device__ inline void inv_lift(int64_t& a, int64_t& b, int64_t& c, int64_t& d)
{
    b = add_(b, d >> 1); d = sub_(d, b >> 1);
    b = add_(b, d);      d = sub_(add_(d, d), b);
    c = add_(c, a);      a = sub_(add_(a, a), c);
    b = add_(b, c);      c = sub_(add_(c, c), b);
    d = add_(d, a);      a = sub_(add_(a, a), d);
}

// One 4-point step along the axis whose index bits are at `shift` (x: 0,
// y: 2, z: 4): the lane gathers its line, runs the step, keeps its output.
template <bool INV>
__device__ inline int64_t lift_axis(int64_t v, int shift)
{
    const int k = lane_id();
    const int base = k & ~(3 << shift), s = 1 << shift, pos = (k >> shift) & 3;
    int64_t a = (int64_t)shfl64((uint64_t)v, base), b = (int64_t)shfl64((uint64_t)v, base + s);
    int64_t c = (int64_t)shfl64((uint64_t)v, base + 2 * s), d = (int64_t)shfl64((uint64_t)v, base + 3 * s);
    if (INV) inv_lift(a, b, c, d); else fwd_lift(a, b, c, d);
    return pos == 0 ? a : (pos == 1 ? b : (pos == 2 ? c : d));
}

__device__ inline int exponent_of(double x)
{
    const int e = __builtin_amdgcn_frexp_exp(x);
    return e < -1022 ? -1022 : e;
}

// ---- bits of one block in LDS (rate words, zeroed before encoding) ---------
// Writer and reader keep their state, including the 64-bit word being
// filled or read, in wave-uniform values (scalar registers), so a word of
// LDS is touched once: the writer stores each word when it is full (lane 0)
// and the last partial one at flush(); the reader loads each word once, as
// the window (lo, hi) slides over it.
struct BitWriter {
    uint64_t* words;
    int rate;
    uint64_t cur = 0;  // the bits of word w written so far
    int w = 0, o = 0;  // word index, bits in cur
    __device__ void put(uint64_t bits, int n)  // n in [0, 64]; bits has no bit at or above n
    {
        if (n == 0) return;
        cur |= bits << o;
        if (o + n >= 64) {
            if (lane_id() == 0 && w < rate) words[w] = cur;
            ++w;
            cur = o ? bits >> (64 - o) : 0;
            o = o + n - 64;
        } else {
            o += n;
        }
    }
    __device__ void flush()
    {
        if (o > 0 && lane_id() == 0 && w < rate) words[w] = cur;
    }
};

struct BitReader {
    const uint64_t* words;
    int rate;
    int w = 0, o = 0;  // lo = word w, hi = word w + 1; o = bits of lo consumed
    uint64_t lo = 0, hi = 0;
    __device__ uint64_t word(int i) const { return i < rate ? uniform64(words[i]) : 0; }
    __device__ BitReader(const uint64_t* ws, int r) : words(ws), rate(r) { lo = word(0); hi = word(1); }
    __device__ uint64_t peek64() const  // the next 64 bits (zeros past the block)
    {
        return o ? (lo >> o) | (hi << (64 - o)) : lo;
    }
    __device__ void skip(int n)  // n in [0, 64]
    {
        o += n;
        if (o >= 64) {
            o -= 64;
            ++w;
            lo = hi;
            hi = word(w + 1);
        }
    }
    __device__ uint64_t get(int n)  // n in [0, 64]
    {
        if (n == 0) return 0;
        uint64_t v = peek64();
        if (n < 64) v &= ((uint64_t)1 << n) - 1;
        skip(n);
        return v;
    }
};

__device__ inline int ctz64(uint64_t v) { return v ? __builtin_ctzll(v) : 64; }

// Group-testing bit-plane coder on this lane's coefficient u (sequency
// position = lane): the FP32 format's rules with planes 63..0.
__device__ inline int code_planes(uint64_t u, int budget, BitWriter& bw, uint64_t* planes_out)
{
    int n = 0, used = 0;
    for (int p = 63; p >= 0; --p) {
        const uint64_t X = __ballot((u >> p) & 1);
        if (planes_out && lane_id() == 0) planes_out[p] = X;
        if (budget <= 0) continue;
        const int m = n < budget ? n : budget;
        bw.put(m < 64 ? X & (((uint64_t)1 << m) - 1) : X, m);
        budget -= m;
        used += m;
        while (n < 64 && budget > 0) {
            const bool g = n < 64 && (X >> n) != 0;
            bw.put(g ? 1 : 0, 1);
            --budget;
            ++used;
            if (!g) break;
            const int z = ctz64(X >> n);  // zeros before the next 1 (it exists)
            if (n + z == 63) {             // the last coefficient's 1 is implied
                const int e = z < budget ? z : budget;
                bw.put(0, e);
                budget -= e;
                used += e;
                n = e == z ? 64 : n + e;
            } else {
                const int e = z + 1 <= budget ? z + 1 : budget;
                bw.put(e == z + 1 ? (uint64_t)1 << z : 0, e);
                budget -= e;
                used += e;
                n += e;
            }
        }
    }
    return used;
}

// The decoder's mirror: returns this lane's coefficient digits.
__device__ inline uint64_t decode_planes(int budget, BitReader& br, uint64_t* planes_out)
{
    const int lane = lane_id();
    int n = 0;
    uint64_t u = 0;
    for (int p = 63; p >= 0; --p) {
        uint64_t X = 0;
        if (budget > 0) {
            const int m = n < budget ? n : budget;
            X = br.get(m);
            budget -= m;
            while (n < 64 && budget > 0) {
                const uint64_t g = br.get(1);
                --budget;
                if (!g) break;
                const int lim = (63 - n) < budget ? (63 - n) : budget;  // zeros readable before 63 / the end
                const int z = ctz64(br.peek64());
                if (z < lim) {  // the run's 1 is read
                    br.get(z + 1);
                    budget -= z + 1;
                    X |= (uint64_t)1 << (n + z);
                    n += z + 1;
                } else {        // lim zeros, then either the implied last 1 or the end of the budget
                    br.get(lim);
                    budget -= lim;
                    n += lim;
                    if (n == 63) {
                        X |= (uint64_t)1 << 63;
                        n = 64;
                    }
                }
            }
        }
        if (planes_out && lane == 0) planes_out[p] = X;
        u |= ((X >> lane) & 1) << p;
    }
    return u;
}

struct EncOut { int32_t* emax; int64_t* q; int64_t* t; uint64_t* u; uint64_t* planes; int32_t* bits; };
struct DecOut { int32_t* emax; uint64_t* planes; uint64_t* u; int64_t* q; };

// Encode one block: x = this lane's value (in-block index = lane). `words`:
// the block's rate words in LDS, zeroed by the caller. Stage outputs for
// block b where given.
__device__ inline void encode_block(double x, int rate, uint64_t* words, EncOut st = {}, int64_t b = 0)
{
    const int lane = lane_id();
    const uint64_t nz = __ballot(x != 0.0);
    BitWriter bw{words, rate};
    if (!nz) {
        bw.put(0, 1);
        if (st.emax && lane == 0) st.emax[b] = INT32_MIN;
        if (st.bits && lane == 0) st.bits[b] = 1;
        return;
    }
    int e = x != 0.0 ? exponent_of(x) : -100000;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int other = __builtin_amdgcn_ds_bpermute((lane ^ o) << 2, e);
        e = e > other ? e : other;
    }
    const int emax = __builtin_amdgcn_readfirstlane(e);
    bw.put(1, 1);
    bw.put((uint64_t)(emax + 1023), 11);
    const int64_t q = (int64_t)ldexp(x, 62 - emax);  // the conversion truncates toward zero
    int64_t t = lift_axis<false>(q, 0);
    t = lift_axis<false>(t, 2);
    t = lift_axis<false>(t, 4);
    const int64_t ts = (int64_t)shfl64((uint64_t)t, kPerm.fwd[lane]);  // sequency order
    const uint64_t u = ((uint64_t)ts + kNB) ^ kNB;
    if (st.emax && lane == 0) st.emax[b] = emax;
    if (st.q) st.q[64 * b + lane] = q;
    if (st.t) st.t[64 * b + lane] = t;
    if (st.u) st.u[64 * b + lane] = u;
    const int used = code_planes(u, 64 * rate - 12, bw, st.planes ? st.planes + 64 * b : nullptr);
    bw.flush();
    if (st.bits && lane == 0) st.bits[b] = 12 + used;
}

// Decode one block from its words in LDS; returns this lane's value.
__device__ inline double decode_block(const uint64_t* words, int rate, DecOut st = {}, int64_t b = 0)
{
    const int lane = lane_id();
    BitReader br(words, rate);
    if (!br.get(1)) {
        if (st.emax && lane == 0) st.emax[b] = INT32_MIN;
        if (st.u) st.u[64 * b + lane] = 0;
        if (st.q) st.q[64 * b + lane] = 0;
        if (st.planes && lane == 0)
            for (int p = 0; p < 64; ++p) st.planes[64 * b + p] = 0;
        return 0.0;
    }
    const int emax = (int)br.get(11) - 1023;
    const uint64_t u = decode_planes(64 * rate - 12, br, st.planes ? st.planes + 64 * b : nullptr);
    const int64_t ts = (int64_t)((u ^ kNB) - kNB);
    int64_t t = (int64_t)shfl64((uint64_t)ts, kPerm.rank[lane]);  // natural order
    t = lift_axis<true>(t, 4);
    t = lift_axis<true>(t, 2);
    t = lift_axis<true>(t, 0);
    if (st.emax && lane == 0) st.emax[b] = emax;
    if (st.u) st.u[64 * b + lane] = u;
    if (st.q) st.q[64 * b + lane] = t;
    return ldexp((double)t, emax - 62);
}

// ---- kernels ----------------------------------------------------------------
constexpr int kWaves = kBlockThreads / 64;

// Whole fields: each wave codes blocks w, w + W, ... (W = waves in the grid).
// Block b of the stream is block (bx, by, bz), x fastest.
__global__ void __launch_bounds__(kBlockThreads)
field_kernel(bool encode, const double* in_f, double* out_f, const uint64_t* in_w, uint64_t* out_w, int nbx, int nby,
             int64_t nblocks, int64_t ld_y, int64_t ld_z, int rate)
{
    __shared__ uint64_t buf[kWaves][kMaxRate];
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    uint64_t* words = buf[wave];
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    const int i = lane & 3, j = (lane >> 2) & 3, l = lane >> 4;
    for (int64_t b = (int64_t)blockIdx.x * kWaves + wave; b < nblocks; b += nwaves) {
        const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby);
        const int64_t bz = b / ((int64_t)nbx * nby);
        const int64_t at = (4 * bz + l) * ld_z + (int64_t)(4 * by + j) * ld_y + 4 * bx + i;
        if (encode) {
            for (int w = lane; w < rate; w += 64) words[w] = 0;
            __builtin_amdgcn_wave_barrier();
            encode_block(in_f[at], rate, words);
            __builtin_amdgcn_wave_barrier();
            for (int w = lane; w < rate; w += 64) out_w[b * rate + w] = words[w];
        } else {
            for (int w = lane; w < rate; w += 64) words[w] = in_w[b * rate + w];
            __builtin_amdgcn_wave_barrier();
            out_f[at] = decode_block(words, rate);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void __launch_bounds__(kBlockThreads)
encode_stages_kernel(const double* blocks, int64_t nblocks, int rate, EncOut st, uint64_t* out_w)
{
    __shared__ uint64_t buf[kWaves][kMaxRate];
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * kWaves + wave;
    if (b >= nblocks) return;  // the whole wave leaves together
    uint64_t* words = buf[wave];
    for (int w = lane; w < rate; w += 64) words[w] = 0;
    __builtin_amdgcn_wave_barrier();
    encode_block(blocks[64 * b + lane], rate, words, st, b);
    __builtin_amdgcn_wave_barrier();
    for (int w = lane; w < rate; w += 64) out_w[b * rate + w] = words[w];
}

__global__ void __launch_bounds__(kBlockThreads)
decode_stages_kernel(const uint64_t* in_w, int64_t nblocks, int rate, DecOut st, double* out)
{
    __shared__ uint64_t buf[kWaves][kMaxRate];
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * kWaves + wave;
    if (b >= nblocks) return;
    uint64_t* words = buf[wave];
    for (int w = lane; w < rate; w += 64) words[w] = in_w[b * rate + w];
    __builtin_amdgcn_wave_barrier();
    const double v = decode_block(words, rate, st, b);
    if (out) out[64 * b + lane] = v;
}

}  // namespace codec64

hipError_t launch_codec64_field(bool encode, const double* in_f, double* out_f, const uint64_t* in_w, uint64_t* out_w,
                                int64_t nx, int64_t ny, int64_t nz, int64_t ld_y, int64_t ld_z, int rate,
                                hipStream_t stream)
{
    const int nbx = (int)(nx / 4), nby = (int)(ny / 4);
    const int64_t nblocks = (int64_t)nbx * nby * (nz / 4);
    if (nblocks == 0) return hipSuccess;
    // enough waves to fill the chip several times over; each loops over blocks
    const int64_t groups = std::min<int64_t>((nblocks + codec64::kWaves - 1) / codec64::kWaves, 256 * 64);
    hipLaunchKernelGGL(codec64::field_kernel, dim3((unsigned)groups), dim3(kBlockThreads), 0, stream, encode, in_f,
                       out_f, in_w, out_w, nbx, nby, nblocks, ld_y, ld_z, rate);
    return hipGetLastError();
}

hipError_t launch_codec64_stages(bool encode, const double* blocks, const uint64_t* in_w, int64_t nblocks, int rate,
                                 int32_t* emax, int64_t* q, int64_t* t, uint64_t* u, uint64_t* planes,
                                 uint64_t* out_w, int32_t* bits, double* out, hipStream_t stream)
{
    if (nblocks <= 0) return hipSuccess;
    const unsigned g = (unsigned)((nblocks + codec64::kWaves - 1) / codec64::kWaves);
    if (encode)
        hipLaunchKernelGGL(codec64::encode_stages_kernel, dim3(g), dim3(kBlockThreads), 0, stream, blocks, nblocks,
                           rate, codec64::EncOut{emax, q, t, u, planes, bits}, out_w);
    else
        hipLaunchKernelGGL(codec64::decode_stages_kernel, dim3(g), dim3(kBlockThreads), 0, stream, in_w, nblocks,
                           rate, codec64::DecOut{emax, planes, u, q}, out);
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

extern __shared__ double dyn_lds64[];  // wave tiles: two staged planes

// FP64 tiles are 64 x 8 cells (2 cells per thread). With the FP32 tile's
// 16 rows a thread keeps 4 cells' 9-plane columns of doubles and the kernel
// needs 186 VGPRs (2 waves per SIMD); 8 rows: 116 (4 waves per SIMD).
constexpr int kTileY64 = 8;

__global__ void __launch_bounds__(kBlockThreads) wave_f64_kernel(Job j, int nx, int ny, int nz)
{
    stencil::wave_tile<double, kTileY64>(j, nx, ny, nz, -1, -1, -1, nullptr, nullptr, (int)blockIdx.x, dyn_lds64);
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

// One wave per block (the field kernel's mapping), blocks of the job's layers.
__device__ inline void ring_codec_job(const Job& j, int nx, int ny, int wg, bool encode, uint64_t* words)
{
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    const int nbx = nx >> 2, nby = ny >> 2;
    const int64_t layer_blocks = (int64_t)nbx * nby;
    const int64_t b = (int64_t)wg * kWaves + wave;
    if (b >= (int64_t)((j.z1 - j.z0 + 3) / 4) * layer_blocks) return;  // the whole wave leaves together
    const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby);
    const int layer = (int)(b / layer_blocks);
    const int i = lane & 3, jj = (lane >> 2) & 3, l = lane >> 4;
    double* at = plane64(j.dst, j.z0 + 4 * layer + l) + (int64_t)(4 * by + jj) * nx + 4 * bx + i;
    uint64_t* stage = static_cast<uint64_t*>(j.stage) + b * j.rate;
    if (encode) {
        for (int w = lane; w < j.rate; w += 64) words[w] = 0;
        __builtin_amdgcn_wave_barrier();
        encode_block(*at, j.rate, words);
        __builtin_amdgcn_wave_barrier();
        for (int w = lane; w < j.rate; w += 64) stage[w] = words[w];
    } else {
        for (int w = lane; w < j.rate; w += 64) words[w] = stage[w];
        __builtin_amdgcn_wave_barrier();
        *at = decode_block(words, j.rate);
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
// operation order as the FP64 step above).
__global__ void __launch_bounds__(kBlockThreads) fused64_kernel(LaunchParams p)
{
    __shared__ uint64_t buf[kWaves][kMaxRate];
    const int wg = (int)blockIdx.x;
    int jdx = 0;
    while (jdx + 1 < p.njobs && wg >= p.wg_begin[jdx + 1]) ++jdx;
    const Job& j = p.jobs[jdx];
    const int local = wg - p.wg_begin[jdx];
    switch (j.kind) {
    case JOB_WAVE:
        stencil::wave_tile<double, kTileY64>(j, p.nx, p.ny, p.nz, p.src_x, p.src_y, p.src_z, p.src_table, p.step_ctr,
                                             local, dyn_lds64);
        break;
    case JOB_DECODE: ring_codec_job(j, p.nx, p.ny, local, false, buf[threadIdx.x >> 6]); break;
    case JOB_ENCODE: ring_codec_job(j, p.nx, p.ny, local, true, buf[threadIdx.x >> 6]); break;
    case JOB_COPY_IN: ring_copy_job(j, p.nx, p.ny, local, true); break;
    case JOB_COPY_OUT: ring_copy_job(j, p.nx, p.ny, local, false); break;
    default: break;
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
    case JOB_ENCODE: return (int32_t)(((planes + 3) / 4 * (nx / 4) * (ny / 4) + kWaves - 1) / kWaves);
    case JOB_COPY_IN:
    case JOB_COPY_OUT: {
        const int64_t per_wg = (int64_t)kBlockThreads * kCopy4PerThread;
        return (int32_t)(((2 * plane / 4 + per_wg - 1) / per_wg) * planes);
    }
    default: return 0;
    }
}

}  // namespace codec64

// Stencil and copy jobs first, codec jobs last (as in the FP32 kernel: the
// codec waves fill the slots the others leave).
bool prepare_jobs_f64(LaunchParams& p, const void** func, unsigned* grid, size_t* lds)
{
    Job sorted[kMaxJobs];
    int n = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < p.njobs; ++i)
            if ((p.jobs[i].kind == JOB_DECODE || p.jobs[i].kind == JOB_ENCODE) == (pass == 1)) sorted[n++] = p.jobs[i];
    int32_t total = 0;
    for (int i = 0; i < n; ++i) {
        p.jobs[i] = sorted[i];
        p.wg_begin[i] = total;
        p.jobs[i].wg_count = codec64::job_workgroups64(p.jobs[i], p.nx, p.ny);
        total += p.jobs[i].wg_count;
    }
    p.wg_begin[p.njobs] = total;
    if (total == 0) return false;
    bool wave = false;
    for (int i = 0; i < n; ++i) wave = wave || p.jobs[i].kind == JOB_WAVE;
    *func = reinterpret_cast<const void*>(&codec64::fused64_kernel);
    *grid = (unsigned)total;
    *lds = wave ? stencil::wave_tile_lds<double, codec64::kTileY64>() : 0;
    return true;
}

hipError_t launch_jobs_f64(LaunchParams& p, hipStream_t stream)
{
    const void* func;
    unsigned grid;
    size_t lds;
    if (!prepare_jobs_f64(p, &func, &grid, &lds)) return hipSuccess;
    hipLaunchKernelGGL(codec64::fused64_kernel, dim3(grid), dim3(kBlockThreads), lds, stream, p);
    return hipGetLastError();
}

}  // namespace oocs
