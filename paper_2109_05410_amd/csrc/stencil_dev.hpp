// stencil_dev.hpp -- gfx950 device code of one stencil time level over a
// z-range of planes held in rings (Sec. III: each cell is updated from its
// neighbours; cells outside the grid are zero).
//
// Common mapping: every thread marches a column of cells up the z-range,
// keeping the z-neighbours it needs in registers (3 planes for heat, 9 for
// the wave), so each input plane value is fetched once per column; the
// lanes of a wave cover consecutive x, so every load and store of a plane
// row is one coalesced access; x neighbours come from the adjacent lanes
// (DPP wave shifts) or from a plane staged in LDS, y neighbours from the
// same thread's registers, the rows above and below, or the staged plane
// (see each function).
//
// The FP32 operation order is fixed (see each function) and the file is
// compiled without floating-point contraction, so a cell's value does not
// depend on how the grid is decomposed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace oocs {
namespace stencil {

// Neighbouring lanes' values by data-parallel moves across the whole wave
// (DPP wave_shr:1 / wave_shl:1, a VALU operation) rather than LDS permutes:
// lane_up(v) is lane l-1's v (lane 0 gets 0), lane_down(v) lane l+1's v
// (lane 63 gets 0). Every lane of the wave must execute the call.
__device__ __forceinline__ float lane_up(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_down(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// Heat, 7 points: u' = c + alpha * (((xm+xp) + (ym+yp)) + (zm+zp) - 6c).
// Mapping: a lane owns 4 consecutive x (one float4), a wave one 256-wide
// row segment, a workgroup 4 rows (one per wave); every lane marches up to
// kZChunk planes in z. The x neighbours come from the adjacent lanes by
// wave shifts (the row ends of the wave from two scalar loads), the y
// neighbours from float4 loads of the rows above and below, the z
// neighbours from the lane's own previous planes. A lane loads the inputs
// of NB planes before it computes and stores any of them: the loads of a
// batch are independent of the stores (which the compiler cannot prove for
// ring pointers), so a wave waits on memory once per batch. nx must be a
// multiple of 4.
template <int NB>
__device__ inline void heat_level(const Job& j, int nx, int ny, int nz, float alpha, int wg)
{
    const int lane = (int)(threadIdx.x & 63), row = (int)(threadIdx.x >> 6);
    const int tiles_x = (nx + kHeatTileX - 1) / kHeatTileX;
    const int tiles_y = (ny + kHeatTileY - 1) / kHeatTileY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x0 = (tile % tiles_x) * kHeatTileX + 4 * lane;
    const int y = (tile / tiles_x) * kHeatTileY + row;
    const int z0 = j.z0 + zc * kZChunk;
    const int z1 = min(j.z1, z0 + kZChunk);
    if (y >= ny || z0 >= z1) return;  // uniform over the wave
    const bool act = x0 < nx;
    const bool hy0 = y > 0, hy1 = y + 1 < ny;
    const bool hl = x0 > 0, hr = x0 + 4 < nx;
    const int64_t xy = (int64_t)y * nx + x0;
    const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    auto ld4 = [&](const float* q) { return *reinterpret_cast<const float4*>(q); };
    float4 cm = (act && z0 > 0) ? ld4(ring_plane(j.src, z0 - 1) + xy) : zero;
    for (int zb = z0; zb < z1; zb += NB) {
        float4 c[NB + 1], ym[NB], yp[NB];
        float el[NB], er[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            c[i] = ym[i] = yp[i] = zero;
            el[i] = er[i] = 0.0f;
            if (act && zb + i < z1) {
                const float* pl = ring_plane(j.src, zb + i) + xy;
                c[i] = ld4(pl);
                if (hy0) ym[i] = ld4(pl - nx);
                if (hy1) yp[i] = ld4(pl + nx);
                if (lane == 0 && hl) el[i] = pl[-1];
                if (lane == 63 && hr) er[i] = pl[4];
            }
        }
        // the plane above the last one of the batch
        const int zt = min(zb + NB, z1);
        c[NB] = zero;
#pragma unroll
        for (int i = 1; i <= NB; ++i)
            if (act && zt == zb + i && zt < nz) c[i] = ld4(ring_plane(j.src, zt) + xy);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            float l = lane_up(c[i].w);
            float r = lane_down(c[i].x);
            if (lane == 0) l = el[i];
            if (lane == 63 || !hr) r = hr ? er[i] : 0.0f;
            if (act && zb + i < z1) {
                const float4 zm = i == 0 ? cm : c[i - 1];
                const float4 zp = c[i + 1];
                const float4 cc = c[i];
                float4 o;
                float t;
                t = (l + cc.y) + (ym[i].x + yp[i].x);    t = t + (zm.x + zp.x); t = t - 6.0f * cc.x; o.x = cc.x + alpha * t;
                t = (cc.x + cc.z) + (ym[i].y + yp[i].y); t = t + (zm.y + zp.y); t = t - 6.0f * cc.y; o.y = cc.y + alpha * t;
                t = (cc.y + cc.w) + (ym[i].z + yp[i].z); t = t + (zm.z + zp.z); t = t - 6.0f * cc.z; o.z = cc.z + alpha * t;
                t = (cc.z + r) + (ym[i].w + yp[i].w);    t = t + (zm.w + zp.w); t = t - 6.0f * cc.w; o.w = cc.w + alpha * t;
                *reinterpret_cast<float4*>(ring_plane(j.dst, zb + i) + xy) = o;
            }
        }
        cm = c[NB - 1];
    }
}

// Heat on a dense field with a tile shape chosen at compile time (batched
// domains, any nx): tile TX x TY columns per 256-thread workgroup
// (TX*TY = 256), ZC planes marched per thread, the inputs of 4 planes loaded
// before any is computed. Same operation order as heat_level.
template <int TX, int TY, int ZC>
__device__ __attribute__((always_inline)) inline void heat_dense(const float* __restrict__ src, float* __restrict__ dst,
                                                                 int nx, int ny, int nz, float alpha, int wg)
{
    constexpr int NB = 4;
    const int tiles_x = (nx + TX - 1) / TX;
    const int tiles_y = (ny + TY - 1) / TY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x = (tile % tiles_x) * TX + (int)(threadIdx.x % TX);
    const int y = (tile / tiles_x) * TY + (int)(threadIdx.x / TX);
    const int z0 = zc * ZC;
    const int z1 = min(nz, z0 + ZC);
    if (x >= nx || y >= ny || z0 >= z1) return;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t xy = (int64_t)y * nx + x;
    const bool hx0 = x > 0, hx1 = x + 1 < nx, hy0 = y > 0, hy1 = y + 1 < ny;
    float cm = z0 > 0 ? src[(z0 - 1) * plane + xy] : 0.0f;
    for (int zb = z0; zb < z1; zb += NB) {
        float c[NB + 1], xm[NB], xp[NB], ym[NB], yp[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            c[i] = xm[i] = xp[i] = ym[i] = yp[i] = 0.0f;
            if (zb + i < z1) {
                const float* pl = src + (zb + i) * plane + xy;
                c[i] = pl[0];
                if (hx0) xm[i] = pl[-1];
                if (hx1) xp[i] = pl[1];
                if (hy0) ym[i] = pl[-nx];
                if (hy1) yp[i] = pl[nx];
            }
        }
        const int zt = min(zb + NB, z1);
        c[NB] = 0.0f;
#pragma unroll
        for (int i = 1; i <= NB; ++i)
            if (zt == zb + i && zt < nz) c[i] = src[zt * plane + xy];
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (zb + i < z1) {
                const float zm = i == 0 ? cm : c[i - 1];
                float t = (xm[i] + xp[i]) + (ym[i] + yp[i]);
                t = t + (zm + c[i + 1]);
                t = t - 6.0f * c[i];
                dst[(zb + i) * plane + xy] = c[i] + alpha * t;
            }
        cm = c[NB - 1];
    }
}

// Heat, K steps in one pass (temporal blocking). A 256-thread workgroup owns
// a 64 x TY column tile whose outer K cells on each side are halo
// (recomputed by the neighbouring tiles) and produces level K on planes
// [z0, z1) from level 0, which it streams over [z0 - K, z1 + K). Wave w owns
// the TY/4 consecutive rows [w*TY/4, (w+1)*TY/4) of the tile, one x per lane,
// in every plane; per cell it keeps the last three planes of every
// intermediate level in registers (the z neighbours). A cell's y neighbours
// are in its own registers except across a strip edge, its x neighbours come
// from the adjacent lanes by shuffles, and only the strips' first and last
// rows of each new plane of levels 0..K-1 go through LDS, double-buffered by
// plane parity, so one barrier per plane suffices: level s at plane q = p - s
// reads level s-1 at plane q as written in the previous iteration. Cells
// outside the grid are zero at every level; tile-border cells have no
// neighbours and are set to zero (they are outside the region a level can
// compute). Level K is written for the tile interior. Same per-cell operation
// order as heat_level, so the result equals K single steps bit for bit.
// Planes are addressed through rings (a dense field is a ring of nz
// planes). lds holds K * 2 * 2 * 4 * 64 floats.
template <int TY, int K>
__device__ __attribute__((always_inline)) inline void heat_tb(const Ring& src, const Ring& dst, int nx, int ny,
                                                                     int nz, float alpha, int z0, int z1, int tile,
                                                                     float* lds)
{
    constexpr int TX = 64, CPT = TY / 4, OX = TX - 2 * K, OY = TY - 2 * K;
    static_assert(TY % 4 == 0 && OY > 0 && CPT >= 2, "tile too small for the depth");
    const int tiles_x = (nx + OX - 1) / OX;
    const int ox = (tile % tiles_x) * OX - K, oy = (tile / tiles_x) * OY - K;
    const int lx = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const int gx = ox + lx;
    const bool xin = gx >= 0 && gx < nx;
    const bool xedge = lx == 0 || lx == TX - 1;
    const bool xout = lx >= K && lx < TX - K;
    bool in[CPT], ok_xy[CPT], out_xy[CPT];
    int64_t off[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int ly = wv * CPT + c, gy = oy + ly;
        in[c] = xin && gy >= 0 && gy < ny;
        ok_xy[c] = in[c] && !xedge && ly > 0 && ly < TY - 1;
        out_xy[c] = in[c] && xout && ly >= K && ly < TY - K;
        off[c] = (int64_t)gy * nx + gx;
    }
    // edge rows of the strips: E(lev, buf, side, wave) -> 64 floats; side 0 = first row, 1 = last row
    auto E = [&](int lev, int buf, int side, int wave) -> float* { return lds + (((lev * 2 + buf) * 2 + side) * 4 + wave) * 64; };
    float w[K][CPT][3];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int c = 0; c < CPT; ++c) w[s][c][0] = w[s][c][1] = w[s][c][2] = 0.0f;
    for (int p = z0 - K; p < z1 + K; ++p) {
        const int b = p & 1;
        const bool pin = p >= 0 && p < nz;
        const float* sp = pin ? ring_plane(src, p) : nullptr;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const float v = (in[c] && pin) ? sp[off[c]] : 0.0f;
            w[0][c][0] = w[0][c][1];
            w[0][c][1] = w[0][c][2];
            w[0][c][2] = v;
        }
        E(0, b, 0, wv)[lx] = w[0][0][2];
        E(0, b, 1, wv)[lx] = w[0][CPT - 1][2];
#pragma unroll
        for (int s = 1; s <= K; ++s) {
            const int q = p - s;
            const int qb = q & 1;
            const bool qin = q >= 0 && q < nz;
            const float above = wv > 0 ? E(s - 1, qb, 1, wv - 1)[lx] : 0.0f;       // row w*CPT - 1
            const float below = wv < 3 ? E(s - 1, qb, 0, wv + 1)[lx] : 0.0f;       // row (w+1)*CPT
            float nv[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const float cc = w[s - 1][c][1];
                const float xm = lane_up(cc);
                const float xp = lane_down(cc);
                const float ym = c > 0 ? w[s - 1][c - 1][1] : above;
                const float yp = c < CPT - 1 ? w[s - 1][c + 1][1] : below;
                float v = 0.0f;
                if (ok_xy[c] && qin) {
                    float t = (xm + xp) + (ym + yp);
                    t = t + (w[s - 1][c][0] + w[s - 1][c][2]);
                    t = t - 6.0f * cc;
                    v = cc + alpha * t;
                }
                nv[c] = v;
            }
            if (s < K) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    w[s][c][0] = w[s][c][1];
                    w[s][c][1] = w[s][c][2];
                    w[s][c][2] = nv[c];
                }
                E(s, qb, 0, wv)[lx] = nv[0];
                E(s, qb, 1, wv)[lx] = nv[CPT - 1];
            } else {
#pragma unroll
                for (int c = 0; c < CPT; ++c)
                    if (out_xy[c] && q >= z0 && q < z1) ring_plane(dst, q)[off[c]] = nv[c];
            }
        }
        __syncthreads();
    }
}

// Tiles of heat_tb over an nx x ny plane.
template <int TY, int K>
__host__ __device__ inline int heat_tb_tiles(int nx, int ny)
{
    return ((nx + 64 - 2 * K - 1) / (64 - 2 * K)) * ((ny + TY - 2 * K - 1) / (TY - 2 * K));
}

// Wave, 25 points:
//   acc = C0X3*p;  for m = 1..4: acc = acc + C_m * (((x+m + x-m) + (y+m + y-m)) + (z+m + z-m))
//   p'  = (2p - pm) + w*acc  (+ amp at the source cell)
// Mapping: a workgroup owns a 64 x TY cell tile (each wave 64 lanes x TY/4
// consecutive rows, so a thread has TY/4 cells) and marches up to kZChunk
// planes. Each plane of p, with its 4-cell halo in x and y, is staged
// through LDS, so the 16 x / y neighbours of a cell are LDS reads, and every
// thread keeps its cells' p(z-4 .. z+4) in registers. Two staged planes
// (double buffered): the next plane's loads are issued before the current
// plane is computed; one barrier per plane. (A ring of six staged planes that
// also supplied p(z+4) at the cell, instead of a second read of p, was
// slower: 214 against 237 GCell/s in core at 1024^3, its 41 KiB of LDS
// leaving room for three workgroups per CU instead of four.)
constexpr int kWaveTileW = 64 + 8;
template <int TY = kWaveTileY>
constexpr int wave_tile_plane() { return kWaveTileW * (TY + 8); }  // values of one staged plane
template <typename T = float, int TY = kWaveTileY>
__host__ __device__ constexpr size_t wave_tile_lds() { return 2 * (size_t)wave_tile_plane<TY>() * sizeof(T); }

// T = float: the FP32 pipeline; T = double: FP64 rings (a ring's plane
// stride counts floats, so a plane of doubles is read through a cast).
template <typename T>
__device__ inline T* ring_plane_t(const Ring& r, int64_t z) { return reinterpret_cast<T*>(ring_plane(r, z)); }

// Planes of a ring visited in order z, z+1, ...: the slot advances without
// the division of ring_plane (wave-uniform, so it stays in scalar registers).
template <typename T>
struct PlaneCursor {
    float* base;
    int64_t ld;
    uint32_t W, slot;
    __device__ PlaneCursor(const Ring& r, int z) : base(r.base), ld(r.ld_z), W((uint32_t)r.W), slot((uint32_t)z % (uint32_t)r.W) {}
    __device__ T* plane() const { return reinterpret_cast<T*>(base + (int64_t)slot * ld); }
    __device__ void next() { slot = slot + 1 == W ? 0u : slot + 1; }
};

// TY: tile rows (a multiple of 4); each thread has TY / 4 cells. ZC: planes
// a workgroup marches. PF: the loads of plane z + 1 (p(n-1), w and p(z+5)
// at the thread's cells) are issued before plane z is computed.
template <typename T, int TY = kWaveTileY, int ZC = kZChunk, bool PF = true>
__device__ inline void wave_tile(const Job& j, int nx, int ny, int nz, int sx, int sy, int sz, const float* src_table,
                                 const int32_t* step_ctr, int wg, T* lds)
{
    const T C0X3 = (T)(-205.0 / 24.0);
    const T C1 = (T)(8.0 / 5.0);
    const T C2 = (T)(-1.0 / 5.0);
    const T C3 = (T)(8.0 / 315.0);
    const T C4 = (T)(-1.0 / 560.0);
    const T CM[4] = {C1, C2, C3, C4};
    constexpr int R = TY / 4;                                           // cells per thread
    constexpr int TW = kWaveTileW, TP = wave_tile_plane<TY>();
    const int tiles_x = (nx + 63) / 64;
    const int tiles_y = (ny + TY - 1) / TY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x0 = (tile % tiles_x) * 64, y0 = (tile / tiles_x) * TY;
    const int z0 = j.z0 + zc * ZC;
    const int z1 = min(j.z1, z0 + ZC);
    if (z0 >= z1) return;  // the same for the whole workgroup
    const int tid = (int)threadIdx.x, lx = tid & 63, wv = tid >> 6;
    const int x = x0 + lx;
    // Offsets within a plane are 32-bit byte offsets (planes of the wave hold
    // less than 4 GiB, which the planner and the in-core entry points check),
    // so every load and store is a wave-uniform plane address plus one 32-bit
    // register.
    bool cin[R], srcc[R];
    uint32_t off[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int y = y0 + wv * R + c;
        cin[c] = x < nx && y < ny;
        srcc[c] = j.has_src && x == sx && y == sy;
        off[c] = cin[c] ? (uint32_t)(((uint64_t)y * nx + x) * sizeof(T)) : 0u;
    }
    auto at = [](const T* plane, uint32_t boff) -> const T& {
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + boff);
    };
    // A staged plane is the tile's centre (this workgroup's cells, TY rows of
    // 64) and its 4-cell halo ring. The centre values are p(z') at the
    // thread's own cells, which the thread already holds in its column
    // queue (read as p(z+4) three planes earlier), so only the halo ring is
    // loaded: halo element h = tid + kBlockThreads*i is the h-th cell of the
    // ring (the 4 rows above, the 4 rows below, then 4 columns left and 4
    // right of each centre row).
    constexpr int HALO = TP - 64 * TY;
    constexpr int HPT = (HALO + kBlockThreads - 1) / kBlockThreads;  // halo values per thread
    uint32_t soff[HPT];
    int sidx[HPT];  // position in the staged plane
    bool sok[HPT], shas[HPT];
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
        const int h = tid + kBlockThreads * i;
        int r, cl;
        if (h < 4 * TW) {
            r = h / TW; cl = h % TW;
        } else if (h < 8 * TW) {
            r = TY + 4 + (h - 4 * TW) / TW; cl = (h - 4 * TW) % TW;
        } else {
            const int e = h - 8 * TW;  // side columns: 8 per centre row
            r = 4 + e / 8;
            cl = (e % 8) < 4 ? (e % 8) : 64 + (e % 8);
        }
        shas[i] = h < HALO;
        sidx[i] = shas[i] ? r * TW + cl : 0;
        const int gx = x0 - 4 + cl, gy = y0 - 4 + r;
        sok[i] = shas[i] && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        soff[i] = sok[i] ? (uint32_t)(((uint64_t)gy * nx + gx) * sizeof(T)) : 0u;
    }
    T st[HPT];
    // staged planes are taken in order z0, z0 + 1, ...
    PlaneCursor<T> cs(j.src, z0), cpm(j.src2, z0), cw(j.ro, z0), cd(j.dst, z0);
    auto stage_load = [&](int z) {  // the halo of the cursor's plane, z; planes outside the grid stage as zeros
        const bool zin = z < nz;
        const T* pl = cs.plane();
        cs.next();
#pragma unroll
        for (int i = 0; i < HPT; ++i) st[i] = (zin && sok[i]) ? at(pl, soff[i]) : (T)0;
    };
    T q[R][9];  // q[c][i] = p(z - 4 + i) at cell c
    // the staged halo, and the centre from the column queue entry `at` (this
    // thread's cells of the plane being staged; zero outside the grid)
    auto stage_store = [&](T* t, int at) {
#pragma unroll
        for (int i = 0; i < HPT; ++i)
            if (shas[i]) t[sidx[i]] = st[i];
#pragma unroll
        for (int c = 0; c < R; ++c) t[(wv * R + c + 4) * TW + lx + 4] = q[c][at];
    };
    auto col = [&](int c, int z) -> T { return (cin[c] && z >= 0 && z < nz) ? at(ring_plane_t<T>(j.src, z), off[c]) : (T)0; };
    PlaneCursor<T> ccol(j.src, z0 + 4);  // p(z + 4) at the cell, read plane by plane
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < 8; ++i) q[c][i] = col(c, z0 - 4 + i);
    // p(n-1), w and p(z+4) at the thread's cells, plane by plane
    T npm[R], nw[R], nq[R];
    auto fetch = [&](int z) {
        const T* ppm = cpm.plane();
        const T* pw = cw.plane();
        const T* pc = ccol.plane();
        cpm.next();
        cw.next();
        ccol.next();
        const bool cz = z + 4 < nz;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            nq[c] = (cin[c] && cz) ? at(pc, off[c]) : (T)0;
            npm[c] = cin[c] ? at(ppm, off[c]) : (T)0;
            nw[c] = cin[c] ? at(pw, off[c]) : (T)0;
        }
    };
    if (PF) fetch(z0);
    stage_load(z0);
    stage_store(lds, 4);
    __syncthreads();
    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const bool more = z + 1 < z1;
        if (!PF) fetch(z);
        T pm[R], w[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            q[c][8] = nq[c];
            pm[c] = npm[c];
            w[c] = nw[c];
        }
        if (more) stage_load(z + 1);  // in flight while this plane is computed
        if (PF && more) fetch(z + 1);
        T* pd = cd.plane();
        cd.next();
        const T* t = lds + b * TP + (wv * R + 4) * TW + lx + 4;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const T* tc = t + c * TW;
            T acc = C0X3 * q[c][4];
#pragma unroll
            for (int m = 1; m <= 4; ++m)
                acc = acc + CM[m - 1] * (((tc[m] + tc[-m]) + (tc[m * TW] + tc[-m * TW])) + (q[c][4 + m] + q[c][4 - m]));
            T v = ((T)2 * q[c][4] - pm[c]) + w[c] * acc;
            if (srcc[c] && z == sz) v = v + (T)(src_table ? src_table[*step_ctr + j.src_off] : j.amp);
            if (cin[c]) *reinterpret_cast<T*>(reinterpret_cast<char*>(pd) + off[c]) = v;
        }
        if (more) stage_store(lds + (b ^ 1) * TP, 5);  // plane z + 1
        __syncthreads();
#pragma unroll
        for (int c = 0; c < R; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) q[c][i] = q[c][i + 1];
    }
}

}  // namespace stencil
}  // namespace oocs
