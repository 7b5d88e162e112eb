// stencil_dev.hpp -- gfx950 device code of one stencil time level over a
// z-range of planes held in rings (Sec. III: each cell is updated from its
// neighbours; cells outside the grid are zero).
//
// Mapping: a 64 x 4 thread tile covers 64 x 4 columns of the xy plane and
// every thread marches up to kZChunk planes in z, keeping the z-neighbours
// it needs in registers (3 planes for heat, 9 for the wave), so each input
// plane value is fetched from memory once per thread column; x and y
// neighbours come through the L1/L2 caches of the neighbouring lanes'
// loads. Lanes of a wave cover 64 consecutive x, so every load and store
// of a plane row is one coalesced 256-byte access.
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

// Heat, 7 points: u' = c + alpha * (((xm+xp) + (ym+yp)) + (zm+zp) - 6c).
__device__ inline void heat_level(const Job& j, int nx, int ny, int nz, float alpha, int wg)
{
    const int tiles_x = (nx + kTileX - 1) / kTileX;
    const int tiles_y = (ny + kTileY - 1) / kTileY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x = (tile % tiles_x) * kTileX + (int)(threadIdx.x % kTileX);
    const int y = (tile / tiles_x) * kTileY + (int)(threadIdx.x / kTileX);
    const int z0 = j.z0 + zc * kZChunk;
    const int z1 = min(j.z1, z0 + kZChunk);
    if (x >= nx || y >= ny || z0 >= z1) return;
    const int64_t xy = (int64_t)y * nx + x;
    auto at = [&](int z) -> const float* { return ring_plane(j.src, z) + xy; };
    float cm = z0 - 1 >= 0 ? *at(z0 - 1) : 0.0f;
    float cc = *at(z0);
    for (int z = z0; z < z1; ++z) {
        const float cp = z + 1 < nz ? *at(z + 1) : 0.0f;
        const float* pl = at(z);
        const float xm = x > 0 ? pl[-1] : 0.0f;
        const float xp = x + 1 < nx ? pl[1] : 0.0f;
        const float ym = y > 0 ? pl[-nx] : 0.0f;
        const float yp = y + 1 < ny ? pl[nx] : 0.0f;
        float s = (xm + xp) + (ym + yp);
        s = s + (cm + cp);
        s = s - 6.0f * cc;
        ring_plane(j.dst, z)[xy] = cc + alpha * s;
        cm = cc;
        cc = cp;
    }
}

// Heat on a dense field with a tile shape chosen at compile time (batched
// domains): tile TX x TY columns per 256-thread workgroup (TX*TY = 256),
// ZC planes marched per thread. Same operation order as heat_level.
template <int TX, int TY, int ZC>
__device__ inline void heat_dense(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny, int nz,
                                  float alpha, int wg)
{
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
    float cm = z0 > 0 ? src[(z0 - 1) * plane + xy] : 0.0f;
    float cc = src[z0 * plane + xy];
    for (int z = z0; z < z1; ++z) {
        const float* pl = src + z * plane + xy;
        const float cp = z + 1 < nz ? pl[plane] : 0.0f;
        const float xm = x > 0 ? pl[-1] : 0.0f;
        const float xp = x + 1 < nx ? pl[1] : 0.0f;
        const float ym = y > 0 ? pl[-nx] : 0.0f;
        const float yp = y + 1 < ny ? pl[nx] : 0.0f;
        float s = (xm + xp) + (ym + yp);
        s = s + (cm + cp);
        s = s - 6.0f * cc;
        dst[z * plane + xy] = cc + alpha * s;
        cm = cc;
        cc = cp;
    }
}

// Wave, 25 points:
//   acc = C0X3*p;  for m = 1..4: acc = acc + C_m * (((x+m + x-m) + (y+m + y-m)) + (z+m + z-m))
//   p'  = (2p - pm) + w*acc  (+ amp at the source cell)
__device__ inline void wave_level(const Job& j, int nx, int ny, int nz, int sx, int sy, int sz,
                                  const float* src_table, const int32_t* step_ctr, int wg)
{
    const float C0X3 = (float)(-205.0 / 24.0);
    const float C1 = (float)(8.0 / 5.0);
    const float C2 = (float)(-1.0 / 5.0);
    const float C3 = (float)(8.0 / 315.0);
    const float C4 = (float)(-1.0 / 560.0);
    const int tiles_x = (nx + kTileX - 1) / kTileX;
    const int tiles_y = (ny + kTileY - 1) / kTileY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x = (tile % tiles_x) * kTileX + (int)(threadIdx.x % kTileX);
    const int y = (tile / tiles_x) * kTileY + (int)(threadIdx.x / kTileX);
    const int z0 = j.z0 + zc * kZChunk;
    const int z1 = min(j.z1, z0 + kZChunk);
    if (x >= nx || y >= ny || z0 >= z1) return;
    const int64_t xy = (int64_t)y * nx + x;
    auto col = [&](int z) -> float { return (z >= 0 && z < nz) ? ring_plane(j.src, z)[xy] : 0.0f; };
    float q0 = col(z0 - 4), q1 = col(z0 - 3), q2 = col(z0 - 2), q3 = col(z0 - 1);
    float q4 = col(z0), q5 = col(z0 + 1), q6 = col(z0 + 2), q7 = col(z0 + 3);
    const bool src_col = j.has_src && x == sx && y == sy;
    for (int z = z0; z < z1; ++z) {
        const float q8 = col(z + 4);
        const float* pl = ring_plane(j.src, z) + xy;
        auto X = [&](int d) -> float { return (x + d >= 0 && x + d < nx) ? pl[d] : 0.0f; };
        auto Y = [&](int d) -> float { return (y + d >= 0 && y + d < ny) ? pl[(int64_t)d * nx] : 0.0f; };
        float acc = C0X3 * q4;
        acc = acc + C1 * (((X(1) + X(-1)) + (Y(1) + Y(-1))) + (q5 + q3));
        acc = acc + C2 * (((X(2) + X(-2)) + (Y(2) + Y(-2))) + (q6 + q2));
        acc = acc + C3 * (((X(3) + X(-3)) + (Y(3) + Y(-3))) + (q7 + q1));
        acc = acc + C4 * (((X(4) + X(-4)) + (Y(4) + Y(-4))) + (q8 + q0));
        const float pm = ring_plane(j.src2, z)[xy];
        const float w = ring_plane(j.ro, z)[xy];
        float v = (2.0f * q4 - pm) + w * acc;
        if (src_col && z == sz) v = v + (src_table ? src_table[*step_ctr + j.src_off] : j.amp);
        ring_plane(j.dst, z)[xy] = v;
        q0 = q1; q1 = q2; q2 = q3; q3 = q4; q4 = q5; q5 = q6; q6 = q7; q7 = q8;
    }
}

}  // namespace stencil
}  // namespace oocs
