// adjoint_dev.hpp -- gfx950 device code of the discrete adjoint of the
// 25-point wave propagator (misfit gradient with respect to w = (v dt/dx)^2).
//
// With p(t+1) = 2p(t) - p(t-1) + w . L p(t) + s(t), receivers r(t) = S p(t)
// and J = 1/2 sum_t |r(t) - d(t)|^2, the multipliers obey (L symmetric under
// zero ghosts)
//   lam(t) = 2 lam(t+1) - lam(t+2) + L(w . lam(t+1)) + S^T (r(t) - d(t))
// and dJ/dw = sum_t lam(t) . L p(t-1). One launch of adjoint_step computes
// lam(t) (without the receiver term, which a second tiny kernel adds) and
// accumulates grad += lam(t+1) . L p(t), the term of index t+1 of the sum.
//
// FP32 operation order (fixed; compiled without contraction):
//   acc = C0X3*(w*l1); acc = acc + C_m*(((wl[x+m] + wl[x-m]) + (wl[y+m] + wl[y-m])) + (wl[z+m] + wl[z-m]))
//   l0  = (2*l1 - l2) + acc,            wl[q] = w[q]*l1[q]
//   lp  = C0X3*p; lp = lp + C_m*(((p[x+m] + p[x-m]) + (p[y+m] + p[y-m])) + (p[z+m] + p[z-m]))
//   g   = g + l1*lp
// Mapping as the forward level: 64 x 4 thread tiles, each thread marching up
// to kZChunk planes with 9-value register queues for w*l1 and for p.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace oocs {
namespace adjoint {

struct StepArgs {
    const float* l1;  // lam(t+1)
    const float* l2;  // lam(t+2)
    const float* w;
    const float* p;   // p(t)
    float* l0;        // lam(t), out
    float* grad;      // accumulated in place
    int nx, ny, nz;
};

__device__ inline void adjoint_step(const StepArgs& a, int wg)
{
    const float C0X3 = (float)(-205.0 / 24.0);
    const float C1 = (float)(8.0 / 5.0);
    const float C2 = (float)(-1.0 / 5.0);
    const float C3 = (float)(8.0 / 315.0);
    const float C4 = (float)(-1.0 / 560.0);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tiles_x = (nx + kTileX - 1) / kTileX;
    const int tiles_y = (ny + kTileY - 1) / kTileY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x = (tile % tiles_x) * kTileX + (int)(threadIdx.x % kTileX);
    const int y = (tile / tiles_x) * kTileY + (int)(threadIdx.x / kTileX);
    const int z0 = zc * kZChunk;
    const int z1 = min(nz, z0 + kZChunk);
    if (x >= nx || y >= ny || z0 >= z1) return;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t xy = (int64_t)y * nx + x;
    auto wl = [&](int z) -> float {
        if (z < 0 || z >= nz) return 0.0f;
        const int64_t c = z * plane + xy;
        return a.w[c] * a.l1[c];
    };
    auto pp = [&](int z) -> float { return (z >= 0 && z < nz) ? a.p[z * plane + xy] : 0.0f; };
    float u0 = wl(z0 - 4), u1 = wl(z0 - 3), u2 = wl(z0 - 2), u3 = wl(z0 - 1);
    float u4 = wl(z0), u5 = wl(z0 + 1), u6 = wl(z0 + 2), u7 = wl(z0 + 3);
    float q0 = pp(z0 - 4), q1 = pp(z0 - 3), q2 = pp(z0 - 2), q3 = pp(z0 - 1);
    float q4 = pp(z0), q5 = pp(z0 + 1), q6 = pp(z0 + 2), q7 = pp(z0 + 3);
    for (int z = z0; z < z1; ++z) {
        const float u8 = wl(z + 4);
        const float q8 = pp(z + 4);
        const int64_t c = z * plane + xy;
        auto WX = [&](int d) -> float { return (x + d >= 0 && x + d < nx) ? a.w[c + d] * a.l1[c + d] : 0.0f; };
        auto WY = [&](int d) -> float {
            return (y + d >= 0 && y + d < ny) ? a.w[c + (int64_t)d * nx] * a.l1[c + (int64_t)d * nx] : 0.0f;
        };
        auto PX = [&](int d) -> float { return (x + d >= 0 && x + d < nx) ? a.p[c + d] : 0.0f; };
        auto PY = [&](int d) -> float { return (y + d >= 0 && y + d < ny) ? a.p[c + (int64_t)d * nx] : 0.0f; };
        float acc = C0X3 * u4;
        acc = acc + C1 * (((WX(1) + WX(-1)) + (WY(1) + WY(-1))) + (u5 + u3));
        acc = acc + C2 * (((WX(2) + WX(-2)) + (WY(2) + WY(-2))) + (u6 + u2));
        acc = acc + C3 * (((WX(3) + WX(-3)) + (WY(3) + WY(-3))) + (u7 + u1));
        acc = acc + C4 * (((WX(4) + WX(-4)) + (WY(4) + WY(-4))) + (u8 + u0));
        const float l1c = a.l1[c];
        a.l0[c] = (2.0f * l1c - a.l2[c]) + acc;
        float lp = C0X3 * q4;
        lp = lp + C1 * (((PX(1) + PX(-1)) + (PY(1) + PY(-1))) + (q5 + q3));
        lp = lp + C2 * (((PX(2) + PX(-2)) + (PY(2) + PY(-2))) + (q6 + q2));
        lp = lp + C3 * (((PX(3) + PX(-3)) + (PY(3) + PY(-3))) + (q7 + q1));
        lp = lp + C4 * (((PX(4) + PX(-4)) + (PY(4) + PY(-4))) + (q8 + q0));
        a.grad[c] = a.grad[c] + l1c * lp;
        u0 = u1; u1 = u2; u2 = u3; u3 = u4; u4 = u5; u5 = u6; u6 = u7; u7 = u8;
        q0 = q1; q1 = q2; q2 = q3; q3 = q4; q4 = q5; q5 = q6; q6 = q7; q7 = q8;
    }
}

}  // namespace adjoint
}  // namespace oocs
