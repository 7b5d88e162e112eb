// adjoint_dev.hpp -- gfx950 device code of the discrete adjoint of the
// 25-point wave propagator (misfit gradient with respect to w = (v dt/dx)^2).
//
// With p(t+1) = 2p(t) - p(t-1) + w . L p(t) + s(t), receivers r(t) = S p(t)
// and J = 1/2 sum_t |r(t) - d(t)|^2, the multipliers obey (L symmetric under
// zero ghosts)
//   lam(t) = 2 lam(t+1) - lam(t+2) + L(w . lam(t+1)) + S^T (r(t) - d(t))
// and dJ/dw = sum_t lam(t) . L p(t-1). One launch of adjoint_step computes
// lam(t) and w . lam(t) (without the receiver term, which a second tiny
// kernel adds to both) and accumulates grad += lam(t+1) . L p(t), the term
// of index t+1 of the sum.
//
// FP32 operation order (fixed; compiled without contraction):
//   acc = C0X3*(w*l1); acc = acc + C_m*(((wl[x+m] + wl[x-m]) + (wl[y+m] + wl[y-m])) + (wl[z+m] + wl[z-m]))
//   l0  = (2*l1 - l2) + acc,            wl[q] = w[q]*l1[q]
//   lp  = C0X3*p; lp = lp + C_m*(((p[x+m] + p[x-m]) + (p[y+m] + p[y-m])) + (p[z+m] + p[z-m]))
//   g   = g + l1*lp
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace oocs {
namespace adjoint {

struct StepArgs {
    const float* l1;   // lam(t+1)
    const float* wl1;  // w . lam(t+1), element by element (kept beside lam)
    const float* l2;   // lam(t+2)
    const float* w;
    const float* p;    // p(t)
    float* l0;         // lam(t), out
    float* wl0;        // w . lam(t), out (the next step's wl1)
    float* grad;       // accumulated in place
    int nx, ny, nz;
};

// One column (x, y) of a 64 x 4 tile over up to kZChunk planes. The product
// w . lam is formed once, when lam is written (wl0 = w * l0, the same FP32
// product as w[q] * l1[q] formed at every use), so the step reads one array
// for the L(w . lam) stencil instead of two. Each thread keeps the z columns
// of w . lam(t+1) and p(t) in registers and loads the x / y neighbours and the
// point values of NB planes before computing them.
template <int NB>
__device__ inline void adjoint_step(const StepArgs& a, int wg)
{
    const float C0X3 = (float)(-205.0 / 24.0);
    const float C1 = (float)(8.0 / 5.0);
    const float C2 = (float)(-1.0 / 5.0);
    const float C3 = (float)(8.0 / 315.0);
    const float C4 = (float)(-1.0 / 560.0);
    const float CM[4] = {C1, C2, C3, C4};
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
    auto colu = [&](int z) -> float { return (z >= 0 && z < nz) ? a.wl1[z * plane + xy] : 0.0f; };
    auto colp = [&](int z) -> float { return (z >= 0 && z < nz) ? a.p[z * plane + xy] : 0.0f; };
    float u[NB + 8], q[NB + 8];  // u[i] = (w . lam(t+1))(zb - 4 + i), q[i] = p(zb - 4 + i)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        u[i] = colu(z0 - 4 + i);
        q[i] = colp(z0 - 4 + i);
    }
    for (int zb = z0; zb < z1; zb += NB) {
        float ux[NB][8], uy[NB][8], px[NB][8], py[NB][8], l1c[NB], l2c[NB], wc[NB], gc[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            u[8 + i] = q[8 + i] = 0.0f;
            l1c[i] = l2c[i] = wc[i] = gc[i] = 0.0f;
#pragma unroll
            for (int m = 0; m < 8; ++m) ux[i][m] = uy[i][m] = px[i][m] = py[i][m] = 0.0f;
            if (zb + i < z1) {
                const int64_t c = (int64_t)(zb + i) * plane + xy;
                u[8 + i] = colu(zb + i + 4);
                q[8 + i] = colp(zb + i + 4);
                const float* U = a.wl1 + c;
                const float* P = a.p + c;
#pragma unroll
                for (int m = 1; m <= 4; ++m) {
                    if (x + m < nx) { ux[i][2 * m - 2] = U[m]; px[i][2 * m - 2] = P[m]; }
                    if (x - m >= 0) { ux[i][2 * m - 1] = U[-m]; px[i][2 * m - 1] = P[-m]; }
                    if (y + m < ny) { uy[i][2 * m - 2] = U[(int64_t)m * nx]; py[i][2 * m - 2] = P[(int64_t)m * nx]; }
                    if (y - m >= 0) { uy[i][2 * m - 1] = U[-(int64_t)m * nx]; py[i][2 * m - 1] = P[-(int64_t)m * nx]; }
                }
                l1c[i] = a.l1[c];
                l2c[i] = a.l2[c];
                wc[i] = a.w[c];
                gc[i] = a.grad[c];
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (zb + i < z1) {
                float acc = C0X3 * u[i + 4];
#pragma unroll
                for (int m = 1; m <= 4; ++m)
                    acc = acc + CM[m - 1] * (((ux[i][2 * m - 2] + ux[i][2 * m - 1]) + (uy[i][2 * m - 2] + uy[i][2 * m - 1])) +
                                             (u[i + 4 + m] + u[i + 4 - m]));
                const float l0 = (2.0f * l1c[i] - l2c[i]) + acc;
                float lp = C0X3 * q[i + 4];
#pragma unroll
                for (int m = 1; m <= 4; ++m)
                    lp = lp + CM[m - 1] * (((px[i][2 * m - 2] + px[i][2 * m - 1]) + (py[i][2 * m - 2] + py[i][2 * m - 1])) +
                                           (q[i + 4 + m] + q[i + 4 - m]));
                const int64_t c = (int64_t)(zb + i) * plane + xy;
                a.l0[c] = l0;
                a.wl0[c] = wc[i] * l0;
                a.grad[c] = gc[i] + l1c[i] * lp;
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            u[i] = u[i + NB];
            q[i] = q[i + NB];
        }
    }
}

}  // namespace adjoint
}  // namespace oocs
