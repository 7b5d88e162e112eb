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

// The product w . lam is formed once, when lam is written (wl0 = w * l0, the
// same FP32 product as w[q] * l1[q] formed at every use), so the L(w . lam)
// stencil reads one array. Mapping as the wave level: a workgroup owns a
// 64 x TY cell tile (each wave 64 lanes x TY/4 consecutive rows) and marches
// up to kZChunk planes; each plane of w . lam(t+1) and of p(t), with its
// 4-cell halo in x and y, is staged through LDS (double buffered, the next
// plane's loads in flight while the current one is computed, one barrier per
// plane), and every thread keeps its cells' z columns of both in registers.
template <int TY>
struct StepTile {
    static constexpr int TW = 64 + 8, TH = TY + 8, TP = TW * TH;  // one staged plane of one array
    static constexpr size_t lds_bytes() { return 4 * (size_t)TP * sizeof(float); }  // 2 arrays x 2 buffers
};

template <int TY>
__device__ inline void adjoint_step(const StepArgs& a, int wg, float* lds)
{
    const float C0X3 = (float)(-205.0 / 24.0);
    const float C1 = (float)(8.0 / 5.0);
    const float C2 = (float)(-1.0 / 5.0);
    const float C3 = (float)(8.0 / 315.0);
    const float C4 = (float)(-1.0 / 560.0);
    const float CM[4] = {C1, C2, C3, C4};
    constexpr int R = TY / 4;
    constexpr int TW = StepTile<TY>::TW, TP = StepTile<TY>::TP;
    constexpr int LPT = (TP + kBlockThreads - 1) / kBlockThreads;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tiles_x = (nx + 63) / 64;
    const int tiles_y = (ny + TY - 1) / TY;
    const int tile = wg % (tiles_x * tiles_y);
    const int zc = wg / (tiles_x * tiles_y);
    const int x0 = (tile % tiles_x) * 64, y0 = (tile / tiles_x) * TY;
    const int z0 = zc * kZChunk;
    const int z1 = min(nz, z0 + kZChunk);
    if (z0 >= z1) return;  // the same for the whole workgroup
    const int64_t plane = (int64_t)nx * ny;
    const int tid = (int)threadIdx.x, lx = tid & 63, wv = tid >> 6;
    const int x = x0 + lx;
    bool cin[R];
    int64_t off[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const int y = y0 + wv * R + c;
        cin[c] = x < nx && y < ny;
        off[c] = (int64_t)y * nx + x;
    }
    int64_t soff[LPT];
    bool sok[LPT];
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
        const int e = tid + kBlockThreads * i;
        const int gx = x0 - 4 + e % TW, gy = y0 - 4 + e / TW;
        sok[i] = e < TP && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        soff[i] = (int64_t)gy * nx + gx;
    }
    float su[LPT], sp[LPT];
    auto stage_load = [&](int z) {
        const float* U = a.wl1 + z * plane;
        const float* P = a.p + z * plane;
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            su[i] = sok[i] ? U[soff[i]] : 0.0f;
            sp[i] = sok[i] ? P[soff[i]] : 0.0f;
        }
    };
    auto stage_store = [&](int buf) {
        float* tu = lds + (2 * buf) * TP;
        float* tp = tu + TP;
#pragma unroll
        for (int i = 0; i < LPT; ++i)
            if (tid + kBlockThreads * i < TP) {
                tu[tid + kBlockThreads * i] = su[i];
                tp[tid + kBlockThreads * i] = sp[i];
            }
    };
    auto colu = [&](int c, int z) -> float { return (cin[c] && z >= 0 && z < nz) ? a.wl1[z * plane + off[c]] : 0.0f; };
    auto colp = [&](int c, int z) -> float { return (cin[c] && z >= 0 && z < nz) ? a.p[z * plane + off[c]] : 0.0f; };
    float u[R][9], q[R][9];  // (w . lam(t+1))(z - 4 + i), p(z - 4 + i) at cell c
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            u[c][i] = colu(c, z0 - 4 + i);
            q[c][i] = colp(c, z0 - 4 + i);
        }
    stage_load(z0);
    stage_store(0);
    __syncthreads();
    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        const bool more = z + 1 < z1;
        if (more) stage_load(z + 1);  // in flight while this plane is computed
        float l1c[R], l2c[R], wc[R], gc[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int64_t o = z * plane + off[c];
            u[c][8] = colu(c, z + 4);
            q[c][8] = colp(c, z + 4);
            l1c[c] = cin[c] ? a.l1[o] : 0.0f;
            l2c[c] = cin[c] ? a.l2[o] : 0.0f;
            wc[c] = cin[c] ? a.w[o] : 0.0f;
            gc[c] = cin[c] ? a.grad[o] : 0.0f;
        }
        const float* tu = lds + (2 * b) * TP + (wv * R + 4) * TW + lx + 4;
        const float* tp = tu + TP;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const float* U = tu + c * TW;
            const float* P = tp + c * TW;
            float acc = C0X3 * u[c][4];
#pragma unroll
            for (int m = 1; m <= 4; ++m)
                acc = acc + CM[m - 1] * (((U[m] + U[-m]) + (U[m * TW] + U[-m * TW])) + (u[c][4 + m] + u[c][4 - m]));
            const float l0 = (2.0f * l1c[c] - l2c[c]) + acc;
            float lp = C0X3 * q[c][4];
#pragma unroll
            for (int m = 1; m <= 4; ++m)
                lp = lp + CM[m - 1] * (((P[m] + P[-m]) + (P[m * TW] + P[-m * TW])) + (q[c][4 + m] + q[c][4 - m]));
            if (cin[c]) {
                const int64_t o = z * plane + off[c];
                a.l0[o] = l0;
                a.wl0[o] = wc[c] * l0;
                a.grad[o] = gc[c] + l1c[c] * lp;
            }
        }
        if (more) stage_store(b ^ 1);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < R; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                u[c][i] = u[c][i + 1];
                q[c][i] = q[c][i + 1];
            }
    }
}

}  // namespace adjoint
}  // namespace oocs
