"""Seeded synthetic inputs for the workloads (no stencil or codec arithmetic
here; both the GPU path and the CPU oracle receive these arrays as inputs).

The paper's own velocity model and data are not published (Sec. VI only
states four double datasets of (1152+2*4)^3 cells), so these stand in:
  - heat: uniform [0, 1) noise (the codec's worst case) or a smooth
    Dirichlet eigenmode;
  - wave: a layered velocity model, 1500..4500 m/s in 6 layers with
    seeded interface depths, dx = 10 m, dt at CFL 0.4, a 15 Hz Ricker
    point source.
Arrays are numpy float32 shaped (nz, ny, nx), x fastest.
"""
from __future__ import annotations

import numpy as np


def heat_uniform(shape, seed: int = 0) -> np.ndarray:
    return np.random.default_rng(seed).random(shape, dtype=np.float32)


def heat_eigenmode(shape, p=(1, 2, 1)) -> np.ndarray:
    nz, ny, nx = shape
    sx = np.sin(np.pi * p[0] * (np.arange(nx) + 1) / (nx + 1))
    sy = np.sin(np.pi * p[1] * (np.arange(ny) + 1) / (ny + 1))
    sz = np.sin(np.pi * p[2] * (np.arange(nz) + 1) / (nz + 1))
    return (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).astype(np.float32)


LAYER_VELOCITIES = (1500.0, 2100.0, 2700.0, 3300.0, 3900.0, 4500.0)


def layered_velocity(shape, seed: int = 1, min_thickness: int = 8) -> np.ndarray:
    """Six horizontal layers (constant in x and y), velocities increasing
    with depth z; five interface depths drawn uniformly on (0, nz) from the
    seed, redrawn until every layer is at least `min_thickness` cells."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    nl = len(LAYER_VELOCITIES)
    mt = min(min_thickness, max(1, nz // (2 * nl)))
    for _ in range(10000):
        cuts = np.sort(rng.integers(1, nz, nl - 1))
        edges = np.concatenate([[0], cuts, [nz]])
        if np.all(np.diff(edges) >= mt):
            break
    else:
        edges = np.linspace(0, nz, nl + 1).astype(int)
    v1 = np.empty(nz, dtype=np.float64)
    for i in range(nl):
        v1[edges[i]:edges[i + 1]] = LAYER_VELOCITIES[i]
    return np.broadcast_to(v1[:, None, None], shape).astype(np.float32)


def wave_dt(dx: float = 10.0, vmax: float = LAYER_VELOCITIES[-1], cfl: float = 0.4) -> float:
    """Time step with vmax*dt/dx = cfl."""
    return cfl * dx / vmax


def wave_coefficient(v: np.ndarray, dt: float, dx: float = 10.0) -> np.ndarray:
    """The read-only field w = (v dt / dx)^2 of the propagator."""
    return ((v.astype(np.float64) * dt / dx) ** 2).astype(np.float32)


def ricker(nsteps: int, dt: float, f: float = 15.0, t0: float | None = None, amp: float = 1.0) -> np.ndarray:
    """Ricker wavelet sampled at t = s*dt, s = 0..nsteps-1 (amplitude per step)."""
    t0 = 1.0 / f if t0 is None else t0
    tau = np.arange(nsteps) * dt - t0
    a = (np.pi * f * tau) ** 2
    return (amp * (1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def source_cell(shape, depth: int = 16):
    nz, ny, nx = shape
    return (nx // 2, ny // 2, min(depth, nz - 1))


def sample_points(shape, per_plane: int = 100, seed: int = 0) -> np.ndarray:
    """Flat indices (into a (nz, ny, nx) field) of `per_plane` distinct seeded
    cells in every z-plane, plane after plane (all of a plane's cells if it
    has fewer). The sampling recipe of the point-wise error: 100 cells per
    plane (Sec. VI-C)."""
    nz, ny, nx = shape
    n = nx * ny
    k = min(per_plane, n)
    rng = np.random.default_rng(seed)
    ij = np.stack([rng.choice(n, k, replace=False) for _ in range(nz)]) if nz > 0 else np.zeros((0, k), np.int64)
    return (np.arange(nz, dtype=np.int64)[:, None] * n + ij).reshape(-1)


def batch_sides(n: int = 64, lo: int = 64, hi: int = 384, seed: int = 2) -> np.ndarray:
    """Cube sides of the batched heat domains, uniform in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, n)
