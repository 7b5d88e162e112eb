"""GPU stencil parity: the HIP heat and wave steps equal the oracle's FP32
steps (same operation order) bit for bit, and the FP64 oracle within a
maximum normwise relative error of 1e-5."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2109_05410_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def max_rel(a, b):
    return float(np.max(np.abs(a.astype(np.float64) - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("shape,k", [((64, 64, 64), 10), ((9, 13, 68), 5), ((5, 4, 4), 1), ((12, 8, 132), 0),
                                     ((33, 17, 64), 7)])
def test_heat_matches_oracle(shape, k):
    u0 = inputs.heat_uniform(shape, seed=0)
    u = torch.from_numpy(u0).to(DEV)
    api.heat7_step_k(u, 0.1, k)
    got = u.cpu().numpy()
    assert np.array_equal(got, O.heat7_f32(u0, 0.1, k))
    if k:
        assert max_rel(got, O.heat7_f64(u0.astype(np.float64), 0.1, k)) <= 1e-5


def test_heat_eigenmode_decay():
    shape = (40, 24, 32)
    u0 = inputs.heat_eigenmode(shape, (1, 2, 1))
    u = torch.from_numpy(u0).to(DEV)
    api.heat7_step_k(u, 0.1, 10)
    nz, ny, nx = shape
    lam = 1 - 0.4 * sum(np.sin(np.pi * p / (2 * (n + 1))) ** 2 for p, n in zip((1, 2, 1), (nx, ny, nz)))
    assert max_rel(u.cpu().numpy(), lam ** 10 * u0.astype(np.float64)) <= 1e-5


@pytest.mark.parametrize("shape,k", [((24, 20, 36), 6), ((24, 20, 36), 5), ((16, 12, 72), 1), ((40, 9, 8), 3)])
def test_wave_matches_oracle(shape, k):
    rng = np.random.default_rng(k)
    p0 = rng.standard_normal(shape).astype(np.float32)
    pm0 = rng.standard_normal(shape).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    amps = rng.standard_normal(k).astype(np.float32)
    nz, ny, nx = shape
    cell = (nx // 2, ny // 2, nz // 3)
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    p = torch.from_numpy(p0).to(DEV)
    pm = torch.from_numpy(pm0).to(DEV)
    api.wave25_step_k(p, pm, torch.from_numpy(w).to(DEV), k, src=(amps, cell))
    want_p, want_pm = O.wave25_f32(p0, pm0, w, k, src=(amps, idx))
    assert np.array_equal(p.cpu().numpy(), want_p)
    assert np.array_equal(pm.cpu().numpy(), want_pm)
    ref_p, _ = O.wave25_f64(p0, pm0, w, k, src=(amps, idx))
    assert max_rel(p.cpu().numpy(), ref_p) <= 1e-5


def test_wave_layered_model_ricker_source():
    """The propagation workload's inputs at a small size: zero initial field,
    layered velocity, Ricker source; 60 steps against both oracles."""
    shape = (48, 40, 44)
    v = inputs.layered_velocity(shape, seed=1)
    dt = inputs.wave_dt()
    w = inputs.wave_coefficient(v, dt)
    amps = inputs.ricker(60, dt)
    cell = inputs.source_cell(shape)
    nz, ny, nx = shape
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    z0 = np.zeros(shape, np.float32)
    p = torch.zeros(shape, device=DEV)
    pm = torch.zeros(shape, device=DEV)
    api.wave25_step_k(p, pm, torch.from_numpy(w).to(DEV), 60, src=(amps, cell))
    want_p, _ = O.wave25_f32(z0, z0, w, 60, src=(amps, idx))
    assert np.array_equal(p.cpu().numpy(), want_p)
    ref_p, _ = O.wave25_f64(z0, z0, w, 60, src=(amps, idx))
    assert max_rel(p.cpu().numpy(), ref_p) <= 1e-5
