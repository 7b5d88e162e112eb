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
                                     ((33, 17, 64), 7), ((40, 200, 300), 5)])
def test_heat_matches_oracle(shape, k):
    """Small fields take the short-chunk one-level launches; the last shape
    (over 2^21 cells, too few workgroups for blocked launches) the level job."""
    u0 = inputs.heat_uniform(shape, seed=0)
    u = torch.from_numpy(u0).to(DEV)
    api.heat7_step_k(u, 0.1, k)
    got = u.cpu().numpy()
    assert np.array_equal(got, O.heat7_f32(u0, 0.1, k))
    if k:
        assert max_rel(got, O.heat7_f64(u0.astype(np.float64), 0.1, k)) <= 1e-5


@pytest.mark.parametrize("k", [6, 9])
def test_heat_blocked_launches_match_oracle(k):
    """A field large enough for the in-core step to take four steps per
    launch with the blocked tiles (over 1024 workgroups), ragged against the
    tiles in every axis; the remainder k mod 4 runs one level per launch."""
    shape = (100, 509, 452)
    u0 = inputs.heat_uniform(shape, seed=11)
    u = torch.from_numpy(u0).to(DEV)
    api.heat7_step_k(u, 0.1, k)
    assert np.array_equal(u.cpu().numpy(), O.heat7_f32(u0, 0.1, k))


def test_heat_full_size_sampled_cells():
    """The in-core step on the 512^3 field (blocked launches), 8 steps, at
    sampled cells: after k steps a cell depends only on the cells within k
    of it, so the oracle on the crop of radius k around it (clipped at the
    domain, whose zero ghosts both sides share) gives its exact value."""
    n, k = 512, 8
    u0 = inputs.heat_uniform((n, n, n), seed=12)
    u = torch.from_numpy(u0).to(DEV)
    api.heat7_step_k(u, 0.1, k)
    got = u.cpu().numpy()
    rng = np.random.default_rng(3)
    pts = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(56)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 3), (n - 1, 0, n - 2), (63, 64, 55), (64, 7, 56),
            (255, 256, 111), (k, n - 1 - k, 200)]
    for z, y, x in pts:
        lo = [max(0, c - k) for c in (z, y, x)]
        hi = [min(n, c + k + 1) for c in (z, y, x)]
        crop = np.ascontiguousarray(u0[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]])
        want = O.heat7_f32(crop, 0.1, k)[z - lo[0], y - lo[1], x - lo[2]]
        assert got[z, y, x] == want, (z, y, x)


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


def test_heat_scratch_argument_checks():
    """A caller-supplied scratch must match u and must not overlap it; with
    a side stream the result is the same as on the current stream."""
    u0 = inputs.heat_uniform((16, 16, 16), seed=2)
    u = torch.from_numpy(u0).to(DEV)
    with pytest.raises(ValueError):
        api.heat7_step_k(u, 0.1, 3, tmp=torch.empty((16, 16, 12), device=DEV))
    with pytest.raises(ValueError):
        api.heat7_step_k(u, 0.1, 3, tmp=u)
    big = torch.empty((2, 16, 16, 16), device=DEV)
    big[0].copy_(u)
    with pytest.raises(ValueError):
        api.heat7_step_k(big[0], 0.1, 3, tmp=big.view(-1)[8:8 + u.numel()].view(16, 16, 16))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    api.heat7_step_k(u, 0.1, 3, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    assert np.array_equal(u.cpu().numpy(), O.heat7_f32(u0, 0.1, 3))
