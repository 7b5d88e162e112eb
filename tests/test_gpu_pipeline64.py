"""GPU out-of-core pipeline in FP64 (the precision of the paper's
experiments, Sec. VI): the wave stencil over rings of doubles with the FP64
block format in the host stores. Small grids spanning several slabs, ragged
last residencies and wrapping rings: the stores after the run equal the
oracle's FP64 replay of the compressed schedule bit for bit, for shared
levels and block restarts, one-way and snake sweeps, streamed and resident
read-only fields, eager launches and graphs; the uncompressed FP64 run
matches the FP64 in-core step bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2109_05410_amd import api

pytestmark = pytest.mark.gpu
DEV = "cuda"
MiB = 1 << 20


def store_of(plan, f, field):
    s = plan.new_store(f)
    plan.put(f, field, s)
    return s


def decoded(store, shape, rate):
    b = store.numpy()
    if rate:
        return O.codec64_decode(b.view(np.uint64), shape, rate)
    return b.view(np.float64).reshape(shape).copy()


def fields(shape, seed, steps):
    rng = np.random.default_rng(seed)
    p0 = rng.standard_normal(shape) * 0.1
    pm0 = rng.standard_normal(shape) * 0.1
    w = 0.02 + 0.1 * rng.random(shape)
    amps = rng.standard_normal(steps).astype(np.float32)  # float amplitudes: exact in double
    return p0, pm0, w, amps


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("rates,k,steps,kw", [
    ([0, 0, 0], 4, 10, {}),
    ([24, 32, 24], 4, 10, {}),
    ([32, 0, 24], 4, 9, {"block_restart": True}),
    ([24, 24, 24], 4, 11, {"snake": True}),
    ([40, 24, 24], 4, 13, {"snake": True, "resident_ro": True}),
    ([68, 12, 1], 2, 5, {}),
    ([24, 24, 32], 4, 13, {"snake": True, "ro_device_store": True}),
    ([24, 24, 32], 4, 13, {"snake": True, "ro_device_store": True, "retain": api.RETAIN_MAX}),
])
def test_fp64_wave_out_of_core_matches_fp64_replay(rates, k, steps, kw, graphs):
    shape = (96, 36, 40)
    p0, pm0, w, amps = fields(shape, k + steps, steps)
    cell = (17, 20, 50)
    print(f"fp64 pipeline: rates={rates} k={k} steps={steps} {kw} graphs={graphs}", flush=True)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 2, k, rates, 16 * MiB, src_cell=cell, fp64=True, **kw)
    plan.set_graphs(graphs)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    nz, ny, nx = shape
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    wp, wpm, _ = O.replay_wave64(p0, pm0, w, steps, k, src=(amps.astype(np.float64), idx), rate_p=rates[0],
                                 rate_pm=rates[1], rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)
    assert np.array_equal(plan.get(0, st[0]), wp)
    # the read-only store is never rewritten
    assert np.array_equal(decoded(st[2], shape, rates[2]), O.codec64_roundtrip(w, rates[2]) if rates[2] else w)


def test_fp64_uncompressed_out_of_core_equals_in_core_step():
    """Larger grid, 4 slabs, k = 6, a wrapping ring: the uncompressed FP64
    pipeline equals the in-core FP64 step bit for bit."""
    shape = (192, 64, 64)
    steps, k = 14, 6
    p0, pm0, w, amps = fields(shape, 5, steps)
    cell = (31, 9, 100)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 4, k, [0, 0, 0], 24 * MiB, src_cell=cell, fp64=True)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    p = torch.from_numpy(p0).to(DEV)
    pm = torch.from_numpy(pm0).to(DEV)
    wd = torch.from_numpy(w).to(DEV)
    api.wave25_step_k_f64(p, pm, wd, steps, src=(amps.astype(np.float64), (cell[0], cell[1], cell[2])))
    torch.cuda.synchronize()
    assert np.array_equal(decoded(st[0], shape, 0), p.cpu().numpy())
    assert np.array_equal(decoded(st[1], shape, 0), pm.cpu().numpy())


@pytest.mark.parametrize("rates,flags", [([24, 24, 24], {"snake": True, "ro_device_store": True}),
                                         ([0, 24, 24], {"snake": True}), ([0, 0, 0], {})])
def test_fp64_at_the_papers_decomposition(rates, flags):
    """The paper's z decomposition (1152 planes, 8 blocks of 144, k = 12,
    halo 48) on a 128 x 128 cross-section, three residencies, the bench's
    flags: the stores equal the GPU's in-core FP64 replay of the compressed
    schedule bit for bit (the replay's own parity with the oracle is pinned
    on small grids above)."""
    shape = (1152, 128, 128)
    steps, k = 36, 12
    p0, pm0, w, amps = fields(shape, 7, steps)
    cell = (64, 64, 16)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 8, k, rates, 256 * MiB, src_cell=cell, fp64=True, **flags)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    p = torch.from_numpy(p0).to(DEV)
    pm = torch.from_numpy(pm0).to(DEV)
    wd = torch.from_numpy(w).to(DEV)
    api.wave64_compressed_run(p, pm, wd, steps, k, src=(amps.astype(np.float64), cell), rate_p=rates[0],
                              rate_pm=rates[1], rate_w=rates[2])
    torch.cuda.synchronize()
    assert np.array_equal(decoded(st[0], shape, rates[0]), p.cpu().numpy())
    assert np.array_equal(decoded(st[1], shape, rates[1]), pm.cpu().numpy())
