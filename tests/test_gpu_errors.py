"""Compression error of the out-of-core pipeline against the FP64 oracle
(the plain stencil, no compression, FP64 from the same FP32 inputs), per
rate and step count, with the metrics of Sec. VI-C: normwise max and L2
relative error and the mean point-wise relative error over 100 seeded
points per plane.

These tests report; their bounds are loose sanity checks (finite, more bits
never worse, the uncompressed run within FP32 rounding). What the compressed
path computes is pinned bit for bit by the replay tests; how far that lands
from the exact solution is a property of the method, printed here per rate
and step count up to 4,320 steps."""
import numpy as np
import pytest

import oracle as O
from paper_2109_05410_amd import api, inputs

pytestmark = pytest.mark.gpu
MiB = 1 << 20
STEPS = (100, 1000, 4320)


def store_of(plan, f, field):
    s = plan.new_store(f)
    plan.put(f, field, s)
    return s


def report(name, rate, steps, e):
    print(f"\n{name} rate {rate:2d} steps {steps:5d}: max_rel {e['max_rel']:.3e}  l2_rel {e['l2_rel']:.3e}  "
          f"pointwise_mean_rel {e['pointwise_mean_rel']:.3e}", flush=True)


def check_table(table, rates):
    for s in STEPS:
        for r in rates:
            assert np.isfinite(table[(r, s)]["max_rel"])
        comp = sorted(r for r in rates if r > 0)
        for lo, hi in zip(comp, comp[1:]):  # more bits per value are never worse
            assert table[(hi, s)]["l2_rel"] <= table[(lo, s)]["l2_rel"] * 1.01 + 1e-12


def test_heat_error_per_rate_and_steps():
    """7-point heat, 64^3 uniform [0, 1) from seed 0, 4 slabs, k = 4."""
    shape = (64, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=0)
    refs, u = {}, u0.astype(np.float64)
    done = 0
    for s in STEPS:
        u = O.heat7_f64(u, 0.1, s - done)
        refs[s] = u
        done = s
    table = {}
    rates = (0, 8, 16)
    for rate in rates:
        plan = api.OutOfCorePlan(shape, api.HEAT7, 4, 4, [rate], 8 * MiB)
        st = store_of(plan, 0, u0)
        done = 0
        for s in STEPS:
            plan.run([st], s - done)
            done = s
            e = O.errors(plan.get(0, st), refs[s])
            table[(rate, s)] = e
            report("heat7 64^3", rate, s, e)
    check_table(table, rates)
    assert table[(0, 100)]["max_rel"] <= 1e-5
    assert all(table[(0, s)]["max_rel"] <= 1e-4 for s in STEPS)
    assert all(table[(16, s)]["max_rel"] <= 1e-2 for s in STEPS)


def test_wave_error_per_rate_and_steps():
    """25-point wave, 128 x 64 x 64, layered velocity 1500-4500 m/s, 15 Hz
    Ricker source, dt at CFL 0.4, 2 slabs, k = 8; all three fields at the
    same rate (the read-only w is compressed once)."""
    shape = (128, 64, 64)
    nz, ny, nx = shape
    dt = inputs.wave_dt()
    w = inputs.wave_coefficient(inputs.layered_velocity(shape, seed=1), dt)
    amps = inputs.ricker(STEPS[-1], dt)
    cell = inputs.source_cell(shape, depth=16)
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    z = np.zeros(shape, np.float32)
    refs = {}
    p, pm = z.astype(np.float64), z.astype(np.float64)
    done = 0
    for s in STEPS:
        p, pm = O.wave25_f64(p, pm, w.astype(np.float64), s - done, src=(amps[done:s].astype(np.float64), idx))
        refs[s] = p
        done = s
    table = {}
    rates = (0, 8, 12, 16)
    for rate in rates:
        plan = api.OutOfCorePlan(shape, api.WAVE25, 2, 8, [rate] * 3, 64 * MiB, src_cell=cell)
        st = [store_of(plan, 0, z), store_of(plan, 1, z), store_of(plan, 2, w)]
        done = 0
        for s in STEPS:
            plan.run(st, s - done, src_amps=amps[done:s])
            done = s
            e = O.errors(plan.get(0, st[0]), refs[s])
            table[(rate, s)] = e
            report("wave25 128x64x64", rate, s, e)
    check_table(table, rates)
    assert table[(0, 100)]["max_rel"] <= 1e-5
    assert all(table[(16, s)]["max_rel"] <= 1e-1 for s in STEPS)
