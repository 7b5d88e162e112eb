"""GPU out-of-core pipeline parity (Sec. III region sharing and temporal
blocking, Sec. V-A separate compression, Sec. V-B pipelined transfers, both
as transfer jobs inside the pipeline kernel and on copy-engine streams).

Small grids that span several slabs, several pipeline groups per slab, a
ragged last residency and rings that wrap: the host store after the run
equals the oracle's replay of the compressed schedule bit for bit (the
oracle's FP32 stencil and codec), and the uncompressed run matches the
FP64 oracle within 1e-5. At the benchmark's full size (512^3, 8 slabs, k=4,
100 steps, 128 MiB device cap) the out-of-core result equals the GPU's
in-core replay bit for bit, and sampled cells equal the oracle computed on
their light cones."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2109_05410_amd import api, inputs

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
        return O.codec_decode(b.view(np.uint64), shape, rate)
    return b.view(np.float32).reshape(shape).copy()


MODES = [(g, m) for m in ("copy", "hybrid", "kernel") for g in (False, True)]
MODE_IDS = [f"{m}-{'graph' if g else 'eager'}" for g, m in MODES]


def xfer(mode):
    """Plan keywords of a transfer mode: copy engines both ways (the default),
    copy-engine loads and kernel stores (hybrid), kernel jobs both ways."""
    return {"copy": {}, "hybrid": {"kernel_stores": True}, "kernel": {"kernel_transfers": True}}[mode]


@pytest.mark.parametrize("graphs,ce", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("rate,k,steps,n,arena", [
    (0, 4, 10, 8, 2 * MiB), (8, 4, 10, 8, 2 * MiB), (16, 4, 9, 4, 3 * MiB), (5, 4, 7, 2, 64 * MiB),
    (0, 3, 8, 4, 2 * MiB),
    (12, 4, 12, 1, 2 * MiB),
])
def test_heat_out_of_core_matches_replay(rate, k, steps, n, arena, graphs, ce):
    shape = (128, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=rate + k)
    plan = api.OutOfCorePlan(shape, api.HEAT7, n, k, [rate], arena, **xfer(ce))
    plan.set_graphs(graphs)
    s = store_of(plan, 0, u0)
    plan.run([s], steps)
    got = decoded(s, shape, rate)
    assert np.array_equal(got, O.replay_heat_f32(u0, 0.1, steps, k, rate))
    assert np.array_equal(plan.get(0, s), got)
    if rate == 0:
        ref = O.heat7_f64(u0.astype(np.float64), 0.1, steps)
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= 1e-5


@pytest.mark.parametrize("graphs,ce", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("rates,k,steps", [([0, 0, 0], 4, 10), ([8, 12, 8], 4, 10), ([16, 16, 16], 3, 7),
                                           ([12, 0, 12], 1, 3),
                                           # the paper's codes 2, 3 and 4 (Sec. VI): one read-write field
                                           # (p(n-1)), the read-only field, both compressed
                                           ([0, 12, 0], 4, 9), ([0, 0, 12], 4, 9), ([0, 12, 12], 4, 9)])
def test_wave_out_of_core_matches_replay(rates, k, steps, graphs, ce):
    shape = (96, 36, 40)
    rng = np.random.default_rng(k)
    p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    amps = rng.standard_normal(steps).astype(np.float32)
    cell = (17, 20, 50)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 2, k, rates, 16 * MiB, src_cell=cell, **xfer(ce))
    plan.set_graphs(graphs)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    nz, ny, nx = shape
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps, idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)
    # the read-only store is never rewritten
    assert np.array_equal(decoded(st[2], shape, rates[2]), O.codec_roundtrip(w, rates[2]) if rates[2] else w)


@pytest.mark.parametrize("graphs,ce", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("rates", [[12, 12, 12], [0, 8, 8], [8, 8, 0]])
def test_resident_read_only_matches_replay(rates, graphs, ce):
    """The read-only field decoded once and kept on the device gives the
    same stores as streaming it; the load is redone after store I/O through
    the arena and for another read-only store."""
    shape = (96, 36, 40)
    rng = np.random.default_rng(3)
    p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    w2 = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    amps = rng.standard_normal(14).astype(np.float32)
    cell = (17, 20, 50)
    idx = cell[0] + shape[2] * (cell[1] + shape[1] * cell[2])
    plan = api.OutOfCorePlan(shape, api.WAVE25, 2, 4, rates, 16 * MiB, src_cell=cell, resident_ro=True, **xfer(ce))
    plan.set_graphs(graphs)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, 9, src_amps=amps[:9])
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, 9, 4, src=(amps[:9], idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)
    # a second read-only store (another velocity model) on the same plan
    st2 = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w2)]
    plan.run(st2, 5, src_amps=amps[9:14])
    wp2, wpm2, _ = O.replay_wave_f32(p0, pm0, w2, 5, 4, src=(amps[9:14], idx), rate_p=rates[0], rate_pm=rates[1],
                                     rate_w=rates[2])
    assert np.array_equal(decoded(st2[0], shape, rates[0]), wp2)
    assert np.array_equal(decoded(st2[1], shape, rates[1]), wpm2)


@pytest.mark.parametrize("graphs,ce", MODES, ids=MODE_IDS)
def test_block_restart_schedule_matches_replay(graphs, ce):
    """The per-block schedule with recomputed halos (Fig. 2) and the shared-level
    schedule give the same bits."""
    shape = (128, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=3)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 8, 4, [8], 2 * MiB, block_restart=True, **xfer(ce))
    plan.set_graphs(graphs)
    s = store_of(plan, 0, u0)
    plan.run([s], 10)
    assert np.array_equal(decoded(s, shape, 8), O.replay_heat_f32(u0, 0.1, 10, 4, 8))
    shape = (96, 36, 40)
    rng = np.random.default_rng(5)
    p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    amps = rng.standard_normal(9).astype(np.float32)
    cell = (17, 20, 50)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 2, 4, [8, 12, 8], 16 * MiB, src_cell=cell, block_restart=True,
                             **xfer(ce))
    plan.set_graphs(graphs)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, 9, src_amps=amps)
    nz, ny, nx = shape
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, 9, 4, src=(amps, idx), rate_p=8, rate_pm=12, rate_w=8)
    assert np.array_equal(decoded(st[0], shape, 8), wp)
    assert np.array_equal(decoded(st[1], shape, 12), wpm)


@pytest.mark.parametrize("rate,k,steps", [(8, 4, 10), (0, 3, 8), (16, 4, 7), (0, 2, 5)])
def test_level_by_level_matches_fused(rate, k, steps):
    """One job per time level (a ring per level) and the temporally blocked
    job per tick (all k levels at once) give the same bits."""
    shape = (128, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=30 + k)
    a_plan = api.OutOfCorePlan(shape, api.HEAT7, 4, k, [rate], 4 * MiB)
    b_plan = api.OutOfCorePlan(shape, api.HEAT7, 4, k, [rate], 4 * MiB, level_by_level=True)
    assert a_plan.info["nrings"] == 2 and b_plan.info["nrings"] == k + 1
    a = store_of(a_plan, 0, u0)
    b = store_of(b_plan, 0, u0)
    a_plan.run([a], steps)
    b_plan.run([b], steps)
    assert torch.equal(a, b)
    assert np.array_equal(decoded(a, shape, rate), O.replay_heat_f32(u0, 0.1, steps, k, rate))


def test_repeated_runs_continue_the_state():
    """Checkpoint/resume: 8 + 5 steps equal 13 steps (k = 4 divides 8); the
    host store between calls is the whole state."""
    shape = (64, 32, 32)
    u0 = inputs.heat_uniform(shape, seed=9)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 4, 4, [8], 4 * MiB)
    s1 = store_of(plan, 0, u0)
    plan.run([s1], 8)
    plan.run([s1], 5)
    s2 = store_of(plan, 0, u0)
    plan.run([s2], 13)
    assert torch.equal(s1, s2)


def test_graph_replays_with_profiling_match_eager():
    """Graph replays (several residencies of each length, profiling timing
    nodes included) give the same store as op-by-op issue."""
    shape = (64, 32, 32)
    u0 = inputs.heat_uniform(shape, seed=4)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 4, 4, [8], 4 * MiB)
    a = store_of(plan, 0, u0)
    b = store_of(plan, 0, u0)
    plan.set_graphs(True)
    plan.set_profiling(True)
    st = plan.run([a], 14)
    assert st.kernel_ms > 0 and st.launches > 0
    plan.set_profiling(False)
    plan.set_graphs(False)
    plan.run([b], 14)
    assert torch.equal(a, b)


def test_stream_waits_match_host_waits():
    """Cross-stream dependencies honoured by stream waits or by host waits
    give the same store, and both equal the replay."""
    shape = (128, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=12)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 8, 4, [8], 2 * MiB)
    a = store_of(plan, 0, u0)
    b = store_of(plan, 0, u0)
    plan.run([a], 14)
    plan.set_host_waits(False)
    plan.run([b], 14)
    assert torch.equal(a, b)
    assert np.array_equal(decoded(a, shape, 8), O.replay_heat_f32(u0, 0.1, 14, 4, 8))


@pytest.mark.parametrize("stencil", ["heat", "wave"])
def test_sdma_writeback_matches_hip_copies(stencil):
    """Write-back copies on an SDMA engine (the default with host waits)
    and through hipMemcpyAsync give the same stores, equal to the replay;
    graph issue and stream waits keep to hipMemcpyAsync."""
    if stencil == "heat":
        shape, rates, k, steps = (128, 64, 64), [8], 4, 14
        fields = [inputs.heat_uniform(shape, seed=21)]
        mk = lambda: api.OutOfCorePlan(shape, api.HEAT7, 8, k, rates, 2 * MiB)  # noqa: E731
    else:
        shape, rates, k, steps = (96, 36, 40), [8, 12, 8], 4, 10
        rng = np.random.default_rng(22)
        fields = [(rng.standard_normal(shape) * 0.1).astype(np.float32),
                  (rng.standard_normal(shape) * 0.1).astype(np.float32),
                  (0.02 + 0.1 * rng.random(shape)).astype(np.float32)]
        mk = lambda: api.OutOfCorePlan(shape, api.WAVE25, 2, k, rates, 16 * MiB)  # noqa: E731
    outs = {}
    for mode in ("sdma", "hip", "graph", "stream", "sdma2", "sdma4"):
        plan = mk()
        assert plan.sdma_available
        plan.set_sdma(mode == "sdma")
        if mode in ("sdma2", "sdma4"):  # every copy split over engines of its own
            plan.set_sdma(int(mode[-1]))
        if mode == "graph":
            plan.set_sdma(True)
            plan.set_graphs(True)
        if mode == "stream":
            plan.set_sdma(True)
            plan.set_host_waits(False)
        st = [store_of(plan, f, a) for f, a in enumerate(fields)]
        r1 = plan.run(st, 8)  # k divides the first call: two calls replay as one
        r2 = plan.run(st, steps - 8)
        if mode.startswith("sdma"):
            assert r1.sdma_copies > 0 and r2.sdma_copies > 0
        else:
            assert r1.sdma_copies == 0 and r2.sdma_copies == 0
        outs[mode] = [s.clone() for s in st]
    for mode in ("hip", "graph", "stream", "sdma2", "sdma4"):
        for a, b in zip(outs["sdma"], outs[mode]):
            assert torch.equal(a, b), mode
    if stencil == "heat":
        assert np.array_equal(decoded(outs["sdma"][0], shape, 8), O.replay_heat_f32(fields[0], 0.1, steps, k, 8))


def test_link_probe_reports_both_engines():
    """The host-link probe runs on the pipeline's engines (SDMA write-back)
    and on hipMemcpyAsync alone, and reports positive rates for each."""
    for sdma in (1, 0, 2, 4):
        r = api.link_probe(32 << 20, 4 << 20, reps=1, sdma=sdma)
        assert r["d2h_engine"] == ("sdma" if sdma else "hipMemcpyAsync")
        assert min(r["h2d_GBps"], r["d2h_GBps"], r["bidir_GBps_each"]) > 1.0


def test_wave_source_longer_than_the_source_table():
    """Runs longer than the device amplitude table are split into chunks of
    whole residencies; the source timing stays exact."""
    from paper_2109_05410_amd import _lib as L  # noqa: F401
    shape = (16, 8, 8)
    steps, k = 65536 + 9, 3
    rng = np.random.default_rng(0)
    w = np.full(shape, 0.05, np.float32)
    amps = rng.standard_normal(steps).astype(np.float32) * 1e-3
    cell = (3, 4, 7)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 1, k, [0, 0, 0], 16 * MiB, src_cell=cell)
    z = np.zeros(shape, np.float32)
    st = [store_of(plan, 0, z), store_of(plan, 1, z), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    p = torch.zeros(shape, device=DEV)
    pm = torch.zeros(shape, device=DEV)
    api.wave25_step_k(p, pm, torch.from_numpy(w).to(DEV), steps, src=(amps, cell))
    assert np.array_equal(decoded(st[0], shape, 0), p.cpu().numpy())


def test_deterministic():
    shape = (64, 32, 32)
    u0 = inputs.heat_uniform(shape, seed=3)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 4, 4, [16], 4 * MiB)
    a = store_of(plan, 0, u0)
    b = store_of(plan, 0, u0)
    plan.run([a], 12)
    plan.run([b], 12)
    assert torch.equal(a, b)


def light_cone_point(u0, steps, z, y, x, alpha=0.1):
    """Oracle FP32 value of one cell after `steps` plain steps, computed on
    the sub-box that holds its light cone (zero ghosts at the real faces;
    the artificial faces are more than `steps` cells away)."""
    nz, ny, nx = u0.shape
    R = steps + 1
    z0, z1 = max(z - R, 0), min(z + R + 1, nz)
    y0, y1 = max(y - R, 0), min(y + R + 1, ny)
    x0, x1 = max(x - R, 0), min(x + R + 1, nx)
    sub = np.ascontiguousarray(u0[z0:z1, y0:y1, x0:x1])
    out = O.heat7_f32(sub, alpha, steps)
    return out[z - z0, y - y0, x - x0]


def heat_light_cone_block_q(u0, rate, k, steps, zb, yb, xb, alpha=0.1):
    """Oracle FP32 values of the 4x4x4 codec block at (zb, yb, xb) after
    `steps` (a multiple of k) steps of the compressed heat schedule (the
    store holds decode(encode()) of u after every k steps), from the block's
    light cone: the box widened by k cells per remaining residency, each a
    union of whole codec blocks when k is a multiple of 4."""
    nz, ny, nx = u0.shape
    m = steps // k
    q = lambda a: O.codec_decode(O.codec_encode(np.ascontiguousarray(a), rate), a.shape, rate)  # noqa: E731

    def box(r):
        return (max(zb - r, 0), min(zb + 4 + r, nz), max(yb - r, 0), min(yb + 4 + r, ny),
                max(xb - r, 0), min(xb + 4 + r, nx))

    z0, z1, y0, y1, x0, x1 = box(k * m)
    u = q(u0[z0:z1, y0:y1, x0:x1])
    for r in range(m):
        u = O.heat7_f32(u, alpha, k)
        a0, a1, b0, b1, c0, c1 = box(k * (m - 1 - r))
        u = q(u[a0 - z0:a1 - z0, b0 - y0:b1 - y0, c0 - x0:c1 - x0])
        z0, z1, y0, y1, x0, x1 = a0, a1, b0, b1, c0, c1
    return u


@pytest.mark.parametrize("rate", [0, 8])
def test_full_size_benchmark_configuration(rate):
    """512^3, 8 slabs of 64 planes, k = 4 (h = 4), 100 steps, device arena
    capped at two slabs (128 MiB): the configuration the benchmark times.
    Compressed: the store equals the GPU's in-core replay bit for bit, and
    sampled codec blocks equal the CPU oracle's values of the same schedule
    on their light cones."""
    shape = (512, 512, 512)
    steps, k = 100, 4
    u0 = inputs.heat_uniform(shape, seed=0)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 8, k, [rate], 128 * MiB)
    assert plan.info["arena_needed"] <= 128 * MiB
    s = store_of(plan, 0, u0)
    plan.run([s], steps)
    got = plan.get(0, s)
    # in-core replay on the GPU with the same kernels (no cap)
    u = torch.from_numpy(u0).to(DEV)
    tmp = torch.empty_like(u)
    if rate:
        u = api.codec_decode(api.codec_encode(u, rate), shape, rate)
    for _ in range(steps // k):
        api.heat7_step_k(u, 0.1, k, tmp=tmp)
        if rate:
            u = api.codec_decode(api.codec_encode(u, rate), shape, rate)
    assert np.array_equal(got, u.cpu().numpy())
    if rate == 0:
        for (z, y, x) in ((0, 0, 0), (63, 255, 300), (64, 17, 511), (300, 500, 2)):
            assert got[z, y, x] == light_cone_point(u0, steps, z, y, x), (z, y, x)
    else:  # codec blocks across a slab boundary and at a corner against the CPU oracle's schedule
        for (zb, yb, xb) in ((60, 256, 300), (508, 508, 0)):
            print(f"oracle block z={zb} y={yb} x={xb}", flush=True)
            want = heat_light_cone_block_q(u0, rate, k, steps, zb, yb, xb)
            assert np.array_equal(got[zb:zb + 4, yb:yb + 4, xb:xb + 4], want), (zb, yb, xb)


_WAVE_FULL = {}


def _wave_full_inputs():
    """1024^3 wave inputs of the benchmark's wave configuration, with
    nonzero initial fields so that every slab boundary carries data."""
    if not _WAVE_FULL:
        shape = (1024, 1024, 1024)
        rng = np.random.default_rng(41)
        dt = inputs.wave_dt()
        _WAVE_FULL.update(
            shape=shape,
            p0=(rng.random(shape, dtype=np.float32) - np.float32(0.5)) * np.float32(1e-2),
            pm0=(rng.random(shape, dtype=np.float32) - np.float32(0.5)) * np.float32(1e-2),
            w=inputs.wave_coefficient(inputs.layered_velocity(shape, seed=1), dt),
            cell=inputs.source_cell(shape),
            amps=inputs.ricker(24, dt),
        )
    return _WAVE_FULL


def wave_light_cone_point(d, steps, z, y, x):
    """Oracle FP32 value of p at one cell after `steps` steps, computed on
    the sub-box holding its light cone (the 25-point star reaches 4 cells
    per step along each axis; the artificial faces are farther than that)."""
    nz, ny, nx = d["shape"]
    R = 4 * steps
    z0, z1 = max(z - R, 0), min(z + R + 1, nz)
    y0, y1 = max(y - R, 0), min(y + R + 1, ny)
    x0, x1 = max(x - R, 0), min(x + R + 1, nx)
    box = lambda a: np.ascontiguousarray(a[z0:z1, y0:y1, x0:x1])  # noqa: E731
    sx, sy, sz = d["cell"]
    src = None
    if z0 <= sz < z1 and y0 <= sy < y1 and x0 <= sx < x1:
        src = (d["amps"][:steps], (sx - x0) + (x1 - x0) * ((sy - y0) + (y1 - y0) * (sz - z0)))
    p, _ = O.wave25_f32(box(d["p0"]), box(d["pm0"]), box(d["w"]), steps, src=src)
    return p[z - z0, y - y0, x - x0]


def wave_light_cone_block_q(d, rate, k, steps, zb, yb, xb):
    """Oracle FP32 values of p on the 4x4x4 codec block at (zb, yb, xb) after
    `steps` (a multiple of k) steps of the compressed schedule: the host
    stores hold decode(encode()) of p and p(n-1) after every k steps, and w is
    quantised once. Worked backwards from the block: after the last k steps
    it needs the quantised state on the block widened by 4k cells (the light
    cone), which needs the state k steps earlier on a box widened by 4k more,
    and so on; every box is a union of whole codec blocks (4k is a multiple
    of 4, and the grid's faces are block faces), so quantising a box equals
    quantising the grid and cutting the box out. Zero ghosts at the real
    faces; the artificial faces are dropped after each residency."""
    nz, ny, nx = d["shape"]
    m = steps // k
    h = 4 * k
    q = lambda a: O.codec_decode(O.codec_encode(np.ascontiguousarray(a), rate), a.shape, rate)  # noqa: E731

    def box(r):  # the block widened by r cells, clipped to the grid
        return (max(zb - r, 0), min(zb + 4 + r, nz), max(yb - r, 0), min(yb + 4 + r, ny),
                max(xb - r, 0), min(xb + 4 + r, nx))

    z0, z1, y0, y1, x0, x1 = box(h * m)
    cut = lambda a: a[z0:z1, y0:y1, x0:x1]  # noqa: E731
    p, pm, w = q(cut(d["p0"])), q(cut(d["pm0"])), q(cut(d["w"]))
    sx, sy, sz = d["cell"]
    for r in range(m):
        src = None
        if z0 <= sz < z1 and y0 <= sy < y1 and x0 <= sx < x1:
            src = (d["amps"][r * k:(r + 1) * k], (sx - x0) + (x1 - x0) * ((sy - y0) + (y1 - y0) * (sz - z0)))
        p, pm = O.wave25_f32(p, pm, w, k, src=src)
        a0, a1, b0, b1, c0, c1 = box(h * (m - 1 - r))
        sl = (slice(a0 - z0, a1 - z0), slice(b0 - y0, b1 - y0), slice(c0 - x0, c1 - x0))
        p, pm, w = q(p[sl]), q(pm[sl]), w[sl]
        z0, z1, y0, y1, x0, x1 = a0, a1, b0, b1, c0, c1
    return p


@pytest.mark.parametrize("policy", ["plain", "bench"])
@pytest.mark.parametrize("rate", [0, 12])
def test_full_size_wave_configuration(rate, policy):
    """1024^3 wave, 8 slabs of 128 planes, k = 12 (h = 48), device arena
    capped at 8 GiB, two residencies (the benchmark's wave configuration;
    "bench": the flags the benchmark runs with, snake sweeps retaining as
    many slabs as the arena holds and the read-only store held in the
    arena): uncompressed, sampled cells on and
    around slab boundaries and near the source equal the oracle on their
    light cones; at 12 bits per value the store equals the GPU's in-core
    replay (12 steps, then decode(encode()) of both time levels; w quantised
    once) bit for bit, and sampled codec blocks (at the source, across a
    slab boundary, at both ends of the retained region, at a corner of the
    grid) equal the CPU oracle's values of the same schedule on their light
    cones."""
    d = _wave_full_inputs()
    shape, steps, k = d["shape"], 24, 12
    flags = {"snake": True, "ro_device_store": True, "retain": api.RETAIN_MAX} if policy == "bench" else {}
    plan = api.OutOfCorePlan(shape, api.WAVE25, 8, k, [rate] * 3, 8 << 30, src_cell=d["cell"], **flags)
    assert plan.info["arena_needed"] <= 8 << 30
    st = [store_of(plan, 0, d["p0"]), store_of(plan, 1, d["pm0"]), store_of(plan, 2, d["w"])]
    plan.run(st, steps, src_amps=d["amps"])
    got = plan.get(0, st[0])
    plan.close()
    del st
    if rate == 0:
        for (z, y, x) in ((127, 5, 1000), (128, 1023, 0), (513, 511, 512), (1023, 700, 300), (20, 512, 512)):
            assert got[z, y, x] == wave_light_cone_point(d, steps, z, y, x), (z, y, x)
    else:
        q = lambda t: api.codec_decode(api.codec_encode(t, rate), shape, rate)  # noqa: E731
        p = q(torch.from_numpy(d["p0"]).to(DEV))
        pm = q(torch.from_numpy(d["pm0"]).to(DEV))
        w = q(torch.from_numpy(d["w"]).to(DEV))
        for r in range(steps // k):
            p, pm = api.wave25_step_k(p, pm, w, k, src=(d["amps"][r * k:(r + 1) * k], d["cell"]))
            p, pm = q(p), q(pm)
        assert np.array_equal(got, p.cpu().numpy())
        del p, pm, w
        for (zb, yb, xb) in ((16, 512, 512), (124, 300, 700), (384, 1020, 64), (640, 0, 512), (1020, 1020, 0)):
            print(f"oracle block z={zb} y={yb} x={xb}", flush=True)
            want = wave_light_cone_block_q(d, rate, k, steps, zb, yb, xb)
            assert np.array_equal(got[zb:zb + 4, yb:yb + 4, xb:xb + 4], want), (zb, yb, xb)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("rate,k,steps,n,arena,lbl,retain", [
    (8, 4, 13, 8, 2 * MiB, False, 0), (0, 4, 10, 4, 2 * MiB, False, 0), (16, 4, 9, 2, 3 * MiB, True, 0),
    (12, 4, 4, 4, 2 * MiB, False, 0), (8, 4, 13, 8, 3 * MiB, False, 4), (0, 4, 10, 4, 3 * MiB, True, 2),
    (12, 4, 17, 8, 5 * MiB, False, 6), (12, 4, 17, 8, 5 * MiB, False, api.RETAIN_MAX),
])
def test_heat_snake_matches_replay(rate, k, steps, n, arena, lbl, retain, graphs):
    """Snake sweeps (alternating direction, the last block, or the last
    `retain` blocks, kept on the device between residencies) give the replay
    bit for bit: odd and even numbers of residencies, a ragged last one, one
    residency only, fused and level-by-level heat, retained regions of half
    the grid, of more (the regions a residency starts and ends with
    overlap) and of the whole grid; a second run on the same plan
    continues."""
    shape = (128, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=30 + rate)
    plan = api.OutOfCorePlan(shape, api.HEAT7, n, k, [rate], arena, snake=True, level_by_level=lbl, retain=retain)
    if retain:
        assert plan.info["retained_planes"] == (128 if retain == api.RETAIN_MAX else 128 // n * retain)
    plan.set_graphs(graphs)
    s = store_of(plan, 0, u0)
    plan.run([s], steps)
    assert np.array_equal(decoded(s, shape, rate), O.replay_heat_f32(u0, 0.1, steps, k, rate))
    plan.run([s], 2 * k)
    want = O.replay_heat_f32(O.replay_heat_f32(u0, 0.1, steps, k, rate), 0.1, 2 * k, k, rate)
    assert np.array_equal(decoded(s, shape, rate), want)


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("rates,resident_ro", [([12, 12, 12], False), ([0, 0, 0], False), ([8, 12, 8], True),
                                               ([0, 12, 12], False)])
def test_wave_snake_matches_replay(rates, resident_ro, graphs):
    shape = (96, 36, 40)
    rng = np.random.default_rng(5)
    p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    steps, k = 17, 4
    amps = rng.standard_normal(steps).astype(np.float32)
    cell = (17, 20, 50)
    idx = cell[0] + shape[2] * (cell[1] + shape[1] * cell[2])
    plan = api.OutOfCorePlan(shape, api.WAVE25, 3, k, rates, 16 * MiB, src_cell=cell, snake=True,
                             resident_ro=resident_ro)
    plan.set_graphs(graphs)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps, idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("rates,retain,ro_dev", [([12, 12, 12], 2, True), ([0, 0, 0], 2, False),
                                                  ([12, 12, 12], 3, True), ([8, 12, 16], api.RETAIN_MAX, True)])
def test_wave_retained_region_matches_replay(rates, retain, ro_dev, graphs):
    """Snake sweeps whose retained region spans two, three or all four
    slabs: the region's planes stay compressed (or raw) in the arena from
    the residency that writes them to the next one, which decodes them
    first (with three slabs the regions a residency starts and ends with
    overlap; with four nothing crosses the link between a call's first and
    last residency); five residencies, a ragged last one, the source inside
    the region; bit for bit the replay."""
    shape = (96, 36, 40)
    rng = np.random.default_rng(6)
    p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    steps, k = 14, 3
    amps = rng.standard_normal(steps).astype(np.float32)
    cell = (17, 20, 70)
    idx = cell[0] + shape[2] * (cell[1] + shape[1] * cell[2])
    plan = api.OutOfCorePlan(shape, api.WAVE25, 4, k, rates, 16 * MiB, src_cell=cell, snake=True, retain=retain,
                             ro_device_store=ro_dev)
    assert plan.info["retained_planes"] == {2: 48, 3: 72, api.RETAIN_MAX: 96}[retain]
    plan.set_graphs(graphs)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    plan.run(st, steps, src_amps=amps)
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps, idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)


@pytest.mark.parametrize("snake", [False, True])
def test_midpoint_pipeline_matches_replay(snake):
    """Plans with mid-point decoding compute the replay in which every
    decode o encode reconstructs mid-points: heat (fused levels) and the
    wave with every field compressed; the store read back by get() too."""
    shape = (128, 64, 64)
    u0 = inputs.heat_uniform(shape, seed=9)
    plan = api.OutOfCorePlan(shape, api.HEAT7, 4, 4, [8], 2 * MiB, midpoint=True, snake=snake)
    s = store_of(plan, 0, u0)
    plan.run([s], 13)
    want = O.replay_heat_f32(u0, 0.1, 13, 4, 8, mid=True)
    assert np.array_equal(O.codec_decode(s.numpy().view(np.uint64), shape, 8, mid=True), want)
    assert np.array_equal(plan.get(0, s), want)
    assert not np.array_equal(want, O.replay_heat_f32(u0, 0.1, 13, 4, 8))

    wshape = (96, 36, 40)
    rng = np.random.default_rng(8)
    p0 = (rng.standard_normal(wshape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(wshape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(wshape)).astype(np.float32)
    amps = rng.standard_normal(13).astype(np.float32)
    cell = (17, 20, 50)
    idx = cell[0] + wshape[2] * (cell[1] + wshape[1] * cell[2])
    wp = api.OutOfCorePlan(wshape, api.WAVE25, 3, 4, [12, 12, 12], 16 * MiB, src_cell=cell, midpoint=True,
                           snake=snake)
    st = [store_of(wp, 0, p0), store_of(wp, 1, pm0), store_of(wp, 2, w)]
    wp.run(st, 13, src_amps=amps)
    rp, rpm, _ = O.replay_wave_f32(p0, pm0, w, 13, 4, src=(amps, idx), rate_p=12, rate_pm=12, rate_w=12, mid=True)
    assert np.array_equal(O.codec_decode(st[0].numpy().view(np.uint64), wshape, 12, mid=True), rp)
    assert np.array_equal(O.codec_decode(st[1].numpy().view(np.uint64), wshape, 12, mid=True), rpm)


@pytest.mark.parametrize("graphs,ce", [(g, m) for m in ("copy", "hybrid") for g in (False, True)],
                         ids=[f"{m}-{'graph' if g else 'eager'}" for m in ("copy", "hybrid") for g in (False, True)])
@pytest.mark.parametrize("rates,snake", [([12, 12, 12], False), ([8, 12, 8], True), ([0, 0, 0], True),
                                         ([0, 12, 12], False)])
def test_device_read_only_store_matches_replay(rates, snake, graphs, ce):
    """The read-only store copied once into the arena and decoded from there
    every residency: the stores equal the replay bit for bit, the host link
    carries nothing of the read-only field after the first run, and a new
    read-only store pointer is copied again."""
    if snake and ce == "hybrid":
        pytest.skip("snake sweeps need copy-engine write-back")
    shape, k, steps = (96, 36, 40), 4, 13
    rng = np.random.default_rng(31)
    p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    w2 = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    amps = rng.standard_normal(steps + 5).astype(np.float32)
    cell = (17, 20, 50)
    kw = dict(src_cell=cell, snake=snake, **xfer(ce))
    ref = api.OutOfCorePlan(shape, api.WAVE25, 2, k, rates, 16 * MiB, **kw)
    plan = api.OutOfCorePlan(shape, api.WAVE25, 2, k, rates, 16 * MiB, ro_device_store=True, **kw)
    plan.set_graphs(graphs)
    sr = [store_of(ref, 0, p0), store_of(ref, 1, pm0), store_of(ref, 2, w)]
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), store_of(plan, 2, w)]
    a = ref.run(sr, steps, src_amps=amps)
    b = plan.run(st, steps, src_amps=amps)
    nz, ny, nx = shape
    idx = cell[0] + nx * (cell[1] + ny * cell[2])
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps[:steps], idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)
    nres = -(-steps // k)
    assert a.h2d_bytes - b.h2d_bytes == nres * plan.store_bytes(2)
    # another read-only store: copied again, results follow it
    s2 = store_of(plan, 2, w2)
    st = [store_of(plan, 0, p0), store_of(plan, 1, pm0), s2]
    plan.run(st, 5, src_amps=amps)
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w2, 5, k, src=(amps[:5], idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(decoded(st[0], shape, rates[0]), wp)
    assert np.array_equal(decoded(st[1], shape, rates[1]), wpm)
