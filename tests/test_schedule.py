"""Host logic of the out-of-core pipeline, checked without a GPU.

The planner's per-residency operation list (three streams: host-to-device
copies, compute, device-to-host copies; Sec. V-B) is
  1. checked for races: a vector-clock happens-before analysis over several
     residencies flags any two conflicting accesses (staging slots, ring
     slots, host-store planes) not ordered by stream order or event edges,
     and any two jobs of one fused launch that touch the same ring slot;
  2. executed sequentially in host order with numpy and the oracle's codec,
     and the resulting host store compared bit for bit with the oracle's
     replay of the compressed schedule. Together with 1 this covers every
     legal concurrent execution.
"""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from paper_2109_05410_amd import _lib as L
from paper_2109_05410_amd.api import HEAT7, WAVE25, OutOfCorePlan

MiB = 1 << 20


def xfer(mode):
    """Plan keywords of a transfer mode: copy engines both ways (the default),
    copy-engine loads and kernel stores (hybrid), kernel jobs both ways."""
    return {"copy": {}, "hybrid": {"kernel_stores": True}, "kernel": {"kernel_transfers": True},
            False: {}, True: {"kernel_transfers": True}}[mode]


def plan(shape, stencil, n, k, rates, arena, **kw):
    return OutOfCorePlan(shape, stencil, n, k, rates, arena, planning_only=True, **kw)


# ---------------------------------------------------------------------------
# validation and geometry
# ---------------------------------------------------------------------------

def test_config_errors():
    with pytest.raises(L.OocsError) as e:
        plan((512, 512, 510), HEAT7, 8, 4, [8], 1 << 30)
    assert e.value.code == L.OOCS_E_ALIGN
    with pytest.raises(L.OocsError) as e:
        plan((1024, 64, 64), WAVE25, 16, 12, [0, 0, 0], 1 << 30)   # 2h = 96 > slab 64
    assert e.value.code == L.OOCS_E_HALO
    with pytest.raises(L.OocsError) as e:
        plan((96, 32, 32), HEAT7, 4, 3, [8], 1 << 30)               # h = 3 not a multiple of 4
    assert e.value.code == L.OOCS_E_ALIGN
    with pytest.raises(L.OocsError) as e:
        plan((64, 32, 32), HEAT7, 4, 4, [35], 1 << 30)
    assert e.value.code == L.OOCS_E_RATE
    with pytest.raises(L.OocsError) as e:
        plan((512, 512, 512), HEAT7, 8, 4, [0], 4 * MiB)
    assert e.value.code == L.OOCS_E_CAP
    with pytest.raises(L.OocsError) as e:
        plan((100, 32, 32), HEAT7, 8, 4, [0], 1 << 30)              # 8 does not divide 100
    assert e.value.code == L.OOCS_E_ARG


@pytest.mark.parametrize("rate", [0, 8, 16])
def test_heat_512_fits_two_slab_cap(rate):
    """512^3 FP32 in 8 slabs of 64 MiB with the device capped at two slabs."""
    p = plan((512, 512, 512), HEAT7, 8, 4, [rate], 128 * MiB)
    info = p.info
    assert info["halo"] == 4 and info["arena_needed"] <= 128 * MiB
    assert info["group"] % 4 == 0 and info["group"] >= 4


@pytest.mark.parametrize("rate", [0, 8, 12, 16])
def test_wave_1024_fits_8gib_cap(rate):
    p = plan((1024, 1024, 1024), WAVE25, 8, 12, [rate, rate, rate], 8 << 30)
    info = p.info
    assert info["halo"] == 48 and info["arena_needed"] <= 8 << 30


def test_slab_chunks_partition_the_axis_and_the_store():
    p = plan((1024, 64, 64), WAVE25, 8, 12, [12, 12, 8], 1 << 30)
    prev_end = 0
    for i in range(8):
        s = p.slab(i)
        assert s["z1"] - s["z0"] == 128
        assert s["r0"] == prev_end
        assert s["r1"] == s["c0"]
        prev_end = s["c1"]
        if i < 7:
            assert (s["c0"], s["c1"]) == (s["z1"] - 48, s["z1"] + 48)
        for f, rate in enumerate((12, 12, 8)):
            per_plane = (64 // 4) * (64 // 4) * rate * 8 // 4  # one 4-plane layer of blocks / 4
            assert s["r_off"][f] == s["r0"] * per_plane
            assert s["r_bytes"][f] == (s["r1"] - s["r0"]) * per_plane
    assert prev_end == 1024
    assert p.store_bytes(0) == 1024 * 64 * 64 * 12 // 8
    assert p.store_bytes(2) == 1024 * 64 * 64 * 8 // 8


def test_region_sharing_loads_each_plane_once_per_residency():
    """Every input plane crosses the host link once per residency: the
    common regions are not transferred twice (Sec. III, Fig. 2)."""
    for shape, st, n, k, rates in (((512, 64, 64), HEAT7, 8, 4, [8]), ((1024, 32, 32), WAVE25, 8, 12, [8, 8, 8])):
        p = plan(shape, st, n, k, rates, 1 << 30)
        ops = p.schedule(k)
        for f in range(len(rates)):
            planes = np.zeros(shape[0], dtype=int)
            for o in ops:
                if o["kind"] in (L.OP_H2D, L.OP_FETCH) and o["field"] == f:
                    planes[o["z0"]:o["z1"]] += 1
            assert np.all(planes == 1)
        for f in ([0] if st == HEAT7 else [0, 1]):
            planes = np.zeros(shape[0], dtype=int)
            for o in ops:
                if o["kind"] in (L.OP_D2H, L.OP_STORE) and o["field"] == f:
                    planes[o["z0"]:o["z1"]] += 1
            assert np.all(planes == 1)


def test_separate_write_back_pairs_remainder_and_previous_common_region():
    """With block restarts, after block i the planes written back are
    C_{i-1} (upper half) and R_i, and the lower half of C_i (Fig. 3b): the
    write-back of block i covers [a_i, a_{i+1}) and nothing else. (With
    shared levels the planes leave as soon as they are final, in 4-plane
    aligned groups; every plane once, tested above.)"""
    for ce in ("copy", "hybrid", "kernel"):
        p = plan((512, 32, 32), HEAT7, 8, 4, [8], 1 << 30, **xfer(ce), block_restart=True)
        for o in p.schedule(4):
            if o["kind"] in (L.OP_D2H, L.OP_STORE):
                assert 64 * o["block"] <= o["z0"] < o["z1"] <= 64 * (o["block"] + 1)
                assert o["z0"] % 4 == 0 and o["z1"] % 4 == 0


# ---------------------------------------------------------------------------
# race detector
# ---------------------------------------------------------------------------

class Geometry:
    def __init__(self, p: OutOfCorePlan):
        self.info = p.info
        self.nz = p.shape[0]
        self.r = self.info["radius"]
        self.W = self.info["ring_planes"]
        self.wave = p.stencil == WAVE25
        self.nin = 2 if self.wave else 1
        self.k = p.cfg.k
        self.ro = self.nin + self.k
        self.nslabs = p.cfg.nslabs
        self.nstage = self.info["nstage"]
        self.X = self.info["retained_planes"]

    def ret_base(self, encode, variant):
        """First plane of the retained region that a decode or an encode of
        a residency with this schedule variant addresses: the region it
        starts with (bottom upward, top downward) or the one it ends with;
        plane z sits at z - base in the buffer."""
        return self.nz - self.X if encode != bool(variant & L.OOCS_SCHED_MIRROR) else 0


def accesses(o, g, variant=0):
    """(resource, is_write) pairs of one op of a residency with schedule
    variant `variant`."""
    K = o["kind"]
    out = []
    if K in (L.OP_H2D, L.OP_FETCH):
        out.append((("in", o["field"], o["slot"]), True))
        out += [(("host", o["field"], z), False) for z in range(o["z0"], o["z1"])]
    elif K in (L.OP_D2H, L.OP_STORE):
        out.append((("out", o["field"], o["slot"]), False))
        out += [(("host", o["field"], z), True) for z in range(o["z0"], o["z1"])]
    elif K == L.OP_DECODE:
        if o["slot"] == L.OOCS_SLOT_RETAINED:  # planes of the retained region, at their place in the buffer
            base = g.ret_base(False, variant)
            assert 0 <= o["z0"] - base and o["z1"] - base <= g.X, "outside the retained buffer"
            out += [(("ret", o["field"], z - base), False) for z in range(o["z0"], o["z1"])]
        elif o["slot"] == L.OOCS_SLOT_DEVICE_STORE:  # the device copy of the read-only store (never written)
            out += [(("devstore", o["field"], z), False) for z in range(o["z0"], o["z1"])]
        else:
            out.append((("in", o["field"], o["slot"]), False))
        R = o["level"]
        out += [(("ring", R, z % g.W[R]), True) for z in range(o["z0"], o["z1"])]
    elif K == L.OP_ENCODE:
        if o["slot"] == L.OOCS_SLOT_RETAINED:
            base = g.ret_base(True, variant)
            assert 0 <= o["z0"] - base and o["z1"] - base <= g.X, "outside the retained buffer"
            out += [(("ret", o["field"], z - base), True) for z in range(o["z0"], o["z1"])]
        else:
            out.append((("out", o["field"], o["slot"]), True))
        R = o["level"]
        out += [(("ring", R, z % g.W[R]), False) for z in range(o["z0"], o["z1"])]
    elif K == L.OP_LEVEL:
        lv, steps = o["level"], max(o["slot"], 1)
        for z in range(max(o["z0"] - g.r * steps, 0), min(o["z1"] + g.r * steps, g.nz)):
            out.append((("ring", lv - 1, z % g.W[lv - 1]), False))
        if g.wave:
            for z in range(o["z0"], o["z1"]):
                out.append((("ring", lv - 2, z % g.W[lv - 2]), False))
                out.append((("ring", g.ro, z % g.W[g.ro]), False))
        out += [(("ring", lv, z % g.W[lv]), True) for z in range(o["z0"], o["z1"])]
    return out


def race_check(p: OutOfCorePlan, steps: int, graph_mode: bool = False):
    """graph_mode: each residency is one graph replay, so everything of the
    previous residency is complete before it starts, and only edges recorded
    inside the residency order its own work."""
    g = Geometry(p)
    ns, n = g.nstage, g.nslabs
    vc = [[0, 0, 0] for _ in range(3)]
    ev_clock = {}
    last_write = {}   # resource -> (stream, stamp, launch_id)
    reads = {}        # resource -> list of (stream, stamp, launch_id)
    pending = []      # compute jobs of the current launch
    launch_id = [0]

    def hb(a_stream, a_stamp, b_stream):
        return vc[b_stream][a_stream] >= a_stamp

    def access(res, write, stream, stamp, lid):
        lw = last_write.get(res)
        if lw is not None:
            s, t, l = lw
            if s == stream:
                assert not (stream == 1 and l == lid), f"write/access in one launch on {res}"
            else:
                assert hb(s, t, stream), f"unordered access after write on {res}"
        if write:
            for s, t, l in reads.get(res, []):
                if s == stream:
                    assert not (stream == 1 and l == lid), f"read/write in one launch on {res}"
                else:
                    assert hb(s, t, stream), f"write not ordered after read on {res}"
            last_write[res] = (stream, stamp, lid)
            reads[res] = []
        else:
            reads.setdefault(res, []).append((stream, stamp, lid))

    done, rnd = 0, 0
    nres = -(-steps // g.k)
    while done < steps:
        kr = min(g.k, steps - done)
        par = rnd % 2
        if graph_mode:
            vc = [[0, 0, 0] for _ in range(3)]
            ev_clock.clear()
            last_write.clear()
            reads.clear()

        def phys(e):
            if e < 4 * ns:
                return e
            i = e - 4 * ns
            prev = i >= n
            if prev:
                i -= n
            return ("blk", (1 - par) if prev else par, i)

        var = p.variant(rnd, nres)
        for o in p.schedule(kr, var):
            s = o["stream"]
            K = o["kind"]
            if K == L.OP_RECORD:
                ev_clock[phys(o["event"])] = list(vc[s])
            elif K == L.OP_WAIT:
                if o["event"] >= 4 * ns + n and (rnd == 0 or graph_mode):
                    continue
                c = ev_clock.get(phys(o["event"]))
                if c is not None:
                    vc[s] = [max(a, b) for a, b in zip(vc[s], c)]
            elif K in (L.OP_DECODE, L.OP_LEVEL, L.OP_ENCODE, L.OP_FETCH, L.OP_STORE):
                assert s == 1
                pending.append(o)
            elif K == L.OP_LAUNCH:
                vc[1][1] += 1
                launch_id[0] += 1
                # gather the launch's accesses, then check them together
                acc = []
                for j in pending:
                    acc += accesses(j, g, var)
                writes = {}
                for res, w in acc:
                    if w:
                        assert res not in writes, f"two writes of {res} in one launch"
                        writes[res] = True
                for res, w in acc:
                    if not w:
                        assert res not in writes, f"read and write of {res} in one launch"
                for res, w in acc:
                    access(res, w, 1, vc[1][1], launch_id[0])
                pending.clear()
            else:  # copies
                vc[s][s] += 1
                for res, w in accesses(o, g, var):
                    access(res, w, s, vc[s][s], -1)
        assert not pending
        done += kr
        rnd += 1


@pytest.mark.parametrize("shape,st,n,k,rates,arena,steps", [
    ((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, 11),
    ((48, 12, 16), HEAT7, 4, 2, [0], 1 * MiB // 4, 9),
    ((64, 12, 12), WAVE25, 2, 3, [8, 12, 8], 4 * MiB, 8),
    ((64, 12, 12), WAVE25, 2, 3, [0, 0, 0], 4 * MiB, 7),
    ((512, 32, 32), HEAT7, 8, 4, [8], 4 * MiB, 12),
    ((1024, 16, 16), WAVE25, 8, 12, [8, 8, 8], 64 * MiB, 36),
])
@pytest.mark.parametrize("restart,ce", [(r, m) for r in (False, True) for m in ("copy", "hybrid", "kernel")])
def test_schedule_has_no_races(shape, st, n, k, rates, arena, steps, restart, ce):
    p = plan(shape, st, n, k, rates, arena, src_cell=(3, 3, 5) if st == WAVE25 else None, block_restart=restart,
             **xfer(ce))
    race_check(p, steps)
    race_check(p, steps, graph_mode=True)


@pytest.mark.parametrize("restart,ce", [(r, m) for r in (False, True) for m in ("copy", "hybrid", "kernel")])
def test_full_size_heat_schedule_has_no_races(restart, ce):
    p = plan((512, 512, 512), HEAT7, 8, 4, [8], 128 * MiB, block_restart=restart, **xfer(ce))
    race_check(p, 12)
    race_check(p, 12, graph_mode=True)


@pytest.mark.parametrize("shape,st,n,k,rates", [((512, 64, 64), HEAT7, 8, 4, [8]),
                                                ((1024, 32, 32), WAVE25, 8, 12, [8, 8, 8])])
def test_level_work_with_and_without_block_restarts(shape, st, n, k, rates):
    """Shared levels compute every plane of every level once per residency;
    block restarts compute each block's shrinking extended range
    [a_i - h + s r, a_{i+1} + h - s r) at step s (Fig. 2), so the halo
    planes are computed twice."""
    nz = shape[0]
    slab = nz // n
    r = 1 if st == HEAT7 else 4
    h = r * k
    nin = 1 if st == HEAT7 else 2
    for restart in (False, True):
        p = plan(shape, st, n, k, rates, 1 << 30, block_restart=restart, level_by_level=True)
        cover = {}
        for o in p.schedule(k):
            if o["kind"] == L.OP_LEVEL:
                c = cover.setdefault(o["level"], np.zeros(nz, dtype=int))
                c[o["z0"]:o["z1"]] += 1
        assert sorted(cover) == list(range(nin, nin + k))
        for lv, c in cover.items():
            s = lv - nin + 1
            want = np.zeros(nz, dtype=int)
            if restart:
                for i in range(n):
                    want[max(i * slab - h + s * r, 0):min((i + 1) * slab + h - s * r, nz)] += 1
            else:
                want[:] = 1
            assert np.array_equal(c, want), (restart, lv)
    if st == HEAT7:  # fused levels: one job per tick advances its planes all k steps
        p = plan(shape, st, n, k, rates, 1 << 30)
        assert p.info["nrings"] == 2
        cover = np.zeros(nz, dtype=int)
        for o in p.schedule(k):
            if o["kind"] == L.OP_LEVEL:
                assert o["level"] == 1 and o["slot"] == k
                cover[o["z0"]:o["z1"]] += 1
        assert np.all(cover == 1)


# ---------------------------------------------------------------------------
# sequential execution with numpy + the oracle codec
# ---------------------------------------------------------------------------

C0X3 = np.float32(-205.0 / 24.0)
CM = [None, np.float32(8.0 / 5.0), np.float32(-1.0 / 5.0), np.float32(8.0 / 315.0), np.float32(-1.0 / 560.0)]


def shift(a, d, axis):
    """a shifted so that out[i] = a[i + d] along axis, zeros outside."""
    out = np.zeros_like(a)
    n = a.shape[axis]
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if d >= 0:
        src[axis] = slice(d, n)
        dst[axis] = slice(0, n - d)
    else:
        src[axis] = slice(0, n + d)
        dst[axis] = slice(-d, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


C0X3_64 = -205.0 / 24.0
CM_64 = [None, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0]


def execute(p: OutOfCorePlan, store, steps, src_amps, alpha=np.float32(0.1)):
    """FP32 arithmetic and format, or FP64 for an fp64 plan."""
    g = Geometry(p)
    nz, ny, nx = p.shape
    rates = list(p.cfg.rate)
    f64 = bool(p.cfg.flags & L.OOCS_PLAN_FP64)
    dt = np.float64 if f64 else np.float32
    enc = O.codec64_encode if f64 else O.codec_encode
    dec = O.codec64_decode if f64 else O.codec_decode
    c0x3, cm, two = (C0X3_64, CM_64, 2.0) if f64 else (C0X3, CM, np.float32(2.0))
    rings = [np.zeros((w, ny, nx), dt) for w in g.W]
    stage_in, stage_out = {}, {}
    sx, sy, sz = p.cfg.src_x, p.cfg.src_y, p.cfg.src_z
    layer_words = lambda rate: (nx // 4) * (ny // 4) * rate

    def plane(R, z):
        if z < 0 or z >= nz:
            return np.zeros((ny, nx), dt)
        return rings[R][z % g.W[R]]

    if p.cfg.flags & L.OOCS_PLAN_RESIDENT_RO:  # decoded once, before the residencies
        rings[g.ro][:nz] = dec(store[2], p.shape, rates[2]) if rates[2] else store[2]
    # snake: the retained buffer, (field, place) -> the share of the plane
    # at that place (words of its 4-plane layer, or raw); plane z of the
    # region an op addresses sits at z - base
    retained = {}

    done, rnd = 0, 0
    nres = -(-steps // g.k)
    while done < steps:
        kr = min(g.k, steps - done)
        var = p.variant(rnd, nres)
        for o in p.schedule(kr, var):
            K = o["kind"]
            z0, z1 = o["z0"], o["z1"]
            if K == L.OP_DECODE and o["slot"] == L.OOCS_SLOT_DEVICE_STORE:
                f, rate = o["field"], rates[o["field"]]
                lw = layer_words(rate)
                data = store[f][z0 // 4 * lw: z1 // 4 * lw] if rate else store[f][z0:z1]
                planes = dec(data, (z1 - z0, ny, nx), rate) if rate else data
                for z in range(z0, z1):
                    rings[o["level"]][z % g.W[o["level"]]] = planes[z - z0]
                continue
            if K == L.OP_DECODE and o["slot"] == L.OOCS_SLOT_RETAINED:
                f, rate = o["field"], rates[o["field"]]
                b = g.ret_base(False, var)
                assert 0 <= z0 - b and z1 - b <= g.X
                if rate:
                    data = np.concatenate([retained[(f, z - b)] for z in range(z0, z1, 4)])
                    planes = dec(data, (z1 - z0, ny, nx), rate)
                else:
                    planes = np.stack([retained[(f, z - b)] for z in range(z0, z1)])
                for z in range(z0, z1):
                    rings[o["level"]][z % g.W[o["level"]]] = planes[z - z0]
                continue
            if K == L.OP_ENCODE and o["slot"] == L.OOCS_SLOT_RETAINED:
                f, rate = o["field"], rates[o["field"]]
                b = g.ret_base(True, var)
                assert 0 <= z0 - b and z1 - b <= g.X
                planes = np.stack([plane(o["level"], z) for z in range(z0, z1)])
                if rate:
                    words = enc(planes, rate)
                    lw = layer_words(rate)
                    for q, z in enumerate(range(z0, z1, 4)):
                        retained[(f, z - b)] = words[q * lw:(q + 1) * lw]
                else:
                    for z in range(z0, z1):
                        retained[(f, z - b)] = planes[z - z0].copy()
                continue
            if K in (L.OP_H2D, L.OP_FETCH):
                f, rate = o["field"], rates[o["field"]]
                if rate:
                    stage_in[(f, o["slot"])] = store[f][z0 // 4 * layer_words(rate): z1 // 4 * layer_words(rate)].copy()
                else:
                    stage_in[(f, o["slot"])] = store[f][z0:z1].copy()
            elif K == L.OP_DECODE:
                f, rate = o["field"], rates[o["field"]]
                data = stage_in[(f, o["slot"])]
                planes = dec(data, (z1 - z0, ny, nx), rate) if rate else data
                for z in range(z0, z1):
                    rings[o["level"]][z % g.W[o["level"]]] = planes[z - z0]
            elif K == L.OP_LEVEL and o["slot"] > 1:
                # fused heat levels: `slot` steps from ring lv-1 to ring lv over
                # [z0, z1), intermediate levels on the shrinking z ranges
                lv, nsteps = o["level"], o["slot"]
                cur = {z: plane(lv - 1, z) for z in range(z0 - nsteps, z1 + nsteps)}
                for s_ in range(1, nsteps + 1):
                    lo_, hi_ = z0 - (nsteps - s_), z1 + (nsteps - s_)
                    nxt = {}
                    for z in range(lo_, hi_):
                        if z < 0 or z >= nz:
                            nxt[z] = np.zeros((ny, nx), np.float32)
                            continue
                        c = cur[z]
                        t_ = (shift(c, -1, 1) + shift(c, 1, 1)) + (shift(c, -1, 0) + shift(c, 1, 0))
                        t_ = t_ + (cur[z - 1] + cur[z + 1])
                        t_ = t_ - np.float32(6.0) * c
                        nxt[z] = c + alpha * t_
                    cur = nxt
                for z in range(z0, z1):
                    rings[lv][z % g.W[lv]] = cur[z]
            elif K == L.OP_LEVEL:
                lv = o["level"]
                for z in range(z0, z1):
                    c = plane(lv - 1, z)
                    if not g.wave:
                        s = (shift(c, -1, 1) + shift(c, 1, 1)) + (shift(c, -1, 0) + shift(c, 1, 0))
                        s = s + (plane(lv - 1, z - 1) + plane(lv - 1, z + 1))
                        s = s - np.float32(6.0) * c
                        v = c + alpha * s
                    else:
                        acc = c0x3 * c
                        for m in range(1, 5):
                            sm = (shift(c, m, 1) + shift(c, -m, 1)) + (shift(c, m, 0) + shift(c, -m, 0))
                            sm = sm + (plane(lv - 1, z + m) + plane(lv - 1, z - m))
                            acc = acc + cm[m] * sm
                        v = (two * c - plane(lv - 2, z)) + plane(g.ro, z) * acc
                        if src_amps is not None and z == sz:
                            v = v.copy()
                            v[sy, sx] = v[sy, sx] + dt(src_amps[done + lv - g.nin])
                    rings[lv][z % g.W[lv]] = v
            elif K == L.OP_ENCODE:
                f, rate = o["field"], rates[o["field"]]
                planes = np.stack([plane(o["level"], z) for z in range(z0, z1)])
                stage_out[(f, o["slot"])] = enc(planes, rate) if rate else planes.copy()
            elif K in (L.OP_D2H, L.OP_STORE):
                f, rate = o["field"], rates[o["field"]]
                data = stage_out[(f, o["slot"])]
                if rate:
                    store[f][z0 // 4 * layer_words(rate): z1 // 4 * layer_words(rate)] = data
                else:
                    store[f][z0:z1] = data
        done += kr
        rnd += 1
    return store


def to_store(field, rate):
    return O.codec_encode(field, rate) if rate else field.astype(np.float32).copy()


def from_store(s, shape, rate):
    return O.codec_decode(s, shape, rate) if rate else s


@pytest.mark.parametrize("rate,k,steps,arena", [(0, 2, 9, MiB // 4), (8, 4, 11, 2 * MiB), (16, 4, 8, 2 * MiB),
                                                (5, 8, 17, 1 * MiB)])
@pytest.mark.parametrize("restart,ce", [(r, m) for r in (False, True) for m in ("copy", "hybrid", "kernel")])
def test_heat_schedule_computes_the_replay(rate, k, steps, arena, restart, ce):
    shape = (48, 12, 16)
    n = 4 if k < 8 else 2
    p = plan(shape, HEAT7, n, k, [rate], arena, block_restart=restart, **xfer(ce))
    u0 = np.random.default_rng(rate).random(shape, dtype=np.float32)
    store = [to_store(u0, rate)]
    # the initial store passes the field through the codec once
    execute(p, store, steps, None)
    got = from_store(store[0], shape, rate)
    want = O.replay_heat_f32(u0, 0.1, steps, k, rate)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("rates,k,steps", [([0, 0, 0], 3, 7), ([8, 12, 6], 3, 8), ([16, 16, 0], 1, 3), ([12, 12, 12], 4, 9)])
@pytest.mark.parametrize("restart,ce", [(r, m) for r in (False, True) for m in ("copy", "hybrid", "kernel")])
def test_wave_schedule_computes_the_replay(rates, k, steps, restart, ce):
    shape = (64, 12, 12)
    rng = np.random.default_rng(k)
    p0 = rng.standard_normal(shape).astype(np.float32)
    pm0 = rng.standard_normal(shape).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    amps = rng.standard_normal(steps).astype(np.float32)
    src = (5, 6, 20)
    p = plan(shape, WAVE25, 2, k, rates, 4 * MiB, src_cell=src, block_restart=restart, **xfer(ce))
    store = [to_store(p0, rates[0]), to_store(pm0, rates[1]), to_store(w, rates[2])]
    execute(p, store, steps, amps)
    got_p = from_store(store[0], shape, rates[0])
    got_pm = from_store(store[1], shape, rates[1])
    idx = src[0] + shape[2] * (src[1] + shape[1] * src[2])
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps, idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(got_p, wp)
    assert np.array_equal(got_pm, wpm)


@pytest.mark.parametrize("nstage", [2, 3, 5])
def test_schedule_staging_depths(nstage):
    """Copies issued 1 (two slots) or 2 ticks late stay ordered for any
    staging depth, and the schedule still computes the replay."""
    p = plan((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, nstage=nstage)
    assert p.info["nstage"] == nstage
    race_check(p, 11)
    race_check(p, 11, graph_mode=True)
    u0 = np.random.default_rng(nstage).random((48, 12, 16), dtype=np.float32)
    store = [to_store(u0, 8)]
    execute(p, store, 11, None)
    assert np.array_equal(from_store(store[0], (48, 12, 16), 8), O.replay_heat_f32(u0, 0.1, 11, 4, 8))


@pytest.mark.parametrize("rates", [[12, 12, 12], [0, 8, 8], [8, 8, 0]])
@pytest.mark.parametrize("ce", ["copy", "hybrid", "kernel"])
def test_resident_read_only_schedule(rates, ce):
    """With the read-only field resident its ring holds the whole field, no
    op of any residency moves or decodes it, the schedule has no races and
    it still computes the oracle's replay."""
    shape = (64, 12, 12)
    rng = np.random.default_rng(7)
    p0 = rng.standard_normal(shape).astype(np.float32)
    pm0 = rng.standard_normal(shape).astype(np.float32)
    w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
    steps, k = 8, 3
    amps = rng.standard_normal(steps).astype(np.float32)
    src = (5, 6, 20)
    p = plan(shape, WAVE25, 2, k, rates, 4 * MiB, src_cell=src, resident_ro=True, **xfer(ce))
    g = Geometry(p)
    assert g.W[g.ro] == shape[0]
    for kr in range(1, k + 1):
        assert all(o["field"] != 2 for o in p.schedule(kr))
    race_check(p, steps)
    race_check(p, steps, graph_mode=True)
    store = [to_store(p0, rates[0]), to_store(pm0, rates[1]), to_store(w, rates[2])]
    execute(p, store, steps, amps)
    idx = src[0] + shape[2] * (src[1] + shape[1] * src[2])
    wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps, idx), rate_p=rates[0], rate_pm=rates[1],
                                   rate_w=rates[2])
    assert np.array_equal(from_store(store[0], shape, rates[0]), wp)
    assert np.array_equal(from_store(store[1], shape, rates[1]), wpm)


def test_resident_read_only_arena_and_errors():
    """The resident field costs its nz planes of arena (the 1024^3 wave at
    12 bits still fits 8 GiB, with smaller groups); heat has no read-only
    field to keep."""
    streamed = plan((1024, 1024, 1024), WAVE25, 8, 12, [12, 12, 12], 8 << 30)
    resident = plan((1024, 1024, 1024), WAVE25, 8, 12, [12, 12, 12], 8 << 30, resident_ro=True)
    ri = resident.info
    assert ri["ring_planes"][-1] == 1024
    assert ri["arena_needed"] <= 8 << 30
    assert ri["group"] <= streamed.info["group"]
    with pytest.raises(L.OocsError):
        plan((64, 16, 16), HEAT7, 2, 2, [8], 4 * MiB, resident_ro=True)


# ---------------------------------------------------------------------------
# snake sweeps
# ---------------------------------------------------------------------------

SNAKE_CASES = [
    ((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, 11),              # fused heat, compressed, 3 residencies
    ((48, 12, 16), HEAT7, 4, 2, [0], MiB // 4, 9),               # raw, 5 residencies
    ((48, 12, 16), HEAT7, 2, 4, [5], 2 * MiB, 16),               # 2 slabs: the two blocks alternate
    ((64, 12, 12), WAVE25, 2, 3, [8, 12, 8], 4 * MiB, 8),
    ((64, 12, 12), WAVE25, 2, 3, [0, 0, 0], 4 * MiB, 7),
    ((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 8 * MiB, 14),
]


@pytest.mark.parametrize("shape,st,n,k,rates,arena,steps", SNAKE_CASES)
def test_snake_schedule_has_no_races(shape, st, n, k, rates, arena, steps):
    p = plan(shape, st, n, k, rates, arena, src_cell=(3, 3, 5) if st == WAVE25 else None, snake=True)
    race_check(p, steps)
    race_check(p, steps, graph_mode=True)


def test_full_size_snake_schedules_have_no_races():
    race_check(plan((512, 512, 512), HEAT7, 8, 4, [8], 128 * MiB, snake=True), 12)
    race_check(plan((1024, 16, 16), WAVE25, 8, 12, [8, 8, 8], 64 * MiB, snake=True, src_cell=(3, 3, 5)), 36)


@pytest.mark.parametrize("shape,st,n,k,rates,arena,steps", SNAKE_CASES)
@pytest.mark.parametrize("level_by_level", [False, True])
def test_snake_schedule_computes_the_replay(shape, st, n, k, rates, arena, steps, level_by_level):
    _snake_replay(shape, st, n, k, rates, arena, steps, level_by_level)


def _snake_replay(shape, st, n, k, rates, arena, steps, level_by_level, retain=0):
    p = plan(shape, st, n, k, rates, arena, src_cell=(3, 3, 5) if st == WAVE25 else None, snake=True,
             level_by_level=level_by_level, retain=retain)
    rng = np.random.default_rng(11)
    if st == HEAT7:
        u0 = rng.random(shape, dtype=np.float32)
        store = [to_store(u0, rates[0])]
        execute(p, store, steps, None)
        assert np.array_equal(from_store(store[0], shape, rates[0]), O.replay_heat_f32(u0, 0.1, steps, k, rates[0]))
    else:
        p0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
        pm0 = (rng.standard_normal(shape) * 0.1).astype(np.float32)
        w = (0.02 + 0.1 * rng.random(shape)).astype(np.float32)
        amps = rng.standard_normal(steps).astype(np.float32)
        store = [to_store(p0, rates[0]), to_store(pm0, rates[1]), to_store(w, rates[2])]
        execute(p, store, steps, amps)
        idx = 3 + shape[2] * (3 + shape[1] * 5)
        wp, wpm, _ = O.replay_wave_f32(p0, pm0, w, steps, k, src=(amps, idx), rate_p=rates[0], rate_pm=rates[1],
                                       rate_w=rates[2])
        assert np.array_equal(from_store(store[0], shape, rates[0]), wp)
        assert np.array_equal(from_store(store[1], shape, rates[1]), wpm)


@pytest.mark.parametrize("resident_ro,retain", [(False, 0), (True, 0), (False, 2), (True, 4), (False, 6)])
def test_snake_keeps_the_last_block_off_the_link(resident_ro, retain):
    """Residency i of R runs upward if i is even, downward if odd; the
    region it ends with (one slab, or `retain` slabs) is neither written
    back (unless i = R - 1) nor loaded by the next residency, for the
    read-write fields; every other plane crosses the link once each way per
    residency, and the read-only field is loaded whole every residency (or
    never, if resident)."""
    shape, n, k = (1024, 16, 16), 8, 12
    slab = shape[0] // n * max(retain, 1)
    p = plan(shape, WAVE25, n, k, [12, 12, 12], 64 * MiB, snake=True, resident_ro=resident_ro, retain=retain)
    assert p.info["retained_planes"] == slab
    R = 4
    for i in range(R):
        v = p.variant(i, R)
        ops = p.schedule(k, v)
        up = i % 2 == 0
        levels = [o for o in ops if o["kind"] == L.OP_LEVEL]
        first, last = levels[0]["z0"], levels[-1]["z1"]
        assert (first < last) if up else (first > last)
        for f in (0, 1, 2):
            h2d = np.zeros(shape[0], int)
            d2h = np.zeros(shape[0], int)
            for o in ops:
                if o["field"] == f and o["kind"] == L.OP_H2D:
                    h2d[o["z0"]:o["z1"]] += 1
                if o["field"] == f and o["kind"] == L.OP_D2H:
                    d2h[o["z0"]:o["z1"]] += 1
            start = slice(0, slab) if up else slice(shape[0] - slab, shape[0])
            end = slice(shape[0] - slab, shape[0]) if up else slice(0, slab)
            want_in = np.ones(shape[0], int)
            want_out = np.ones(shape[0], int)
            if f == 2:
                want_in[:] = 0 if resident_ro else 1
                want_out[:] = 0
            else:
                if i > 0:
                    want_in[start] = 0
                if i < R - 1:
                    want_out[end] = 0
            assert np.array_equal(h2d, want_in), (i, f)
            assert np.array_equal(d2h, want_out), (i, f)


# retained regions of several slabs: (case, retain, planes retained)
RETAIN_CASES = [
    (((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, 11), 2, 24),          # half the grid, fused heat
    (((48, 12, 16), HEAT7, 4, 2, [0], MiB // 4, 9), 2, 24),          # raw
    (((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, 11), 3, 36),          # the regions overlap
    (((48, 12, 16), HEAT7, 4, 4, [5], 2 * MiB, 9), 4, 48),           # the whole grid
    (((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 8 * MiB, 14), 2, 64),
    (((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 8 * MiB, 14), 3, 96),
    (((96, 12, 12), WAVE25, 6, 2, [8, 0, 8], 8 * MiB, 9), 5, 80),
    (((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 8 * MiB, 14), L.OOCS_RETAIN_MAX, 128),
    (((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 600_000, 14), L.OOCS_RETAIN_MAX, 64),
    (((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 560_000, 14), L.OOCS_RETAIN_MAX, 32),
]


@pytest.mark.parametrize("case,retain,planes", RETAIN_CASES)
def test_retained_regions_have_no_races(case, retain, planes):
    shape, st, n, k, rates, arena, steps = case
    p = plan(shape, st, n, k, rates, arena, src_cell=(3, 3, 5) if st == WAVE25 else None, snake=True, retain=retain)
    assert p.info["retained_planes"] == planes
    race_check(p, steps)
    race_check(p, steps, graph_mode=True)


@pytest.mark.parametrize("case,retain,planes", RETAIN_CASES)
def test_retained_regions_compute_the_replay(case, retain, planes):
    shape, st, n, k, rates, arena, steps = case
    _snake_replay(shape, st, n, k, rates, arena, steps, False, retain=retain)


@pytest.mark.parametrize("rule", ["zero", "swapped"])
def test_retained_addressing_mistakes_are_caught(rule, monkeypatch):
    """The race detector and the executor are not vacuous for retained
    regions: with a wrong buffer-place rule planted in their model (every op
    at base 0, or the decode and encode bases swapped), a plan whose regions
    overlap fails the race check or the replay."""
    wrong = {
        "zero": lambda self, encode, variant: 0,
        "swapped": lambda self, encode, variant: self.nz - self.X if encode == bool(variant & L.OOCS_SCHED_MIRROR) else 0,
    }[rule]
    monkeypatch.setattr(Geometry, "ret_base", wrong)
    for (shape, st, n, k, rates, arena, steps), retain in [(((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, 11), 3),
                                                            (((128, 12, 12), WAVE25, 4, 4, [12, 12, 12], 8 * MiB, 14), 3)]:
        p = plan(shape, st, n, k, rates, arena, src_cell=(3, 3, 5) if st == WAVE25 else None, snake=True,
                 retain=retain)
        with pytest.raises((AssertionError, KeyError)):
            race_check(p, steps)
            _snake_replay(shape, st, n, k, rates, arena, steps, False, retain=retain)


def test_retain_max_at_the_wave_size():
    """1024^3 wave, 8 slabs, k = 12, 8 GiB: at 12 bits per value five of
    the eight slabs of compressed p and p(n-1) fit beside the pipeline, at
    8 bits all of them (the grid then crosses the link only in a call's
    first and last residency), raw planes leave room for the one slab
    only; the group size is the one the plan takes with a single retained
    slab, and the plan one slab larger would not fit."""
    kw = dict(snake=True, ro_device_store=True)
    one = plan((1024, 1024, 1024), WAVE25, 8, 12, [12, 12, 12], 8 << 30, **kw)
    most = plan((1024, 1024, 1024), WAVE25, 8, 12, [12, 12, 12], 8 << 30, retain=L.OOCS_RETAIN_MAX, **kw)
    assert most.info["retained_planes"] == 640 and most.info["arena_needed"] <= 8 << 30
    assert most.info["group"] == one.info["group"] and most.info["nstage"] == one.info["nstage"]
    with pytest.raises(L.OocsError) as e:
        plan((1024, 1024, 1024), WAVE25, 8, 12, [12, 12, 12], 8 << 30, retain=6, group=most.info["group"],
             nstage=most.info["nstage"], **kw)
    assert e.value.code == L.OOCS_E_CAP
    assert plan((1024, 1024, 1024), WAVE25, 8, 12, [8, 8, 8], 8 << 30, retain=L.OOCS_RETAIN_MAX,
                **kw).info["retained_planes"] == 1024
    raw = plan((1024, 1024, 1024), WAVE25, 8, 12, [0, 0, 0], 8 << 30, retain=L.OOCS_RETAIN_MAX, **kw)
    assert raw.info["retained_planes"] == 128
    race_check(plan((1024, 16, 16), WAVE25, 8, 12, [8, 8, 8], 64 * MiB, snake=True, src_cell=(3, 3, 5),
                    retain=L.OOCS_RETAIN_MAX), 36)


def test_wave_planes_under_4_gib():
    """The wave tile addresses a plane with 32-bit byte offsets: a wave plan
    or an in-core wave step whose planes hold 4 GiB or more is refused
    before any device call (heat has no such limit)."""
    big = (16, 32768, 32768)  # 2^30 values per plane: 4 GiB in FP32
    for kw in ({}, {"fp64": True}):
        with pytest.raises(L.OocsError) as e:
            plan(big, WAVE25, 2, 1, [0, 0, 0], 1 << 40, **kw)
        assert e.value.code == L.OOCS_E_ARG
    with pytest.raises(L.OocsError) as e:  # FP64: 2^29 values per plane are 4 GiB already
        plan((16, 16384, 32768), WAVE25, 2, 1, [0, 0, 0], 1 << 40, fp64=True)
    assert e.value.code == L.OOCS_E_ARG
    plan((16, 16384, 32768), WAVE25, 2, 1, [0, 0, 0], 1 << 40)  # 2 GiB FP32 planes are fine
    plan(big, HEAT7, 2, 1, [0], 1 << 40)
    fake = C.c_void_p(1)  # never dereferenced: the check comes first
    for fn, esz in ((L.lib().oocs_wave25_step_k, 4), (L.lib().oocs_wave25_step_k_f64, 8)):
        ny = (1 << 32) // esz // 32768
        rc = fn(fake, fake, fake, C.c_int64(32768), C.c_int64(ny), C.c_int64(8), C.c_int64(1), None,
                C.c_int64(-1), C.c_int64(-1), C.c_int64(-1), None)
        assert rc == L.OOCS_E_ARG


def test_retain_errors():
    for kw in ({"retain": 5}, {"retain": -2}, {"snake": False, "retain": 1}):
        with pytest.raises(L.OocsError) as e:
            plan((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, **{"snake": True, **kw})
        assert e.value.code == L.OOCS_E_ARG
    assert plan((48, 12, 16), HEAT7, 3, 4, [8], 2 * MiB, snake=True, retain=L.OOCS_RETAIN_MAX).info["retained_planes"] == 48


def test_snake_needs_copy_engines_shared_levels_and_two_slabs():
    for kw in ({"kernel_transfers": True}, {"kernel_stores": True}, {"block_restart": True}):
        with pytest.raises(L.OocsError) as e:
            plan((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, snake=True, **kw)
        assert e.value.code == L.OOCS_E_ARG
    with pytest.raises(L.OocsError):
        plan((48, 12, 16), HEAT7, 1, 4, [8], 2 * MiB, snake=True)
    with pytest.raises(L.OocsError):
        plan((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB).schedule(4, L.OOCS_SCHED_MIRROR)


# ---------------------------------------------------------------------------
# FP64 plans (the paper's precision, Sec. VI): the same schedules over planes
# of doubles and the FP64 block format
# ---------------------------------------------------------------------------

def to_store64(field, rate):
    return O.codec64_encode(field, rate) if rate else field.astype(np.float64).copy()


def from_store64(s, shape, rate):
    return O.codec64_decode(s, shape, rate) if rate else s


@pytest.mark.parametrize("rates,k,steps,kw", [
    ([0, 0, 0], 3, 7, {}), ([24, 32, 24], 4, 9, {}), ([32, 0, 24], 4, 9, {"block_restart": True}),
    ([40, 40, 40], 4, 11, {"snake": True}), ([24, 24, 24], 4, 9, {"snake": True, "resident_ro": True}),
    ([68, 12, 0], 2, 5, {}), ([24, 32, 24], 4, 13, {"snake": True, "retain": 2, "ro_device_store": True}),
])
def test_fp64_wave_schedule_computes_the_fp64_replay(rates, k, steps, kw):
    shape = (64, 12, 12)
    rng = np.random.default_rng(k + len(kw))
    p0 = rng.standard_normal(shape)
    pm0 = rng.standard_normal(shape)
    w = 0.02 + 0.1 * rng.random(shape)
    amps = rng.standard_normal(steps).astype(np.float32)  # float amplitudes, exact in double
    src = (5, 6, 20)
    p = plan(shape, WAVE25, 2, k, rates, 8 * MiB, src_cell=src, fp64=True, **kw)
    store = [to_store64(p0, rates[0]), to_store64(pm0, rates[1]), to_store64(w, rates[2])]
    execute(p, store, steps, amps)
    idx = src[0] + shape[2] * (src[1] + shape[1] * src[2])
    wp, wpm, _ = O.replay_wave64(p0, pm0, w, steps, k, src=(amps.astype(np.float64), idx), rate_p=rates[0],
                                 rate_pm=rates[1], rate_w=rates[2])
    assert np.array_equal(from_store64(store[0], shape, rates[0]), wp)
    assert np.array_equal(from_store64(store[1], shape, rates[1]), wpm)


def test_fp64_plan_sizes():
    """Planes and raw stores hold 8-byte values; a compressed store holds
    rate bits per value whatever the precision; the device rings double."""
    shape = (64, 16, 16)
    p32 = plan(shape, WAVE25, 2, 4, [0, 0, 0], 64 * MiB)
    p64 = plan(shape, WAVE25, 2, 4, [0, 0, 0], 64 * MiB, fp64=True)
    assert p64.info["plane_bytes"] == 8 * 16 * 16 == 2 * p32.info["plane_bytes"]
    assert p64.store_bytes(0) == 8 * 64 * 16 * 16
    assert p64.info["ring_planes"] == p32.info["ring_planes"]
    assert p64.info["arena_needed"] > p32.info["arena_needed"]
    c64 = plan(shape, WAVE25, 2, 4, [24, 68, 32], 64 * MiB, fp64=True)
    assert [c64.store_bytes(f) for f in range(3)] == [64 * 16 * 16 * r // 8 for r in (24, 68, 32)]
    race_check(c64, 9)
    race_check(plan(shape, WAVE25, 2, 4, [24, 24, 24], 64 * MiB, fp64=True, snake=True), 13)
    race_check(plan(shape, WAVE25, 2, 4, [24, 24, 24], 64 * MiB, fp64=True, snake=True, retain=2), 13)


def test_fp64_plan_errors():
    shape = (64, 16, 16)
    for rates in ([69, 0, 0], [-1, 0, 0]):
        with pytest.raises(L.OocsError) as e:
            plan(shape, WAVE25, 2, 4, rates, 64 * MiB, fp64=True)
        assert e.value.code == L.OOCS_E_RATE
    with pytest.raises(L.OocsError) as e:  # FP32 stays capped at 34
        plan(shape, WAVE25, 2, 4, [35, 0, 0], 64 * MiB)
    assert e.value.code == L.OOCS_E_RATE
    for kw in ({"midpoint": True}, {"kernel_transfers": True}, {"kernel_stores": True}):
        with pytest.raises(L.OocsError) as e:
            plan(shape, WAVE25, 2, 4, [24, 24, 24], 64 * MiB, fp64=True, **kw)
        assert e.value.code == L.OOCS_E_ARG
    with pytest.raises(L.OocsError) as e:
        plan((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, fp64=True)
    assert e.value.code == L.OOCS_E_ARG


# ---------------------------------------------------------------------------
# the read-only store held on the device
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rates,k,steps,kw", [
    ([8, 12, 8], 4, 9, {}), ([0, 0, 0], 3, 7, {}), ([12, 12, 12], 4, 13, {"snake": True}),
    ([0, 12, 12], 4, 9, {"block_restart": True}), ([12, 0, 8], 4, 9, {"kernel_stores": True}),
    ([24, 24, 24], 4, 9, {"fp64": True}),
])
def test_device_store_schedule_computes_the_replay(rates, k, steps, kw):
    """Decoding the read-only chunks from the device copy of the store gives
    the replay bit for bit; no host-to-device copy of that field remains;
    the schedule has no races."""
    shape = (64, 12, 12)
    rng = np.random.default_rng(steps)
    f64 = kw.get("fp64", False)
    dt = np.float64 if f64 else np.float32
    p0 = rng.standard_normal(shape).astype(dt)
    pm0 = rng.standard_normal(shape).astype(dt)
    w = (0.02 + 0.1 * rng.random(shape)).astype(dt)
    amps = rng.standard_normal(steps).astype(np.float32)
    src = (5, 6, 20)
    p = plan(shape, WAVE25, 2, k, rates, 8 * MiB, src_cell=src, ro_device_store=True, **kw)
    for kr in range(1, k + 1):
        ops = p.schedule(kr)
        assert not any(o["field"] == 2 and o["kind"] in (L.OP_H2D, L.OP_FETCH) for o in ops)
        assert any(o["kind"] == L.OP_DECODE and o["slot"] == L.OOCS_SLOT_DEVICE_STORE for o in ops)
    race_check(p, steps)
    race_check(p, steps, graph_mode=True)
    ts, fs = (to_store64, from_store64) if f64 else (to_store, from_store)
    store = [ts(p0, rates[0]), ts(pm0, rates[1]), ts(w, rates[2])]
    execute(p, store, steps, amps)
    idx = src[0] + shape[2] * (src[1] + shape[1] * src[2])
    replay = O.replay_wave64 if f64 else O.replay_wave_f32
    a = amps.astype(np.float64) if f64 else amps
    wp, wpm, _ = replay(p0, pm0, w, steps, k, src=(a, idx), rate_p=rates[0], rate_pm=rates[1], rate_w=rates[2])
    assert np.array_equal(fs(store[0], shape, rates[0]), wp)
    assert np.array_equal(fs(store[1], shape, rates[1]), wpm)


def test_device_store_arena_and_errors():
    shape = (64, 16, 16)
    a = plan(shape, WAVE25, 2, 4, [12, 12, 12], 64 * MiB)
    b = plan(shape, WAVE25, 2, 4, [12, 12, 12], 64 * MiB, ro_device_store=True)
    # the streamed slots of the read-only field go, its whole store comes in
    assert b.info["arena_needed"] > a.info["arena_needed"] - a.info["nstage"] * a.info["group"] * 16 * 16 * 12 // 8
    assert b.info["arena_needed"] >= b.store_bytes(2)
    for kw in ({"resident_ro": True}, {"kernel_transfers": True}):
        with pytest.raises(L.OocsError) as e:
            plan(shape, WAVE25, 2, 4, [12, 12, 12], 64 * MiB, ro_device_store=True, **kw)
        assert e.value.code == L.OOCS_E_ARG
    with pytest.raises(L.OocsError) as e:
        plan((48, 12, 16), HEAT7, 4, 4, [8], 2 * MiB, ro_device_store=True)
    assert e.value.code == L.OOCS_E_ARG
