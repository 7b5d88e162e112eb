#!/usr/bin/env python3
"""Benchmark of the out-of-core compressed stencil pipeline on one MI355X.

Headline workload: the 25-point 8th-order acoustic wave (two read-write
fields p(n), p(n-1) and the read-only w = (v dt/dx)^2) on a 1024^3 FP32 grid
(4 GiB per field), layered velocity model 1500..4500 m/s, 15 Hz Ricker point
source, dt at CFL 0.4; split into 8 z-slabs of 128 planes, k = 12 steps per
residency (halo 48 planes), device memory capped at an 8 GiB arena; all three
fields in pinned host stores, compressed at 12 bits per value (37.5 % of the
bits, the paper's 24/64 ratio for doubles), against the same pipeline
uncompressed and at 8 and 16 bits per value.

Schedule: shared time levels between neighbouring blocks and snake sweeps
(residencies alternate direction; the blocks a residency ends with stay on
the device, compressed, for the next one: as many slabs as the arena holds),
the orchestration the paper leaves to future work
(Sec. VII); one retained slab, one-way sweeps and the paper's per-block
schedule of Fig. 2 are reported beside it. The read-only field's host store
is copied into the arena once (1.5 GiB at 12 bits, inside the 8 GiB cap) and
decoded from there every residency; the planes of p and p(n-1) outside the
retained region cross the host link both ways every round. The paper's flow, which streams every field's chunks (the
read-only ones included) over the link every residency, with one retained
slab, is reported beside it, and the paper's codes 2-4 use it.

One bench step = one round of the method: every block of the grid advanced
k = 12 steps (12 * 1024^3 cell updates), all transfers included. The timed
rounds start from the developed wavefield of the middle of the 4,320-step
run (step 2,160, made by an in-core GPU run of the same propagator): the
codec's cost depends on the data, and the middle of the run is its average.

Reported besides: the other rates, the paper's codes 2-4 (which fields are
compressed), one-way sweeps, the per-block schedule of Fig. 2 (halo recompute), the
per-stage breakdown (Sec. VI-B), the whole 4,320-step run per rate with the
Sec. VI-C errors against the uncompressed run every 480 steps, the fused
pipeline kernel against the HBM and VALU rooflines, the host link, the
512^3 heat workload and the other rows' workloads, and the CPU oracle on a
bounded sample of the headline workload.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_START = time.perf_counter()

# ---- headline: 1024^3 wave ------------------------------------------------------
WAVE_SHAPE = (1024, 1024, 1024)
WAVE_SLABS = 8
WAVE_K = 12
WAVE_CAP = 8 << 30
WAVE_STEPS = 4320
WAVE_START = 2160           # the timed rounds start here (middle of the run)
WAVE_SEGMENT = 480          # error snapshots of the whole run every 480 steps
HEADLINE_RATE = 12
WAVE_RATES = (0, 16, 12, 8)
FULL_RUN_RATES = (8, 12, 16)

# ---- 512^3 heat (the other out-of-core workload) ----------------------------------
HEAT_SHAPE = (512, 512, 512)
HEAT_SLABS = 8
HEAT_K = 4
HEAT_TIME_STEPS = 100
HEAT_CAP = 128 << 20
ALPHA = 0.1
HEAT_RATES = (0, 16, 8)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 64 lanes x 2.4 GHz (one wave64 VALU instruction
# per CU per clock, packed FP32 not used)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
METRIC = "end-to-end GCell-updates/s, compressed vs uncompressed out-of-core; HBM GB/s %"
COUNTERS = os.path.join(ROOT, "profiles", "wave1024_rate12_counters.json")
KERNEL_SOURCES = ("paper_2109_05410_amd/csrc/kernels.hip", "paper_2109_05410_amd/csrc/codec_dev.hpp",
                  "paper_2109_05410_amd/csrc/stencil_dev.hpp", "paper_2109_05410_amd/csrc/internal.hpp")
PROFILE_EVERY = 3


def log(msg):
    print(f"# [{time.perf_counter() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_counters(key):
    """Per-launch figures of each kernel ({kernel name: value}) from committed
    rocprofv3 counter runs of the headline workload, if they were taken on the
    current kernel source; else None. key: "hbm_bytes_per_launch"
    (FETCH_SIZE + WRITE_SIZE, calibrated) or "alu_ops_per_launch"
    (SQ_INSTS_VALU x 64 lanes)."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_hash") != kernel_source_hash():
        return None
    return c.get(key)


def _rounded(x):
    """Floats to 5 significant digits (small error figures keep their value)."""
    if isinstance(x, dict):
        return {k: _rounded(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_rounded(v) for v in x]
    return float(f"{x:.5g}") if isinstance(x, float) else x


def _timed(torch, fn, reps=1):
    """Wall time of fn() between device synchronizations (seconds per call)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def kernel_summary(stats, steps, profile):
    """Launch statistics of a list of RunStats (per bench step)."""
    nl = sum(s.launches for s in stats)
    kms = sum(s.kernel_ms for s in stats)
    tl = sum(s.timed_launches for s in stats)
    tb = sum(s.timed_bytes for s in stats)
    return {
        "launches_per_step": nl // steps,
        "codec_bytes_per_launch": sum(s.codec_bytes for s in stats) / max(nl, 1),
        "stencil_bytes_per_launch": sum(s.stencil_bytes for s in stats) / max(nl, 1),
        "bytes_per_launch": tb / max(tl, 1),
        "timed_launches_per_step": tl // steps,
        "avg_launch_us": kms * 1e3 / max(tl, 1) if profile and tl else None,
        "achieved_GBps": tb / (kms * 1e-3) / 1e9 if kms > 0 else None,
        "gpu_busy_frac": None,
    }


# ---------------------------------------------------------------------------
# 1024^3 wave
# ---------------------------------------------------------------------------

class WaveInputs:
    def __init__(self, inputs):
        import numpy as np

        self.dt = inputs.wave_dt()
        self.w = inputs.wave_coefficient(inputs.layered_velocity(WAVE_SHAPE, seed=1), self.dt)
        self.cell = inputs.source_cell(WAVE_SHAPE)
        self.amps = inputs.ricker(WAVE_STEPS + 4096, self.dt)
        self.zero = np.zeros(WAVE_SHAPE, np.float32)


def wave_state(api, torch, wi, steps):
    """(p(steps), p(steps - 1)) of the run from rest, by the in-core GPU
    propagator (the uncompressed out-of-core pipeline gives the same bits)."""
    p = torch.zeros(WAVE_SHAPE, dtype=torch.float32, device="cuda")
    pm = torch.zeros_like(p)
    wd = torch.from_numpy(wi.w).cuda()
    for t0 in range(0, steps, WAVE_SEGMENT):
        n = min(WAVE_SEGMENT, steps - t0)
        api.wave25_step_k(p, pm, wd, n, src=(wi.amps[t0:t0 + n], wi.cell))
        torch.cuda.synchronize()
    out = (p.cpu().numpy(), pm.cpu().numpy())
    del p, pm, wd
    torch.cuda.empty_cache()
    return out


def wave_plan(api, wi, rates, **flags):
    """The 1024^3 wave plan; snake sweeps unless flags say otherwise (the
    per-block schedule excludes them), retaining as many slabs as the arena
    holds, the read-only store held on the device unless flags say otherwise
    (a decoded resident field excludes it)."""
    flags.setdefault("snake", not flags.get("block_restart", False))
    flags.setdefault("retain", api.RETAIN_MAX if flags["snake"] else 0)
    flags.setdefault("ro_device_store", not flags.get("resident_ro", False))
    return api.OutOfCorePlan(WAVE_SHAPE, api.WAVE25, WAVE_SLABS, WAVE_K, list(rates), WAVE_CAP, src_cell=wi.cell,
                             **flags)


def wave_window(api, torch, wi, state, rates, rounds, warmup, profile=False, breakdown_rounds=0, **flags):
    """`warmup` untimed rounds from the state at WAVE_START, then `rounds`
    timed rounds (one oocs_run call); optionally `breakdown_rounds` more with
    the per-stage breakdown on."""
    p, pm = state
    plan = wave_plan(api, wi, rates, **flags)
    st = [plan.new_store(f) for f in range(3)]
    plan.put(0, p, st[0])
    plan.put(1, pm, st[1])
    plan.put(2, wi.w, st[2])
    t = WAVE_START
    for _ in range(warmup):
        plan.run(st, WAVE_K, src_amps=wi.amps[t:t + WAVE_K])
        t += WAVE_K
    plan.set_profiling(profile, every=PROFILE_EVERY)
    n = WAVE_K * rounds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = plan.run(st, n, src_amps=wi.amps[t:t + n])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t += n
    plan.set_profiling(False)
    info = plan.info
    cells = float(WAVE_SHAPE[0] * WAVE_SHAPE[1] * WAVE_SHAPE[2]) * n
    out = {
        "rates": list(rates),
        "rounds_timed": rounds,
        "steps_timed": n,
        "window": f"steps {t - n}..{t} of the {WAVE_STEPS}-step run",
        "gcells_per_s": cells / dt / 1e9,
        "ms_per_round": dt / rounds * 1e3,
        "group_planes": info["group"],
        "retained_planes": info["retained_planes"],
        "arena_used_bytes": s.arena_bytes,
        "h2d_GBps": s.h2d_bytes / dt / 1e9,
        "d2h_GBps": s.d2h_bytes / dt / 1e9,
        "h2d_bytes_per_round": s.h2d_bytes // rounds,
        "d2h_bytes_per_round": s.d2h_bytes // rounds,
        "d2h_engine": "sdma" if s.sdma_copies else "hipMemcpyAsync",
        "host_enqueue_frac": s.enqueue_ms * 1e-3 / dt,
        "kernel": kernel_summary([s], rounds, profile),
    }
    if profile and s.timed_launches:
        out["kernel"]["gpu_busy_frac"] = s.kernel_ms * 1e-3 * (s.launches / s.timed_launches) / dt
    if breakdown_rounds:
        plan.set_breakdown(True)
        nb = WAVE_K * breakdown_rounds
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = plan.run(st, nb, src_amps=wi.amps[t:t + nb])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / breakdown_rounds
        plan.set_breakdown(False)
        out["breakdown_ms_per_round"] = {k: v / breakdown_rounds for k, v in b.breakdown_ms.items()}
        out["breakdown_wall_ms_per_round"] = wall
    plan.close()
    del st
    return out


def field_errors(torch, a, ref, idx):
    """Sec. VI-C errors of device field a against device field ref: mean
    point-wise relative error over the sampled cells idx (cells whose
    reference magnitude is at most 1e-30 of the largest are left out), the
    same mean over the sampled cells whose reference magnitude exceeds 1e-3
    of the largest (where the wave has arrived: ahead of the front the
    values are tiny and a block-floating-point codec's error relative to
    them is large), and the normwise max and L2 relative errors."""
    d = a - ref
    rmax = float(ref.abs().max())
    num = float(torch.linalg.vector_norm(d, dtype=torch.float64))
    den = float(torch.linalg.vector_norm(ref, dtype=torch.float64))
    av = a.view(-1)[idx].double()
    rv = ref.view(-1)[idx].double()
    rel = (av - rv).abs() / rv.abs()
    keep = rv.abs() > 1e-30 * rmax
    big = rv.abs() > 1e-3 * rmax
    return {
        "pointwise_mean_rel": float(rel[keep].mean()) if int(keep.sum()) else 0.0,
        "sampled_used": int(keep.sum()),
        "pointwise_mean_rel_above_1e-3_max": float(rel[big].mean()) if int(big.sum()) else 0.0,
        "sampled_above_1e-3_max": int(big.sum()),
        "max_rel": float(d.abs().max()) / rmax if rmax > 0 else float(d.abs().max()),
        "l2_rel": num / den if den > 0 else num,
    }


def wave_full_run(api, torch, inputs, wi, rates, deadline_s):
    """The whole 4,320-step run at each rate from rest, in segments of 480
    steps; after each segment the compressed state p(n) decoded from its host
    store is compared with the uncompressed run (the in-core GPU propagator,
    bit-identical to the uncompressed pipeline) at the same step. The time of
    each rate's runs alone gives its whole-run rate. Stops at the deadline
    (seconds since the bench started) and says so."""
    import numpy as np

    idx = torch.from_numpy(inputs.sample_points(WAVE_SHAPE, 100, seed=0)).cuda()
    p = torch.zeros(WAVE_SHAPE, dtype=torch.float32, device="cuda")
    pm = torch.zeros_like(p)
    wd = torch.from_numpy(wi.w).cuda()
    dec = torch.empty_like(p)
    plans, stores, secs = {}, {}, {}
    for r in rates:
        plans[r] = wave_plan(api, wi, [r] * 3)
        stores[r] = [plans[r].new_store(f) for f in range(3)]
        plans[r].put(0, wi.zero, stores[r][0])
        plans[r].put(1, wi.zero, stores[r][1])
        plans[r].put(2, wi.w, stores[r][2])
        secs[r] = 0.0
    curve = []
    done = 0
    truncated = False
    while done < WAVE_STEPS:
        if time.perf_counter() - T_START > deadline_s:
            truncated = True
            break
        n = min(WAVE_SEGMENT, WAVE_STEPS - done)
        amps = wi.amps[done:done + n]
        api.wave25_step_k(p, pm, wd, n, src=(amps, wi.cell))
        torch.cuda.synchronize()
        row = {"step": done + n}
        for r in rates:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plans[r].run(stores[r], n, src_amps=amps)
            secs[r] += time.perf_counter() - t0
            words = stores[r][0].cuda().view(torch.int64)
            api.codec_decode(words, WAVE_SHAPE, r, out=dec)
            row[f"rate{r}"] = field_errors(torch, dec, p, idx)
            del words
        done += n
        curve.append(row)
        log(f"wave full run: step {done}: " +
            ", ".join(f"rate {r} pw {row[f'rate{r}']['pointwise_mean_rel']:.2e} l2 {row[f'rate{r}']['l2_rel']:.2e}"
                      for r in rates))
    cells = float(np.prod(WAVE_SHAPE)) * done
    out = {
        "steps_run": done,
        "truncated_at_deadline": truncated,
        "rates": {f"rate{r}": {"s": secs[r], "gcells_per_s": cells / secs[r] / 1e9 if secs[r] else None}
                  for r in rates},
        "errors_vs_uncompressed": curve,
        "reference": "in-core FP32 GPU run (bit-identical to the uncompressed pipeline); errors of p(n) decoded "
                     "from each compressed host store",
    }
    for r in rates:
        plans[r].close()
    del plans, stores, p, pm, wd, dec
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# FP64 replica of the paper's experiment (Sec. VI-A): FP64 fields, the FP64
# format at 24 and 32 bits per value, the paper's decomposition (8 blocks of
# 144 planes, k = 12)
# ---------------------------------------------------------------------------

FP64_SHAPE = (1152, 1152, 1152)  # the interior of the paper's (1152 + 2*4)^3 grid; outside cells are zero
FP64_SLABS = 8
FP64_K = 12
FP64_CAP = 32 << 30              # device arena: the 32 GB of the paper's GPU
# (name, bits per double of p, p(n-1), w; read-only store in the arena; retained slabs, 0 = one)
FP64_CODES = (("code1", [0, 0, 0], False, 0), ("code2", [0, 32, 0], False, 0), ("code3", [0, 0, 32], False, 0),
              ("code4", [0, 24, 24], False, 0), ("all24", [24, 24, 24], False, 0),
              ("code4_ro_device_store", [0, 24, 24], True, 0), ("all24_ro_device_store", [24, 24, 24], True, 0),
              ("all24_ro_device_store_retain_max", [24, 24, 24], True, -1))


def fp64_replica(api, torch, inputs, wi, state, rounds=2):
    """The paper's four codes in FP64 (1 = no compression, 2 = p(n-1) at 32
    bits/value, 3 = the read-only field at 32, 4 = both at 24; and every
    field at 24) on the 1152^3 grid, in the paper's flow (the read-only
    chunks streamed every residency), codes 4 and all-24 with the read-only
    store held in the arena, and all-24 with as many slabs retained as fit
    (six timed rounds, so that the call's first and last residencies, which
    move every plane, weigh less). Synthetic data: the 1024^3 FP32 state
    at step WAVE_START placed in the grid's low corner, cast to double, and
    the layered model on the whole grid in double. One untimed round, then
    `rounds` timed rounds per code; snake sweeps."""
    import numpy as np

    nz, ny, nx = FP64_SHAPE
    n0 = WAVE_SHAPE[0]
    p = np.zeros(FP64_SHAPE)
    p[:n0, :n0, :n0] = state[0]
    pm = np.zeros(FP64_SHAPE)
    pm[:n0, :n0, :n0] = state[1]
    v = inputs.layered_velocity((nz, 4, 4), seed=1)[:, 0, 0].astype(np.float64)
    w = np.empty(FP64_SHAPE)
    w[...] = ((v * wi.dt / 10.0) ** 2)[:, None, None]
    cell = inputs.source_cell(FP64_SHAPE)
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()  # pinned blocks cached by earlier sections
    raw = nx * ny * nz * 8
    bufs = [torch.empty(raw, dtype=torch.uint8, pin_memory=True) for _ in range(3)]
    out = {"grid": list(FP64_SHAPE), "nslabs": FP64_SLABS, "k": FP64_K, "device_cap_bytes": FP64_CAP,
           "data": f"1024^3 FP32 wavefield of step {WAVE_START} in the low corner, cast to double; layered model "
                   "in double", "codes": {}}
    for name, rates, ro_dev, retain in FP64_CODES:
        rr = rounds if retain == 0 else 3 * rounds
        cells = float(nx * ny * nz) * FP64_K * rr
        plan = api.OutOfCorePlan(FP64_SHAPE, api.WAVE25, FP64_SLABS, FP64_K, rates, FP64_CAP, src_cell=cell,
                                 fp64=True, snake=True, ro_device_store=ro_dev,
                                 retain=api.RETAIN_MAX if retain < 0 else retain)
        st = [bufs[f][:plan.store_bytes(f)] for f in range(3)]
        for f, a in enumerate((p, pm, w)):
            plan.put(f, a, st[f])
        t = WAVE_START
        plan.run(st, FP64_K, src_amps=wi.amps[t:t + FP64_K])
        t += FP64_K
        n = FP64_K * rr
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = plan.run(st, n, src_amps=wi.amps[t:t + n])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["codes"][name] = {
            "rates_bits_per_double": rates,
            "read_only_store_on_device": ro_dev,
            "rounds_timed": rr,
            "gcells_per_s": cells / dt / 1e9,
            "ms_per_round": dt / rr * 1e3,
            "h2d_GBps": s.h2d_bytes / dt / 1e9,
            "d2h_GBps": s.d2h_bytes / dt / 1e9,
            "h2d_bytes_per_round": s.h2d_bytes // rr,
            "d2h_bytes_per_round": s.d2h_bytes // rr,
            "group_planes": plan.info["group"],
            "retained_planes": plan.info["retained_planes"],
            "arena_used_bytes": s.arena_bytes,
        }
        log(f"FP64 {name}: {out['codes'][name]['gcells_per_s']:.1f} GCell-updates/s, "
            f"{out['codes'][name]['ms_per_round']:.0f} ms/round")
        plan.close()
        del plan, st  # the views keep the pinned buffers alive
    out["codec64_512"] = codec64_rates(api, torch, state)
    log(f"FP64 codec: {out['codec64_512']}")
    base = out["codes"]["code1"]["gcells_per_s"]
    out["speedup_vs_code1"] = {k: v["gcells_per_s"] / base for k, v in out["codes"].items() if k != "code1"}
    out["paper_context"] = "V100-PCIe 32 GB, 4 x 1160^3 doubles: code 2 1.16x, code 3 1.18x, code 4 1.20x (Sec. VI-A)"
    del bufs, p, pm, w
    torch.cuda.synchronize()
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()  # give the 37 GB of pinned stores back before the next sections pin theirs
    torch.cuda.empty_cache()
    return out


FP64_ERR_SHAPE = (512, 512, 512)


def fp64_error_curve(api, torch, inputs, wi, deadline_s):
    """Sec. VI-C in the paper's precision: the whole 4,320-step run in FP64
    from rest on a 512^3 grid (layered model in double, the Ricker source),
    under the compressed schedule (every k = 12 steps the compressed fields
    pass through decode(encode()) with the FP64 format; the out-of-core
    decomposition is exact, so this is the state the FP64 pipeline reaches)
    for the paper's codes 2, 3 and 4, against the uncompressed FP64 run;
    errors of p(n) every 480 steps. Also the in-core FP64 step rate."""
    import numpy as np

    nz, ny, nx = FP64_ERR_SHAPE
    v = inputs.layered_velocity((nz, 4, 4), seed=1)[:, 0, 0].astype(np.float64)
    w0 = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(((v * wi.dt / 10.0) ** 2)[:, None, None],
                                                               FP64_ERR_SHAPE))).cuda()
    cell = inputs.source_cell(FP64_ERR_SHAPE)
    amps = wi.amps.astype(np.float64)
    idx = torch.from_numpy(inputs.sample_points(FP64_ERR_SHAPE, 100, seed=0)).cuda()
    codes = {"code2": (0, 32, 0), "code3": (0, 0, 32), "code4": (0, 24, 24)}
    ref = [torch.zeros(FP64_ERR_SHAPE, dtype=torch.float64, device="cuda") for _ in range(2)]
    runs = {}
    for name, (rp, rpm, rw) in codes.items():
        w = w0.clone()
        if rw:
            api.codec64_roundtrip_(w, rw)  # the read-only store, compressed once
        runs[name] = [torch.zeros_like(ref[0]), torch.zeros_like(ref[0]), w]
    curve = []
    done = 0
    t_ref = 0.0
    while done < WAVE_STEPS and time.perf_counter() - T_START <= deadline_s:
        n = min(WAVE_SEGMENT, WAVE_STEPS - done)
        src = (amps[done:done + n], cell)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.wave25_step_k_f64(ref[0], ref[1], w0, n, src=src)
        torch.cuda.synchronize()
        t_ref += time.perf_counter() - t0
        row = {"step": done + n}
        for name, (rp, rpm, rw) in codes.items():
            p, pm, w = runs[name]
            api.wave64_compressed_run(p, pm, w, n, WAVE_K, src=src, rate_p=rp, rate_pm=rpm, rate_w=rw, initial=False)
            row[name] = field_errors(torch, p, ref[0], idx)
        done += n
        curve.append(row)
        log(f"FP64 error curve: step {done}: " +
            ", ".join(f"{c} pw {row[c]['pointwise_mean_rel']:.2e} l2 {row[c]['l2_rel']:.2e}" for c in codes))
    out = {
        "grid": list(FP64_ERR_SHAPE), "k": WAVE_K, "steps_run": done, "truncated_at_deadline": done < WAVE_STEPS,
        "codes": {c: list(r) for c, r in codes.items()},
        "in_core_fp64_gcells_per_s": float(nx * ny * nz) * done / t_ref / 1e9 if t_ref else None,
        "errors_vs_uncompressed_fp64": curve,
        "paper_context": "mean point-wise relative error ~1e-6 to 1e-7 at 24-32 bits per double (Sec. VI-C)",
    }
    del runs, ref, w0
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# 512^3 heat
# ---------------------------------------------------------------------------

def heat_variant(api, torch, u0, rate, steps, warmup, breakdown=False, **flags):
    """One rate of the 512^3 heat pipeline: `warmup` untimed bench steps of
    100 time steps, then `steps` timed ones (wall clock)."""
    plan = api.OutOfCorePlan(HEAT_SHAPE, api.HEAT7, HEAT_SLABS, HEAT_K, [rate], HEAT_CAP, alpha=ALPHA, **flags)
    store = plan.new_store(0)
    plan.put(0, u0, store)
    for _ in range(warmup):
        plan.run([store], HEAT_TIME_STEPS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [plan.run([store], HEAT_TIME_STEPS) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = float(HEAT_SHAPE[0] * HEAT_SHAPE[1] * HEAT_SHAPE[2]) * HEAT_TIME_STEPS * steps
    out = {
        "rate": rate,
        "gcells_per_s": cells / dt / 1e9,
        "ms_per_100_steps": dt / steps * 1e3,
        "group_planes": plan.info["group"],
        "arena_used_bytes": stats[0].arena_bytes,
        "h2d_GBps": sum(s.h2d_bytes for s in stats) / dt / 1e9,
        "d2h_GBps": sum(s.d2h_bytes for s in stats) / dt / 1e9,
        "launches_per_100_steps": stats[0].launches,
    }
    if breakdown:
        plan.set_breakdown(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = plan.run([store], HEAT_TIME_STEPS)
        torch.cuda.synchronize()
        out["breakdown_ms_per_100_steps"] = b.breakdown_ms
        out["breakdown_wall_ms"] = (time.perf_counter() - t0) * 1e3
        plan.set_breakdown(False)
    plan.close()
    del store
    return out


def heat_in_core_rate(api, torch, u0):
    """The in-core heat step on the whole 512^3 field resident in HBM (no cap)."""
    u = torch.from_numpy(u0).cuda()
    tmp = torch.empty_like(u)
    api.heat7_step_k(u, ALPHA, 4, tmp=tmp)
    t = _timed(torch, lambda: api.heat7_step_k(u, ALPHA, HEAT_TIME_STEPS, tmp=tmp))
    return HEAT_SHAPE[0] * HEAT_SHAPE[1] * HEAT_SHAPE[2] * HEAT_TIME_STEPS / t / 1e9


def small_in_core(api, torch, inputs, reps=200):
    """The in-core step at its own small size: 10 heat steps of a 64^3
    field (1 MiB), one call per 10 steps, averaged over reps calls."""
    u = torch.from_numpy(inputs.heat_uniform((64, 64, 64), seed=5)).cuda()
    tmp = torch.empty_like(u)
    api.heat7_step_k(u, ALPHA, 10, tmp=tmp)
    t = _timed(torch, lambda: api.heat7_step_k(u, ALPHA, 10, tmp=tmp), reps=reps)
    return {"grid": [64, 64, 64], "steps": 10, "us_per_call": round(t * 1e6, 1),
            "gcells_per_s": round(64 ** 3 * 10 / t / 1e9, 2), "calls": reps}


def codec_rates(api, torch, u0, rate=8):
    """Field encode and decode of the 512^3 heat field: values per second and
    algorithmic bytes (4 + rate/8 per value) per second."""
    u = torch.from_numpy(u0).cuda()
    w = api.codec_encode(u, rate)
    out = torch.empty_like(u)
    api.codec_decode(w, HEAT_SHAPE, rate, out=out)
    n = u.numel()
    te = _timed(torch, lambda: api.codec_encode(u, rate, out=w), reps=5)
    td = _timed(torch, lambda: api.codec_decode(w, HEAT_SHAPE, rate, out=out), reps=5)
    b = n * (4 + rate / 8)
    return {
        "rate": rate,
        "encode_Gvalues_per_s": round(n / te / 1e9, 1), "encode_GBps": round(b / te / 1e9, 1),
        "encode_hbm_frac": round(b / te / 1e9 / HBM_PEAK_GBS, 4),
        "decode_Gvalues_per_s": round(n / td / 1e9, 1), "decode_GBps": round(b / td / 1e9, 1),
        "decode_hbm_frac": round(b / td / 1e9 / HBM_PEAK_GBS, 4),
    }


def codec64_rates(api, torch, state, rate=24):
    """FP64-format encode and decode of a 512^3 double field (the centre of
    the 1024^3 FP32 wavefield cast to double): values per second and
    algorithmic bytes (8 + rate/8 per value) per second."""
    import numpy as np

    c = WAVE_SHAPE[0] // 2
    u = torch.from_numpy(np.ascontiguousarray(state[0][c - 256:c + 256, c - 256:c + 256, c - 256:c + 256],
                                              dtype=np.float64)).cuda()
    shape = tuple(u.shape)
    w = api.codec64_encode(u, rate)
    out = torch.empty_like(u)
    api.codec64_decode(w, shape, rate, out=out)
    n = u.numel()
    te = _timed(torch, lambda: api.codec64_encode(u, rate, out=w), reps=3)
    td = _timed(torch, lambda: api.codec64_decode(w, shape, rate, out=out), reps=3)
    b = n * (8 + rate / 8)
    del u, w, out
    return {
        "rate": rate, "grid": list(shape),
        "encode_Gvalues_per_s": round(n / te / 1e9, 2), "encode_GBps": round(b / te / 1e9, 1),
        "encode_hbm_frac": round(b / te / 1e9 / HBM_PEAK_GBS, 4),
        "decode_Gvalues_per_s": round(n / td / 1e9, 2), "decode_GBps": round(b / td / 1e9, 1),
        "decode_hbm_frac": round(b / td / 1e9 / HBM_PEAK_GBS, 4),
    }


BATCH_STEPS = 200


def batched_rate(api, torch, inputs):
    """64 heat cubes with sides uniform in [64, 384], 200 steps: a graph of
    one launch per group (autotuned tiles and temporal-blocking depth, the
    default) against one persistent launch and against separate per-domain
    launches."""
    import tempfile

    sides = inputs.batch_sides()
    fields = [torch.from_numpy(inputs.heat_uniform((int(s),) * 3, seed=3 + j)).cuda() for j, s in enumerate(sides)]
    cells = float(sum(int(s) ** 3 for s in sides)) * BATCH_STEPS
    with tempfile.TemporaryDirectory() as td:
        t0 = time.perf_counter()
        b = api.HeatBatch(fields, tune=True, tune_cache=os.path.join(td, "tune.json"))
        tune_s = time.perf_counter() - t0
    b.run(BATCH_STEPS)  # builds the graph
    tl = _timed(torch, lambda: b.run(BATCH_STEPS))
    b.set_persistent(True)
    b.run(BATCH_STEPS, check=True)
    tb = _timed(torch, lambda: b.run(BATCH_STEPS))
    b.check()
    b.set_persistent(False)
    b.run_per_domain(1)
    tp = _timed(torch, lambda: b.run_per_domain(BATCH_STEPS))
    tiles = {}
    for i in range(len(sides)):
        tiles[str(b.tile(i))] = tiles.get(str(b.tile(i)), 0) + 1
    out = {
        "domains": len(sides), "steps": BATCH_STEPS, "cells": int(cells / BATCH_STEPS),
        "depth": b.depth, "tiles": tiles, "tune_s": round(tune_s, 2),
        "graph_of_launches_gcells_per_s": round(cells / tl / 1e9, 1),
        "persistent_gcells_per_s": round(cells / tb / 1e9, 1),
        "per_domain_gcells_per_s": round(cells / tp / 1e9, 1),
        "speedup_vs_per_domain": round(tp / tl, 3),
        "persistent_vs_graph_of_launches": round(tl / tb, 3),
        "hbm_GBps_equiv": round(cells * 8 / tl / 1e9, 1),
    }
    b.close()
    del fields
    torch.cuda.empty_cache()
    return out


ADJ_STEPS = 2000


def adjoint_rate(api, torch, inputs, steps=ADJ_STEPS, every=10, rate=12):
    """Misfit gradient of the 25-point wave on 512^3 (layered model, 15 Hz
    Ricker at the source cell) with 64 receivers on the plane z = 2 near the
    top face (8 x 8, spacing 64, offset 32), 2000 steps: forward with
    (p, p_prev) checkpoints every 10 steps compressed at 12 bits per value
    into pinned host memory (200 checkpoints, about 75 GiB), then the
    backward pass (restore, recompute, adjoint). The observed record comes
    from the model with a +5 % Gaussian blob (sigma = 12 cells) at
    (320, 256, 24), beside the source and under the receivers, so the
    direct wave crosses it within the first few hundred steps, by a forward
    run of the same problem."""
    import numpy as np

    shape = (512, 512, 512)
    nz, ny, nx = shape
    dt = inputs.wave_dt()
    c = np.float32(dt / 10.0)
    v = inputs.layered_velocity(shape, seed=1)
    vt = torch.from_numpy(v).cuda()
    ar = torch.arange(512, dtype=torch.float32, device="cuda")
    r2 = (ar[:, None, None] - 24.0) ** 2 + (ar[None, :, None] - 256.0) ** 2 + (ar[None, None, :] - 320.0) ** 2
    v_true = (vt * (1.0 + 0.05 * torch.exp(-r2 / (2.0 * 12.0 ** 2)))).contiguous()
    del r2
    amps = inputs.ricker(steps, dt)
    cell = inputs.source_cell(shape)
    rcv = np.array([(32 + 64 * (i % 8)) + nx * ((32 + 64 * (i // 8)) + ny * 2) for i in range(64)], np.int64)
    # the checkpoint store is one host allocation: pinned where the host can
    # pin it whole (this box pins about 48 GiB in all), else pageable memory
    # through which the runtime stages the copies; the record says which
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()  # pinned blocks cached by earlier sections
    t0 = time.perf_counter()
    want_steps = steps
    prob = api.WaveProblem(shape, steps, amps[:steps], cell, rcv, np.zeros((steps, 64), np.float32),
                           float(c), ckpt_every=every, ckpt_rate=rate)
    alloc_s = time.perf_counter() - t0
    prob.forward(v_true)  # the observed record (residuals against zero data)
    torch.cuda.synchronize()
    prob.obs.copy_(prob.res)
    del v_true
    J = [0.0]

    def fwd():
        J[0] = prob.forward(vt)

    tf = _timed(torch, fwd)
    tg = _timed(torch, lambda: prob.gradient(vt))
    cells = float(nx * ny * nz) * steps
    out = {
        "grid": list(shape), "steps": steps, "steps_asked": want_steps, "ckpt_every": every, "ckpt_rate": rate,
        "receivers": 64, "misfit": J[0],
        "forward_s": round(tf, 3), "backward_s": round(tg, 3),
        "gradient_gcell_steps_per_s": round(cells / (tf + tg) / 1e9, 2),
        "host_ckpt_bytes": int(prob.ckpt.numel()),
        "host_ckpt_pinned": prob.ckpt_pinned,
        "host_ckpt_alloc_s": round(alloc_s, 1),
        "ckpt_d2h_GBps": round(prob.ckpt.numel() / tf / 1e9, 1),
    }
    del prob
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# CPU baseline and probes
# ---------------------------------------------------------------------------

CPU_SAMPLE_PLANES = 512


def cpu_baseline(wi, state):
    """The oracle (plain C, OpenMP, FP64) on a bounded sample of the headline
    workload: one residency (12 FP64 wave steps, then decode(encode()) of
    p(n) and p(n-1) at 12 bits per value) on the first 512 planes of the
    1024^2 grid (half of it), from the developed state at step 2,160 (the
    source is in these planes)."""
    import numpy as np

    import oracle as O

    O.lib()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    sl = slice(0, CPU_SAMPLE_PLANES)
    p = state[0][sl].astype(np.float64)
    pm = state[1][sl].astype(np.float64)
    w = wi.w[sl].astype(np.float64)
    nz, ny, nx = p.shape
    cx, cy, cz = wi.cell
    src = (wi.amps[WAVE_START:WAVE_START + WAVE_K].astype(np.float64), cx + nx * (cy + ny * cz))
    t0 = time.perf_counter()
    p, pm = O.wave25_f64(p, pm, w, WAVE_K, src=src)
    p = O.codec_roundtrip_f64(p, HEADLINE_RATE)
    pm = O.codec_roundtrip_f64(pm, HEADLINE_RATE)
    t = time.perf_counter() - t0
    cells = float(nx * ny * nz) * WAVE_K
    out = {
        "value": cells / t / 1e9,
        "unit": "GCell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one residency ({WAVE_K} FP64 wave steps + decode(encode()) of p(n), p(n-1) at "
                  f"{HEADLINE_RATE} bits/value) on planes 0..{CPU_SAMPLE_PLANES - 1} of the 1024^2 x 1024 grid "
                  f"from the step-{WAVE_START} state, {t:.1f} s",
        "host_cpu": _cpu_model(),
    }
    out["single_thread"] = _oracle_one_thread(wi, state)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


CPU_ONE_THREAD_PLANES = 32


def _oracle_one_thread(wi, state):
    """The same residency on planes 0..31 with one OpenMP thread, in a child
    process (the thread count is fixed when the oracle's runtime starts)."""
    import subprocess
    import tempfile

    import numpy as np

    sl = slice(0, CPU_ONE_THREAD_PLANES)
    cx, cy, cz = wi.cell
    with tempfile.TemporaryDirectory() as td:
        np.save(os.path.join(td, "p.npy"), state[0][sl])
        np.save(os.path.join(td, "pm.npy"), state[1][sl])
        np.save(os.path.join(td, "w.npy"), wi.w[sl])
        np.save(os.path.join(td, "a.npy"), wi.amps[WAVE_START:WAVE_START + WAVE_K])
        code = (
            "import sys, time, numpy as np; sys.path.insert(0, sys.argv[1]); import oracle as O; d = sys.argv[2]\n"
            "p, pm, w = (np.load(d + f).astype(np.float64) for f in ('/p.npy', '/pm.npy', '/w.npy'))\n"
            "a = np.load(d + '/a.npy').astype(np.float64); nz, ny, nx = p.shape\n"
            f"src = (a, {cx} + nx * ({cy} + ny * {cz}))\n"
            "O.lib(); t0 = time.perf_counter()\n"
            f"p, pm = O.wave25_f64(p, pm, w, {WAVE_K}, src=src)\n"
            f"p = O.codec_roundtrip_f64(p, {HEADLINE_RATE}); pm = O.codec_roundtrip_f64(pm, {HEADLINE_RATE})\n"
            "print(time.perf_counter() - t0)\n"
        )
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code, ROOT, td], capture_output=True, text=True, env=env,
                           timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    t = float(r.stdout.strip().splitlines()[-1])
    cells = float(CPU_ONE_THREAD_PLANES * WAVE_SHAPE[1] * WAVE_SHAPE[2]) * WAVE_K
    return {"value": cells / t / 1e9, "unit": "GCell-updates/s", "cores": 1,
            "sample": f"the same residency on planes 0..{CPU_ONE_THREAD_PLANES - 1}, {t:.1f} s"}


def copy_probe():
    """A plain device copy of known size (1 GiB read + 1 GiB written), used to
    scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 4, "copies": 3}), flush=True)


def host_link(api, chunk, sdma=True):
    """Achievable host-link bandwidth with pinned memory, moved with the
    pipeline's engines in copies of the pipeline's size (one group of
    planes of one field): each direction alone, and both at once (about
    1 GiB each way, mean of 5 timed passes)."""
    nbytes = max(1, (1 << 30) // chunk) * chunk
    r = api.link_probe(nbytes, chunk, reps=5, sdma=sdma)
    return {k: (round(v, 2) if isinstance(v, float) else v) for k, v in r.items()}


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed rounds (12 time steps of the whole grid each)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline rate's rounds only (for profiler runs)")
    ap.add_argument("--no-full-run", action="store_true", help="skip the 4,320-step runs and their error curve")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the heat, codec, batched and adjoint workloads")
    ap.add_argument("--deadline", type=float, default=450.0,
                    help="seconds after start beyond which the 4,320-step runs stop (the line is still printed)")
    ap.add_argument("--copy-probe", action="store_true", help="only run the counter-calibration copy")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 replica of the paper's codes")
    ap.add_argument("--fp64-only", action="store_true", help="run the FP64 replica only (for profiler runs)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this benchmark runs on exactly one GPU (the pipeline is a single-GPU "
              "out-of-core pipeline; multi-GPU sharding is a design note only). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

    import torch

    from paper_2109_05410_amd import api, inputs

    torch.cuda.set_device(0)
    wi = WaveInputs(inputs)
    log(f"developing the wavefield to step {WAVE_START} in core")
    state = wave_state(api, torch, wi, WAVE_START)
    head_rates = [HEADLINE_RATE] * 3
    log("headline rounds")
    head = wave_window(api, torch, wi, state, head_rates, args.steps, args.warmup, profile=True)
    log(f"rate {HEADLINE_RATE}: {head['gcells_per_s']:.1f} GCell-updates/s, {head['ms_per_round']:.1f} ms/round")
    if args.headline_only:
        print(json.dumps({"headline": _rounded(head)}), flush=True)
        return
    # the link probe right after the headline, its pinned buffers allocated
    # like the stores' (later sections pin tens of GB more)
    chunk = head["group_planes"] * WAVE_SHAPE[1] * WAVE_SHAPE[2] * HEADLINE_RATE // 8
    link = host_link(api, chunk)
    log(f"host link: {link}")
    if args.fp64_only:
        rep = fp64_replica(api, torch, inputs, wi, state)
        err = fp64_error_curve(api, torch, inputs, wi, args.deadline)
        print(json.dumps({"fp64_replica": _rounded(rep), "fp64_error_curve": _rounded(err)}), flush=True)
        return
    variants = {f"rate{HEADLINE_RATE}": head}
    vr = max(2, min(args.steps, 8))
    for r in WAVE_RATES:
        if r == HEADLINE_RATE:
            continue
        key = "uncompressed" if r == 0 else f"rate{r}"
        variants[key] = wave_window(api, torch, wi, state, [r] * 3, args.steps if r else vr, 1)
        log(f"{key}: {variants[key]['gcells_per_s']:.1f} GCell-updates/s")
    # the paper's flow: every field's chunks streamed over the link every
    # residency (the snake's one retained slab aside)
    streamed = {}
    for r in (HEADLINE_RATE, 0):
        key = "uncompressed" if r == 0 else f"rate{r}"
        streamed[key] = wave_window(api, torch, wi, state, [r] * 3, args.steps if r else vr, 1,
                                    ro_device_store=False, retain=1)
        log(f"streamed read-only {key}: {streamed[key]['gcells_per_s']:.1f} GCell-updates/s")
    # one retained slab (the plain snake)
    variants[f"rate{HEADLINE_RATE}_retain_one_slab"] = wave_window(api, torch, wi, state, head_rates, args.steps, 1,
                                                                   retain=1)
    log(f"retain one slab: {variants[f'rate{HEADLINE_RATE}_retain_one_slab']['gcells_per_s']:.1f} GCell-updates/s")
    # the read-only field decoded once and kept on the device (4 GiB)
    variants[f"rate{HEADLINE_RATE}_resident_decoded_ro"] = wave_window(api, torch, wi, state, head_rates, vr, 1,
                                                                      resident_ro=True)
    # the paper's codes (Sec. VI), in the paper's flow: 1 = nothing compressed,
    # 2 = one read-write field (p(n-1)), 3 = the read-only field, 4 = both, at
    # the headline rate
    codes = {}
    for code, rates in ((2, [0, HEADLINE_RATE, 0]), (3, [0, 0, HEADLINE_RATE]), (4, [0, HEADLINE_RATE, HEADLINE_RATE])):
        codes[f"code{code}"] = wave_window(api, torch, wi, state, rates, vr, 1, ro_device_store=False, retain=1)
        log(f"code {code}: {codes[f'code{code}']['gcells_per_s']:.1f} GCell-updates/s")
    codes["code1"] = {"same_as": "streamed_read_only.uncompressed"}
    fp64 = None
    if not args.no_fp64:
        log("FP64 replica (1152^3, the paper's codes)")
        fp64 = fp64_replica(api, torch, inputs, wi, state)
    # one-way sweeps (every residency upward, every block through the host
    # link): the schedule without the snake's retained block
    oneway = {}
    for r in (HEADLINE_RATE, 0):
        key = "uncompressed" if r == 0 else f"rate{r}"
        oneway[key] = wave_window(api, torch, wi, state, [r] * 3, args.steps if r else vr, 1, snake=False)
        log(f"one-way {key}: {oneway[key]['gcells_per_s']:.1f} GCell-updates/s")
    # the per-block schedule of Fig. 2 (every block recomputes its halo)
    restart = {}
    for r in (HEADLINE_RATE, 0):
        key = "uncompressed" if r == 0 else f"rate{r}"
        restart[key] = wave_window(api, torch, wi, state, [r] * 3, 2, 1, block_restart=True)
        log(f"block restart {key}: {restart[key]['gcells_per_s']:.1f} GCell-updates/s")
    # per-stage breakdown (Sec. VI-B), 2 rounds per rate
    breakdown = {}
    for r in WAVE_RATES:
        key = "uncompressed" if r == 0 else f"rate{r}"
        b = wave_window(api, torch, wi, state, [r] * 3, 1, 0, breakdown_rounds=2, snake=False)
        breakdown[key] = {"ms_per_round": b["breakdown_ms_per_round"], "wall_ms_per_round": b["breakdown_wall_ms_per_round"]}
        log(f"breakdown {key}: {breakdown[key]}")
    extras = {}
    if not args.no_extras:
        u0 = inputs.heat_uniform(HEAT_SHAPE, seed=0)
        heat = {}
        for r in HEAT_RATES:
            heat["uncompressed" if r == 0 else f"rate{r}"] = heat_variant(api, torch, u0, r, 3, 1, breakdown=True)
        heat["snake_rate8"] = heat_variant(api, torch, u0, 8, 3, 1, snake=True)
        heat["snake_uncompressed"] = heat_variant(api, torch, u0, 0, 1, 1, snake=True)
        heat["block_restart_rate8"] = heat_variant(api, torch, u0, 8, 2, 1, block_restart=True)
        heat["block_restart_uncompressed"] = heat_variant(api, torch, u0, 0, 1, 1, block_restart=True)
        heat["in_core_gcells_per_s"] = heat_in_core_rate(api, torch, u0)
        extras["heat_512"] = heat
        log(f"heat 512^3: rate 8 {heat['rate8']['gcells_per_s']:.1f}, uncompressed "
            f"{heat['uncompressed']['gcells_per_s']:.1f} GCell-updates/s")
        extras["in_core_64"] = small_in_core(api, torch, inputs)
        extras["codec_512"] = codec_rates(api, torch, u0)
        extras["batched_heat"] = batched_rate(api, torch, inputs)
        log(f"batched: {extras['batched_heat']}")
        extras["adjoint_512"] = adjoint_rate(api, torch, inputs)
        log(f"adjoint: {extras['adjoint_512']}")
        del u0
    full = None
    if not args.no_full_run:
        log("whole 4,320-step runs")
        full = wave_full_run(api, torch, inputs, wi, FULL_RUN_RATES, args.deadline)
        if fp64 is not None:
            log("FP64 error curve (512^3, the paper's codes)")
            fp64["error_curve_512"] = fp64_error_curve(api, torch, inputs, wi, args.deadline)
    traffic = measured_counters("hbm_bytes_per_launch")
    alu_ops = measured_counters("alu_ops_per_launch")
    kname, kstat = "fused_kernel", head["kernel"]
    achieved = kstat["achieved_GBps"]
    raw = variants["uncompressed"]
    line = {
        "metric": METRIC,
        "value": round(head["gcells_per_s"], 3),
        "unit": "GCell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_round"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "wave25 1024^3 FP32 (p, p_prev, read-only w), layered 1500-4500 m/s model, 15 Hz Ricker, "
                        "8 z-slabs, k=12 (halo 48), device arena capped at 8 GiB, all three host stores at "
                        "12 bits/value, snake sweeps retaining as many slabs as the arena holds, w's compressed "
                        "store held in the arena; one bench step = one "
                        "round (every block advanced 12 steps) from the step-2160 state of the 4320-step run",
            "schedule": "shared levels, snake sweeps (alternating direction; the last blocks of a residency, as "
                        "many slabs as the arena holds, kept compressed on the device); the "
                        "read-only store copied into the arena once and decoded from there every residency",
            "grid": list(WAVE_SHAPE), "nslabs": WAVE_SLABS, "k": WAVE_K, "time_steps_per_bench_step": WAVE_K,
            "device_cap_bytes": WAVE_CAP, "rate_bits_per_value": HEADLINE_RATE,
        },
        "speedup_vs_uncompressed": round(head["gcells_per_s"] / raw["gcells_per_s"], 3),
        "speedup_vs_uncompressed_streamed": round(head["gcells_per_s"] / streamed["uncompressed"]["gcells_per_s"], 3),
        "variants": _rounded(variants),
        "streamed_read_only": _rounded(streamed),
        "paper_codes": _rounded(codes),
        "fp64_replica": _rounded(fp64) if fp64 else None,
        "block_restart": _rounded(restart),
        "one_way_sweeps": _rounded(oneway),
        "breakdown_ms_per_round": _rounded(breakdown),
        "full_run_4320": _rounded(full),
        "other_workloads": _rounded(extras),
        "host_link": link,
        "paper_context": "1.20x over uncompressed out-of-core (V100-PCIe, FP64 25-point wave, 24/64 bits, Sec. VI-A)",
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic.get(kname) if isinstance(traffic, dict) else None,
            "bytes_per_launch": round(kstat["bytes_per_launch"]),
            "avg_launch_us": round(kstat["avg_launch_us"], 2) if kstat["avg_launch_us"] else None,
        },
    }
    ops = alu_ops.get(kname) if isinstance(alu_ops, dict) else None
    alu_achieved = ops / (kstat["avg_launch_us"] * 1e-6) / 1e12 if ops and kstat["avg_launch_us"] else None
    line["alu_roofline"] = {
        "bound": "alu",
        "kernel": kname,
        "achieved": round(alu_achieved, 2) if alu_achieved else None,
        "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "T VALU lane-ops/s",
        "frac": round(alu_achieved / VALU_PEAK_TOPS, 4) if alu_achieved else None,
        "ops_per_launch": ops,
        "ops_source": "SQ_INSTS_VALU x 64 from profiles/wave1024_rate12_counters.json (issued, not algorithmic)",
    }
    # The host link as a bound on the round: each direction's bytes at that
    # direction's probe rate alone, and the larger direction's bytes at the
    # rate each way with both directions busy (copies of the pipeline's size on
    # its engines); the round cannot be shorter than the largest of these.
    h2d_pk, d2h_pk, bi_pk = link.get("h2d_GBps"), link.get("d2h_GBps"), link.get("bidir_GBps_each")
    hb, db = head["h2d_bytes_per_round"], head["d2h_bytes_per_round"]
    bounds = {}
    if h2d_pk:
        bounds["host-to-device alone"] = hb / (h2d_pk * 1e9) * 1e3
    if d2h_pk:
        bounds["device-to-host alone"] = db / (d2h_pk * 1e9) * 1e3
    if bi_pk:
        bounds["both directions at once"] = max(hb, db) / (bi_pk * 1e9) * 1e3
    which = max(bounds, key=bounds.get) if bounds else None
    t_bound = bounds[which] if which else None
    line["host_link_roofline"] = {
        "bound": f"host link, {which}" if which else None,
        "achieved_GBps_h2d": round(head["h2d_GBps"], 2),
        "achieved_GBps_d2h": round(head["d2h_GBps"], 2),
        "peak_GBps_h2d_alone": h2d_pk,
        "peak_GBps_d2h_alone": d2h_pk,
        "peak_GBps_each_way_both_busy": bi_pk,
        "link_bound_ms_per_round": round(t_bound, 2) if t_bound else None,
        "ms_per_round": round(head["ms_per_round"], 2),
        "frac": round(t_bound / head["ms_per_round"], 4) if t_bound else None,
        "peak_source": "host_link: ~1 GiB in pinned copies of the pipeline's group size on its engines "
                       "(hipMemcpyAsync up, SDMA down), each direction alone and both at once, measured right after "
                       "the headline; frac = link-bound time / measured round time",
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wi, state)
    line["bench_wall_s"] = round(time.perf_counter() - T_START, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
