"""Python API over liboocs. PyTorch supplies device memory, pinned host
memory and streams; every step of the computation runs in the HIP library.

Fields are torch tensors shaped (nz, ny, nx), float32, C-contiguous
(x fastest), on the current CUDA (HIP) device.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return C.c_void_p(t.data_ptr())


def _field(t: torch.Tensor, name: str):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 3:
        raise ValueError(f"{name} must be a contiguous float32 (nz, ny, nx) device tensor")
    nz, ny, nx = t.shape
    return nx, ny, nz


# ---------------------------------------------------------------------------
# Codec
# ---------------------------------------------------------------------------

def codec_bytes(nx: int, ny: int, nz: int, rate: int) -> int:
    return int(L.lib().oocs_codec_bytes(nx, ny, nz, rate))


def codec_encode(field: torch.Tensor, rate: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Encode a (nz, ny, nx) float32 field; returns the words as an int64
    tensor (bit pattern of the uint64 words)."""
    nx, ny, nz = _field(field, "field")
    nb = codec_bytes(nx, ny, nz, rate)
    if nb == 0:
        L.check(L.OOCS_E_ALIGN if rate > 0 else L.OOCS_E_RATE)
    if out is None:
        out = torch.empty(nb // 8, dtype=torch.int64, device=field.device)
    L.check(L.lib().oocs_codec_encode(_dptr(field), nx, ny, nz, nx, nx * ny, rate, _dptr(out),
                                      out.numel() * 8, _stream_ptr(stream)))
    return out


def codec_decode(words: torch.Tensor, shape, rate: int, out: torch.Tensor | None = None, stream=None,
                 mid: bool = False) -> torch.Tensor:
    """mid: mid-point reconstruction of the digits the budget cut off."""
    nz, ny, nx = shape
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=words.device)
    _field(out, "out")
    r = rate | (L.OOCS_DECODE_MIDPOINT if mid else 0)
    L.check(L.lib().oocs_codec_decode(_dptr(words), words.numel() * words.element_size(), nx, ny, nz, r,
                                      _dptr(out), nx, nx * ny, _stream_ptr(stream)))
    return out


def codec_encode_stages(blocks: torch.Tensor, rate: int) -> dict:
    """blocks: (N, 64) float32 device tensor, natural in-block order."""
    n = blocks.shape[0]
    dev = blocks.device
    o = {
        "emax": torch.empty(n, dtype=torch.int32, device=dev),
        "q": torch.empty((n, 64), dtype=torch.int32, device=dev),
        "t": torch.empty((n, 64), dtype=torch.int32, device=dev),
        "u": torch.empty((n, 64), dtype=torch.int32, device=dev),
        "plane": torch.empty((n, 32), dtype=torch.int64, device=dev),
        "words": torch.empty((n, rate), dtype=torch.int64, device=dev),
        "bits_used": torch.empty(n, dtype=torch.int32, device=dev),
    }
    L.check(L.lib().oocs_codec_encode_stages(_dptr(blocks.contiguous()), n, rate, _dptr(o["emax"]), _dptr(o["q"]),
                                             _dptr(o["t"]), _dptr(o["u"]), _dptr(o["plane"]), _dptr(o["words"]),
                                             _dptr(o["bits_used"]), _stream_ptr()))
    return o


def codec_decode_stages(words: torch.Tensor, rate: int, mid: bool = False) -> dict:
    """words: (N, rate) int64 device tensor; mid: mid-point reconstruction."""
    n = words.shape[0]
    dev = words.device
    o = {
        "emax": torch.empty(n, dtype=torch.int32, device=dev),
        "plane": torch.empty((n, 32), dtype=torch.int64, device=dev),
        "u": torch.empty((n, 64), dtype=torch.int32, device=dev),
        "q": torch.empty((n, 64), dtype=torch.int32, device=dev),
        "out": torch.empty((n, 64), dtype=torch.float32, device=dev),
    }
    L.check(L.lib().oocs_codec_decode_stages(_dptr(words.contiguous()), n, rate | (L.OOCS_DECODE_MIDPOINT if mid else 0),
                                             _dptr(o["emax"]), _dptr(o["plane"]),
                                             _dptr(o["u"]), _dptr(o["q"]), _dptr(o["out"]), _stream_ptr()))
    return o


# ---------------------------------------------------------------------------
# FP64 format and FP64 wave step (the paper's precision)
# ---------------------------------------------------------------------------

def _field64(t: torch.Tensor, name: str):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 3:
        raise ValueError(f"{name} must be a contiguous float64 (nz, ny, nx) device tensor")
    nz, ny, nx = t.shape
    return nx, ny, nz


def codec64_encode(field: torch.Tensor, rate: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    nx, ny, nz = _field64(field, "field")
    nb = int(L.lib().oocs_codec64_bytes(nx, ny, nz, rate))
    if nb == 0:
        L.check(L.OOCS_E_ALIGN if rate > 0 else L.OOCS_E_RATE)
    if out is None:
        out = torch.empty(nb // 8, dtype=torch.int64, device=field.device)
    L.check(L.lib().oocs_codec64_encode(_dptr(field), nx, ny, nz, nx, nx * ny, rate, _dptr(out), out.numel() * 8,
                                        _stream_ptr(stream)))
    return out


def codec64_decode(words: torch.Tensor, shape, rate: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    nz, ny, nx = shape
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float64, device=words.device)
    _field64(out, "out")
    L.check(L.lib().oocs_codec64_decode(_dptr(words), words.numel() * words.element_size(), nx, ny, nz, rate,
                                        _dptr(out), nx, nx * ny, _stream_ptr(stream)))
    return out


def codec64_encode_stages(blocks: torch.Tensor, rate: int) -> dict:
    """blocks: (N, 64) float64 device tensor, natural in-block order."""
    n = blocks.shape[0]
    dev = blocks.device
    o = {
        "emax": torch.empty(n, dtype=torch.int32, device=dev),
        "q": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "t": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "u": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "plane": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "words": torch.empty((n, rate), dtype=torch.int64, device=dev),
        "bits_used": torch.empty(n, dtype=torch.int32, device=dev),
    }
    L.check(L.lib().oocs_codec64_encode_stages(_dptr(blocks.contiguous()), n, rate, _dptr(o["emax"]), _dptr(o["q"]),
                                               _dptr(o["t"]), _dptr(o["u"]), _dptr(o["plane"]), _dptr(o["words"]),
                                               _dptr(o["bits_used"]), _stream_ptr()))
    return o


def codec64_decode_stages(words: torch.Tensor, rate: int) -> dict:
    n = words.shape[0]
    dev = words.device
    o = {
        "emax": torch.empty(n, dtype=torch.int32, device=dev),
        "plane": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "u": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "q": torch.empty((n, 64), dtype=torch.int64, device=dev),
        "out": torch.empty((n, 64), dtype=torch.float64, device=dev),
    }
    L.check(L.lib().oocs_codec64_decode_stages(_dptr(words.contiguous()), n, rate, _dptr(o["emax"]), _dptr(o["plane"]),
                                               _dptr(o["u"]), _dptr(o["q"]), _dptr(o["out"]), _stream_ptr()))
    return o


def wave25_step_k_f64(p: torch.Tensor, pm: torch.Tensor, w: torch.Tensor, k: int, src=None, stream=None):
    """k FP64 leapfrog steps in place on (pm, p) = (p(n-1), p(n)).
    src = (amplitudes (k,), (x, y, z)) or None."""
    nx, ny, nz = _field64(p, "p")
    _field64(pm, "pm")
    _field64(w, "w")
    amps = None
    sx = sy = sz = -1
    if src is not None:
        a, (sx, sy, sz) = src
        amps = np.ascontiguousarray(a, dtype=np.float64)
        if amps.size < k:
            raise ValueError("need one source amplitude per step")
    ap = amps.ctypes.data_as(C.c_void_p) if amps is not None else None
    L.check(L.lib().oocs_wave25_step_k_f64(_dptr(p), _dptr(pm), _dptr(w), nx, ny, nz, k, ap, sx, sy, sz,
                                           _stream_ptr(stream)))
    return p, pm


def codec64_roundtrip_(f: torch.Tensor, rate: int, scratch: torch.Tensor | None = None) -> torch.Tensor:
    """f <- decode(encode(f)) in place with the FP64 format (on the device)."""
    words = codec64_encode(f, rate, out=scratch)
    codec64_decode(words, tuple(f.shape), rate, out=f)
    return f


def wave64_compressed_run(p, pm, w, steps: int, k: int, src=None, rate_p=0, rate_pm=0, rate_w=0,
                          initial: bool = True):
    """The compressed out-of-core schedule's state in FP64, on the GPU: the
    stores start as decode(encode()) of the initial fields (initial=True;
    the read-only w only then), and every k steps the read-write fields pass
    through decode(encode()) with the FP64 format. The out-of-core
    decomposition is exact, so this is the state a blocked FP64 run
    reaches. Works in place on the device tensors (pm, p, w).
    src = (amplitudes (steps,), (x, y, z)) or None."""
    if initial:
        for f, r in ((w, rate_w), (p, rate_p), (pm, rate_pm)):
            if r:
                codec64_roundtrip_(f, r)
    done = 0
    while done < steps:
        n = min(k, steps - done)
        s = None if src is None else (np.asarray(src[0])[done:done + n], src[1])
        wave25_step_k_f64(p, pm, w, n, src=s)
        if rate_p:
            codec64_roundtrip_(p, rate_p)
        if rate_pm:
            codec64_roundtrip_(pm, rate_pm)
        done += n
    return p, pm


# ---------------------------------------------------------------------------
# In-core steps
# ---------------------------------------------------------------------------

def heat7_step_k(u: torch.Tensor, alpha: float, k: int, tmp: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """k heat steps in place on u. tmp: scratch of u's shape on u's device,
    not overlapping u (allocated here if None)."""
    nx, ny, nz = _field(u, "u")
    if tmp is None:
        tmp = torch.empty_like(u)
    else:
        _field(tmp, "tmp")
        if tmp.shape != u.shape or tmp.device != u.device:
            raise ValueError("tmp must have u's shape and device")
        ua, ta = u.data_ptr(), tmp.data_ptr()
        nb = u.numel() * 4
        if ua < ta + nb and ta < ua + nb:
            raise ValueError("tmp must not overlap u")
    if stream is not None:
        # the kernels on `stream` use tmp after this call returns: keep the
        # caching allocator from handing its block out before they finish
        tmp.record_stream(stream)
    L.check(L.lib().oocs_heat7_step_k(_dptr(u), _dptr(tmp), nx, ny, nz, C.c_float(alpha), k, _stream_ptr(stream)))
    return u


def wave25_step_k(p: torch.Tensor, pm: torch.Tensor, w: torch.Tensor, k: int, src=None, stream=None):
    """k leapfrog steps in place on (pm, p) = (p(n-1), p(n)).
    src = (amplitudes (k,) float32 array, (x, y, z)) or None."""
    nx, ny, nz = _field(p, "p")
    _field(pm, "pm")
    _field(w, "w")
    amps = None
    sx = sy = sz = -1
    if src is not None:
        a, (sx, sy, sz) = src
        amps = np.ascontiguousarray(a, dtype=np.float32)
        if amps.size < k:
            raise ValueError("need one source amplitude per step")
    ap = amps.ctypes.data_as(C.c_void_p) if amps is not None else None
    L.check(L.lib().oocs_wave25_step_k(_dptr(p), _dptr(pm), _dptr(w), nx, ny, nz, k, ap, sx, sy, sz,
                                       _stream_ptr(stream)))
    return p, pm


# ---------------------------------------------------------------------------
# Out-of-core plan
# ---------------------------------------------------------------------------

HEAT7 = L.OOCS_HEAT7
WAVE25 = L.OOCS_WAVE25
RETAIN_MAX = L.OOCS_RETAIN_MAX


def link_probe(nbytes: int = 256 << 20, chunk: int = 4 << 20, reps: int = 3, sdma: int = 1) -> dict:
    """Host-link bandwidth with pinned buffers, moved with the pipeline's
    engines (host to device by hipMemcpyAsync, device to host on an SDMA
    engine where available; sdma >= 2: each chunk split over that many
    engines): each direction alone and both at once, GB/s."""
    h_in = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    h_out = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d_a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d_b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = (C.c_double * 4)()
    L.check(L.lib().oocs_link_probe(d_a.data_ptr(), d_b.data_ptr(), h_in.data_ptr(), h_out.data_ptr(), nbytes, chunk,
                                    reps, int(sdma), out))
    return {"h2d_GBps": out[0], "d2h_GBps": out[1], "bidir_GBps_each": out[2],
            "d2h_engine": "sdma" if out[3] else "hipMemcpyAsync", "bytes": nbytes, "chunk_bytes": chunk}


@dataclass
class RunStats:
    wall_ms: float
    enqueue_ms: float
    rounds: int
    h2d_bytes: int
    d2h_bytes: int
    cell_updates: int
    launches: int
    codec_bytes: int
    stencil_bytes: int
    kernel_ms: float
    xfer_bytes: int
    timed_launches: int
    timed_bytes: int
    sdma_copies: int
    stage_ms: tuple
    arena_bytes: int

    STAGES = ("h2d", "decode", "step", "encode", "d2h")

    @property
    def breakdown_ms(self) -> dict:
        """Per-stage summed durations (plans with set_breakdown(True))."""
        return dict(zip(self.STAGES, self.stage_ms))

    @property
    def gcells_per_s(self) -> float:
        return self.cell_updates / (self.wall_ms * 1e-3) / 1e9 if self.wall_ms > 0 else 0.0


class OutOfCorePlan:
    """An out-of-core pipeline over a host store, using at most `arena_bytes`
    of device memory (one torch allocation made here, handed to the library).

    Field slots: heat uses 0 (u); the wave uses 0 = p(n), 1 = p(n-1),
    2 = w (read-only).

    block_restart: every block restarts the level fronts and recomputes its
    halo (the per-block schedule of Fig. 2) instead of sharing every level's
    planes with its neighbour. Transfers: hipMemcpyAsync on two copy streams
    (the three-stream pipeline of Sec. V-B, default); kernel_stores:
    write-back by STORE jobs in the pipeline kernel; kernel_transfers: loads
    by FETCH jobs as well. level_by_level (heat,
    k <= 4): one job and one ring per time level instead of one temporally
    blocked job per tick. resident_ro (wave): the read-only field is decoded
    once into the arena and stays there instead of being streamed every
    residency. snake: residencies alternate the sweep direction and the
    block a residency ends with stays on the device (compressed, or raw if
    uncompressed) for the next one; retain (snake): the region kept there
    spans that many slabs (0 = one, at most nslabs), or as many as the
    arena holds with RETAIN_MAX. Results are identical. midpoint: every
    decode reconstructs the digits the budget cut off at the middle of their
    range (a different, lower-error state). fp64 (wave): FP64 fields and
    the FP64 block format (rates up to 68); put/get take and return float64
    arrays; copy-engine transfers only. ro_device_store (wave): the
    read-only field's store is copied once into the arena and decoded from
    there every residency (no host-link traffic for it after the first
    run)."""

    def __init__(self, shape, stencil: int, nslabs: int, k: int, rates, arena_bytes: int,
                 alpha: float = 0.1, src_cell=None, group: int = 0, nstage: int = 0,
                 planning_only: bool = False, device=None, block_restart: bool = False,
                 kernel_transfers: bool = False, level_by_level: bool = False, kernel_stores: bool = False,
                 resident_ro: bool = False, snake: bool = False, midpoint: bool = False, fp64: bool = False,
                 ro_device_store: bool = False, retain: int = 0):
        nz, ny, nx = shape
        cfg = L.Config()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.stencil = stencil
        cfg.nslabs = nslabs
        cfg.k = k
        cfg.group = group
        for i in range(L.OOCS_MAX_FIELDS):
            cfg.rate[i] = rates[i] if i < len(rates) else 0
        cfg.nstage = nstage
        cfg.alpha = alpha
        cfg.flags = ((L.OOCS_PLAN_BLOCK_RESTART if block_restart else 0)
                     | (L.OOCS_PLAN_KERNEL_TRANSFERS if kernel_transfers else 0)
                     | (L.OOCS_PLAN_LEVEL_BY_LEVEL if level_by_level else 0)
                     | (L.OOCS_PLAN_KERNEL_STORES if kernel_stores else 0)
                     | (L.OOCS_PLAN_RESIDENT_RO if resident_ro else 0)
                     | (L.OOCS_PLAN_SNAKE if snake else 0)
                     | (L.OOCS_PLAN_MIDPOINT if midpoint else 0)
                     | (L.OOCS_PLAN_FP64 if fp64 else 0)
                     | (L.OOCS_PLAN_RO_DEVICE_STORE if ro_device_store else 0))
        sx, sy, sz = src_cell if src_cell is not None else (-1, -1, -1)
        cfg.src_x, cfg.src_y, cfg.src_z = sx, sy, sz
        cfg.retain = retain
        self.cfg = cfg
        self.shape = (nz, ny, nx)
        self.dtype = np.float64 if fp64 else np.float32
        self.stencil = stencil
        self.arena = None
        ptr = None
        if not planning_only:
            self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device or "cuda")
            ptr = C.c_void_p(self.arena.data_ptr())
        h = C.c_void_p()
        L.check(L.lib().oocs_plan_create(C.byref(cfg), ptr, arena_bytes, C.byref(h)))
        self._h = h
        self.nfields = 1 if stencil == HEAT7 else 3

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().oocs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> dict:
        i = L.PlanInfo()
        L.check(L.lib().oocs_plan_get_info(self._h, C.byref(i)))
        return {
            "group": i.group, "halo": i.halo, "radius": i.radius, "nlevels": i.nlevels, "nrings": i.nrings,
            "ring_planes": list(i.ring_planes[: i.nrings]), "plane_bytes": i.plane_bytes,
            "arena_needed": i.arena_needed, "nstage": i.nstage, "store_bytes": list(i.store_bytes),
            "retained_planes": i.retained_planes,
        }

    def slab(self, i: int) -> dict:
        s = L.SlabInfo()
        L.check(L.lib().oocs_plan_slab(self._h, i, C.byref(s)))
        return {k: (list(getattr(s, k)) if k.endswith(("_off", "_bytes")) else getattr(s, k)) for k, _ in s._fields_}

    def schedule(self, kr: int, variant: int = 0) -> list[dict]:
        """Op list of a residency of kr steps; variant: OOCS_SCHED_* bits
        (snake plans)."""
        n = L.check(L.lib().oocs_plan_schedule_variant_len(self._h, kr, variant))
        ops = []
        o = L.Op()
        for i in range(n):
            L.check(L.lib().oocs_plan_schedule_variant_op(self._h, kr, variant, i, C.byref(o)))
            ops.append({k: getattr(o, k) for k, _ in o._fields_})
        return ops

    def variant(self, i: int, nres: int) -> int:
        """Schedule variant oocs_run uses for residency i of nres."""
        if not self.cfg.flags & L.OOCS_PLAN_SNAKE:
            return 0
        return ((L.OOCS_SCHED_MIRROR if i % 2 else 0) | (L.OOCS_SCHED_RETAIN_IN if i > 0 else 0)
                | (L.OOCS_SCHED_RETAIN_OUT if i < nres - 1 else 0))

    def store_bytes(self, f: int) -> int:
        return int(L.lib().oocs_store_bytes(self._h, f))

    def new_store(self, f: int) -> torch.Tensor:
        """A pinned host buffer for field slot f's store."""
        return torch.empty(self.store_bytes(f), dtype=torch.uint8, pin_memory=True)

    def put(self, f: int, field, store: torch.Tensor):
        """Build store f from a host field (numpy or CPU tensor; FP32, or FP64
        in an fp64 plan)."""
        a = np.ascontiguousarray(field.numpy() if isinstance(field, torch.Tensor) else field, dtype=self.dtype)
        if a.shape != self.shape:
            raise ValueError("field shape mismatch")
        L.check(L.lib().oocs_store_put(self._h, f, a.ctypes.data_as(C.c_void_p), C.c_void_p(store.data_ptr())))

    def get(self, f: int, store: torch.Tensor) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.dtype)
        L.check(L.lib().oocs_store_get(self._h, f, C.c_void_p(store.data_ptr()), out.ctypes.data_as(C.c_void_p)))
        return out

    def run(self, stores, steps: int, src_amps=None) -> RunStats:
        ptrs = (C.c_void_p * L.OOCS_MAX_FIELDS)()
        for i, s in enumerate(stores):
            ptrs[i] = s.data_ptr() if s is not None else None
        amps = None
        if src_amps is not None:
            amps = np.ascontiguousarray(src_amps, dtype=np.float32)
            if amps.size < steps:
                raise ValueError("need one source amplitude per step")
        st = L.Stats()
        L.check(L.lib().oocs_run(self._h, ptrs, steps, amps.ctypes.data_as(C.c_void_p) if amps is not None else None,
                                 C.byref(st)))
        vals = [getattr(st, name) for name, _ in L.Stats._fields_]
        vals[[n for n, _ in L.Stats._fields_].index("stage_ms")] = tuple(st.stage_ms)
        return RunStats(*vals)

    def set_profiling(self, on, every: int = 1):
        """Time every `every`-th launch with events (on=False: no timing)."""
        L.check(L.lib().oocs_plan_set_profiling(self._h, int(every) if on else 0))

    def set_breakdown(self, on: bool):
        """Per-stage timing of later runs (one launch per stage per tick, every
        copy timed); RunStats.breakdown_ms then holds the stage times."""
        L.check(L.lib().oocs_plan_set_breakdown(self._h, 1 if on else 0))

    def set_graphs(self, on: bool):
        L.check(L.lib().oocs_plan_set_graphs(self._h, 1 if on else 0))

    def set_host_waits(self, on: bool):
        """Op-by-op issue: block the host on pending cross-stream events (True,
        default) or make the stream wait on them (False)."""
        L.check(L.lib().oocs_plan_set_host_waits(self._h, 1 if on else 0))

    def set_sdma(self, on):
        """Device-to-host copies on an SDMA engine through the HSA runtime
        (True or 1, default, where available), split over `on` engines (an
        int >= 2), or with hipMemcpyAsync (False or 0)."""
        L.check(L.lib().oocs_plan_set_sdma(self._h, int(on)))

    @property
    def sdma_available(self) -> bool:
        return bool(L.lib().oocs_plan_sdma_available(self._h))



# ---------------------------------------------------------------------------
# Misfit gradient (adjoint with compressed checkpoints) and autograd
# ---------------------------------------------------------------------------

class WaveProblem:
    """A wave misfit problem: source wavelet, receivers, observed records and
    checkpoint policy. Holds the device workspace and the host checkpoint
    store (allocated here with torch, handed to the library). pinned: True =
    pinned host memory, False = pageable memory (the runtime stages the
    copies), None = pinned where the host can pin the whole store, else
    pageable (ckpt_pinned says which)."""

    def __init__(self, shape, steps: int, src_amps, src_cell, rcv_cells, observed, vscale: float,
                 ckpt_every: int = 10, ckpt_rate: int = 0, device="cuda", pinned: bool | None = None):
        nz, ny, nx = shape
        c = L.AdjointCfg()
        c.nx, c.ny, c.nz = nx, ny, nz
        c.steps = steps
        c.ckpt_every = ckpt_every
        c.ckpt_rate = ckpt_rate
        rcv = np.ascontiguousarray(rcv_cells, dtype=np.int64).reshape(-1)
        if rcv.size and (rcv.min() < 0 or rcv.max() >= nx * ny * nz):
            raise ValueError("receiver index outside the grid")
        c.nrcv = rcv.size
        c.src_x, c.src_y, c.src_z = src_cell
        c.vscale = vscale
        self.cfg = c
        self.shape = (nz, ny, nx)
        self.src = np.ascontiguousarray(src_amps, dtype=np.float32)
        if self.src.size < steps:
            raise ValueError("need one source amplitude per step")
        self.rcv = torch.from_numpy(rcv).to(device)
        obs = torch.as_tensor(observed, dtype=torch.float32).reshape(steps, rcv.size)
        self.obs = obs.to(device).contiguous()
        self.res = torch.empty_like(self.obs)
        wb = int(L.lib().oocs_adjoint_workspace_bytes(C.byref(c)))
        if wb == 0:
            L.check(L.OOCS_E_ARG)
        self.work = torch.empty(wb, dtype=torch.uint8, device=device)
        nbytes = int(L.lib().oocs_adjoint_ckpt_bytes(C.byref(c)))
        self.ckpt = None
        if pinned is not False:
            try:
                self.ckpt = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
            except (RuntimeError, torch.OutOfMemoryError):
                if pinned:
                    raise
        self.ckpt_pinned = self.ckpt is not None
        if self.ckpt is None:
            self.ckpt = torch.empty(nbytes, dtype=torch.uint8)
        # forward() overwrites the one checkpoint store and residual buffer:
        # each call gets a new generation, and a gradient is only valid for
        # the generation it was taken from
        self.generation = 0

    def _common(self, v):
        _field(v, "v")
        return (C.byref(self.cfg), _dptr(v), self.src.ctypes.data_as(C.c_void_p), _dptr(self.rcv))

    def forward(self, v: torch.Tensor) -> float:
        J = C.c_double()
        cfg, pv, ps, pr = self._common(v)
        self.generation += 1  # the store is being overwritten: earlier generations are stale from here on
        L.check(L.lib().oocs_wave_forward_ckpt(cfg, pv, ps, pr, _dptr(self.obs), _dptr(self.res), _dptr(self.work),
                                               self.work.numel(), C.c_void_p(self.ckpt.data_ptr()), C.byref(J),
                                               _stream_ptr()))
        return J.value

    def gradient(self, v: torch.Tensor, generation: int | None = None) -> torch.Tensor:
        """dJ/dv for the checkpoints of the last forward() call. generation:
        the value of self.generation right after the forward() whose
        gradient is wanted; a later forward() makes it stale (error)."""
        if generation is not None and generation != self.generation:
            raise RuntimeError(f"stale gradient request: the checkpoints of forward #{generation} were overwritten "
                               f"by forward #{self.generation} on the same WaveProblem")
        g = torch.empty_like(v)
        cfg, pv, ps, pr = self._common(v)
        L.check(L.lib().oocs_wave_adjoint(cfg, pv, ps, pr, _dptr(self.res), _dptr(self.work), self.work.numel(),
                                          C.c_void_p(self.ckpt.data_ptr()), _dptr(g), _stream_ptr()))
        return g


class WaveMisfit(torch.autograd.Function):
    """J(v) = 1/2 sum |S p(t) - d(t)|^2 for the 25-point wave from rest;
    backward runs the adjoint with checkpoint recompute on the GPU."""

    @staticmethod
    def forward(ctx, v, problem: WaveProblem):
        v = v.detach().contiguous()
        J = problem.forward(v)
        ctx.problem = problem
        ctx.generation = problem.generation
        ctx.save_for_backward(v)
        return torch.tensor(J, dtype=torch.float64, device=v.device)

    @staticmethod
    def backward(ctx, gJ):
        (v,) = ctx.saved_tensors
        g = ctx.problem.gradient(v, generation=ctx.generation)
        return (g * gJ.to(g.dtype)), None


# ---------------------------------------------------------------------------
# Batched in-core heat domains
# ---------------------------------------------------------------------------

class HeatBatch:
    """Independent heat domains advanced together: by default one launch per
    k steps for all domains, all launches replayed as one graph;
    set_persistent(True): one persistent kernel per run (items of every
    domain, tile and group of k steps from a device queue). `fields` are
    (nz, ny, nx) float32 device tensors, updated in place by run(). depth:
    0 = temporal-blocking depth chosen by the autotuner, or 1, 2, 4."""

    def __init__(self, fields, alpha: float = 0.1, tune: bool = True, tune_cache: str | None = None,
                 depth: int = 0):
        self.fields = [f for f in fields]
        for f in self.fields:
            _field_any(f)
        self.scratch = [torch.empty_like(f) for f in self.fields]
        n = len(self.fields)
        arr = (L.Domain * n)()
        for i, (f, s) in enumerate(zip(self.fields, self.scratch)):
            nz, ny, nx = f.shape
            arr[i] = L.Domain(f.data_ptr(), s.data_ptr(), nx, ny, nz)
        self._arr = arr
        self.table = torch.empty(int(L.lib().oocs_batch_table_bytes(n)), dtype=torch.uint8, device=self.fields[0].device)
        h = C.c_void_p()
        L.check(L.lib().oocs_batch_create(arr, n, C.c_float(alpha), _dptr(self.table), self.table.numel(),
                                          tune_cache.encode() if tune_cache else None, 1 if tune else 0,
                                          int(depth), _stream_ptr(), C.byref(h)))
        self._h = h

    def run(self, steps: int, stream=None, check: bool = False):
        """Advance every domain; check=True waits for the run and raises if a
        persistent launch's bounded wait gave up."""
        L.check(L.lib().oocs_batch_run(self._h, steps, _stream_ptr(stream)))
        if check:
            self.check(stream)

    def check(self, stream=None):
        L.check(L.lib().oocs_batch_check(self._h, _stream_ptr(stream)))

    def set_persistent(self, on: bool):
        L.check(L.lib().oocs_batch_set_persistent(self._h, 1 if on else 0))

    def set_wait_limit(self, polls: int, never_satisfied: bool = False):
        L.check(L.lib().oocs_batch_set_wait_limit(self._h, int(polls), 1 if never_satisfied else 0))

    def run_per_domain(self, steps: int, stream=None):
        L.check(L.lib().oocs_batch_run_per_domain(self._h, steps, _stream_ptr(stream)))

    def tile(self, i: int):
        """(tx, ty, zc, k) of domain i's configuration at the batch depth."""
        tx, ty, zc, k = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        L.check(L.lib().oocs_batch_domain_tile(self._h, i, C.byref(tx), C.byref(ty), C.byref(zc), C.byref(k)))
        return tx.value, ty.value, zc.value, k.value

    @property
    def depth(self) -> int:
        return self.tile(0)[3]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().oocs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _field_any(t: torch.Tensor):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 3:
        raise ValueError("domain fields must be contiguous float32 (nz, ny, nx) device tensors")
