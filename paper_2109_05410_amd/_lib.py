"""ctypes binding of liboocs (include/oocs.h): same names, argument
marshalling only. Every computation happens in the HIP library; if the
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liboocs.so")

OOCS_OK = 0
OOCS_E_ARG = -1
OOCS_E_ALIGN = -2
OOCS_E_HALO = -3
OOCS_E_CAP = -4
OOCS_E_RATE = -5
OOCS_E_SIZE = -6
OOCS_E_HIP = -7
OOCS_E_STATE = -8
OOCS_E_TIMEOUT = -9

OOCS_HEAT7 = 1
OOCS_WAVE25 = 2
OOCS_MAX_FIELDS = 3
OOCS_MAX_RATE = 34
OOCS_MAX_RATE64 = 68
OOCS_NOALLOC_MAX_CELLS = 1 << 24
OOCS_PLAN_BLOCK_RESTART = 1
OOCS_PLAN_KERNEL_TRANSFERS = 2
OOCS_PLAN_LEVEL_BY_LEVEL = 4
OOCS_PLAN_KERNEL_STORES = 8
OOCS_PLAN_RESIDENT_RO = 16
OOCS_PLAN_SNAKE = 32
OOCS_RETAIN_MAX = -1
OOCS_PLAN_MIDPOINT = 64
OOCS_PLAN_FP64 = 128
OOCS_PLAN_RO_DEVICE_STORE = 256
OOCS_DECODE_MIDPOINT = 0x100
OOCS_SCHED_MIRROR = 1
OOCS_SCHED_RETAIN_IN = 2
OOCS_SCHED_RETAIN_OUT = 4
OOCS_SLOT_RETAINED = -2
OOCS_SLOT_DEVICE_STORE = -3

OP_H2D, OP_DECODE, OP_LEVEL, OP_ENCODE, OP_D2H, OP_LAUNCH, OP_RECORD, OP_WAIT, OP_FETCH, OP_STORE = range(1, 11)


class OocsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liboocs error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("stencil", C.c_int32), ("nslabs", C.c_int32), ("k", C.c_int32), ("group", C.c_int32),
        ("rate", C.c_int32 * OOCS_MAX_FIELDS), ("nstage", C.c_int32),
        ("alpha", C.c_float), ("flags", C.c_int32),
        ("src_x", C.c_int64), ("src_y", C.c_int64), ("src_z", C.c_int64),
        ("retain", C.c_int32),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("group", C.c_int64), ("halo", C.c_int64), ("radius", C.c_int64), ("nlevels", C.c_int64),
        ("nrings", C.c_int64), ("ring_planes", C.c_int64 * 16), ("plane_bytes", C.c_int64),
        ("arena_needed", C.c_int64), ("nstage", C.c_int64), ("store_bytes", C.c_int64 * OOCS_MAX_FIELDS),
        ("retained_planes", C.c_int64),
    ]


class SlabInfo(C.Structure):
    _fields_ = [
        ("z0", C.c_int64), ("z1", C.c_int64), ("r0", C.c_int64), ("r1", C.c_int64),
        ("c0", C.c_int64), ("c1", C.c_int64),
        ("r_off", C.c_int64 * OOCS_MAX_FIELDS), ("r_bytes", C.c_int64 * OOCS_MAX_FIELDS),
        ("c_off", C.c_int64 * OOCS_MAX_FIELDS), ("c_bytes", C.c_int64 * OOCS_MAX_FIELDS),
    ]


class Op(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("stream", C.c_int32), ("field", C.c_int32), ("level", C.c_int32),
        ("slot", C.c_int32), ("block", C.c_int32), ("tick", C.c_int32), ("event", C.c_int32),
        ("z0", C.c_int64), ("z1", C.c_int64),
    ]


class AdjointCfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64), ("steps", C.c_int64), ("ckpt_every", C.c_int64),
        ("ckpt_rate", C.c_int32), ("nrcv", C.c_int32), ("src_x", C.c_int64), ("src_y", C.c_int64),
        ("src_z", C.c_int64), ("vscale", C.c_float), ("pad0", C.c_int32),
    ]


class Domain(C.Structure):
    _fields_ = [("d_u", C.c_void_p), ("d_scratch", C.c_void_p), ("nx", C.c_int64), ("ny", C.c_int64),
                ("nz", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [
        ("wall_ms", C.c_double), ("enqueue_ms", C.c_double), ("rounds", C.c_int64),
        ("h2d_bytes", C.c_int64), ("d2h_bytes", C.c_int64), ("cell_updates", C.c_int64),
        ("launches", C.c_int64), ("codec_bytes", C.c_int64), ("stencil_bytes", C.c_int64),
        ("kernel_ms", C.c_double), ("xfer_bytes", C.c_int64),
        ("timed_launches", C.c_int64), ("timed_bytes", C.c_int64), ("sdma_copies", C.c_int64),
        ("stage_ms", C.c_double * 5), ("arena_bytes", C.c_int64),
    ]


# name -> (restype, argtypes); this list is the binding of every symbol in include/oocs.h
_P = C.c_void_p
_I64 = C.c_int64
_SIGS = {
    "oocs_version": (C.c_int, []),
    "oocs_last_error": (C.c_char_p, []),
    "oocs_codec_bytes": (C.c_size_t, [_I64, _I64, _I64, C.c_int]),
    "oocs_codec_encode": (C.c_int, [_P, _I64, _I64, _I64, _I64, _I64, C.c_int, _P, C.c_size_t, _P]),
    "oocs_codec_decode": (C.c_int, [_P, C.c_size_t, _I64, _I64, _I64, C.c_int, _P, _I64, _I64, _P]),
    "oocs_codec_encode_stages": (C.c_int, [_P, _I64, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]),
    "oocs_codec_decode_stages": (C.c_int, [_P, _I64, C.c_int, _P, _P, _P, _P, _P, _P]),
    "oocs_heat7_step_k": (C.c_int, [_P, _P, _I64, _I64, _I64, C.c_float, _I64, _P]),
    "oocs_heat7_step_k_noalloc": (C.c_int, [_P, _I64, _I64, _I64, C.c_float, _I64, _P]),
    "oocs_wave25_step_k": (C.c_int, [_P, _P, _P, _I64, _I64, _I64, _I64, _P, _I64, _I64, _I64, _P]),
    "oocs_plan_create": (C.c_int, [C.POINTER(Config), _P, C.c_size_t, C.POINTER(_P)]),
    "oocs_plan_destroy": (C.c_int, [_P]),
    "oocs_plan_get_info": (C.c_int, [_P, C.POINTER(PlanInfo)]),
    "oocs_plan_slab": (C.c_int, [_P, C.c_int, C.POINTER(SlabInfo)]),
    "oocs_plan_schedule_len": (C.c_int64, [_P, C.c_int]),
    "oocs_plan_schedule_op": (C.c_int, [_P, C.c_int, _I64, C.POINTER(Op)]),
    "oocs_plan_schedule_variant_len": (C.c_int64, [_P, C.c_int, C.c_int]),
    "oocs_plan_schedule_variant_op": (C.c_int, [_P, C.c_int, C.c_int, _I64, C.POINTER(Op)]),
    "oocs_store_bytes": (C.c_size_t, [_P, C.c_int]),
    "oocs_store_put": (C.c_int, [_P, C.c_int, _P, _P]),
    "oocs_store_get": (C.c_int, [_P, C.c_int, _P, _P]),
    "oocs_run": (C.c_int, [_P, C.POINTER(_P), _I64, _P, C.POINTER(Stats)]),
    "oocs_plan_set_profiling": (C.c_int, [_P, C.c_int]),
    "oocs_plan_set_breakdown": (C.c_int, [_P, C.c_int]),
    "oocs_plan_set_graphs": (C.c_int, [_P, C.c_int]),
    "oocs_plan_set_host_waits": (C.c_int, [_P, C.c_int]),
    "oocs_plan_set_sdma": (C.c_int, [_P, C.c_int]),
    "oocs_plan_sdma_available": (C.c_int, [_P]),
    "oocs_link_probe": (C.c_int, [_P, _P, _P, _P, C.c_size_t, C.c_size_t, C.c_int, C.c_int,
                                  C.POINTER(C.c_double)]),
    "oocs_codec64_bytes": (C.c_size_t, [_I64, _I64, _I64, C.c_int]),
    "oocs_codec64_encode": (C.c_int, [_P, _I64, _I64, _I64, _I64, _I64, C.c_int, _P, C.c_size_t, _P]),
    "oocs_codec64_decode": (C.c_int, [_P, C.c_size_t, _I64, _I64, _I64, C.c_int, _P, _I64, _I64, _P]),
    "oocs_codec64_encode_stages": (C.c_int, [_P, _I64, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]),
    "oocs_codec64_decode_stages": (C.c_int, [_P, _I64, C.c_int, _P, _P, _P, _P, _P, _P]),
    "oocs_wave25_step_k_f64": (C.c_int, [_P, _P, _P, _I64, _I64, _I64, _I64, _P, _I64, _I64, _I64, _P]),
    "oocs_batch_table_bytes": (C.c_size_t, [C.c_int]),
    "oocs_batch_create": (C.c_int, [C.POINTER(Domain), C.c_int, C.c_float, _P, C.c_size_t, C.c_char_p, C.c_int,
                                    C.c_int, _P, C.POINTER(_P)]),
    "oocs_batch_run": (C.c_int, [_P, _I64, _P]),
    "oocs_batch_set_persistent": (C.c_int, [_P, C.c_int]),
    "oocs_batch_set_wait_limit": (C.c_int, [_P, _I64, C.c_int]),
    "oocs_batch_check": (C.c_int, [_P, _P]),
    "oocs_batch_run_per_domain": (C.c_int, [_P, _I64, _P]),
    "oocs_batch_domain_tile": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                         C.POINTER(C.c_int)]),
    "oocs_batch_destroy": (C.c_int, [_P]),
    "oocs_adjoint_workspace_bytes": (C.c_size_t, [C.POINTER(AdjointCfg)]),
    "oocs_adjoint_ckpt_bytes": (C.c_size_t, [C.POINTER(AdjointCfg)]),
    "oocs_wave_forward_ckpt": (C.c_int, [C.POINTER(AdjointCfg), _P, _P, _P, _P, _P, _P, C.c_size_t, _P,
                                         C.POINTER(C.c_double), _P]),
    "oocs_wave_adjoint": (C.c_int, [C.POINTER(AdjointCfg), _P, _P, _P, _P, _P, C.c_size_t, _P, _P, _P]),
}
SYMBOLS = tuple(_SIGS)

_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise OocsError(OOCS_E_STATE, f"{LIB_PATH} is not built; run paper_2109_05410_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(rc: int) -> int:
    if rc < 0:
        msg = lib().oocs_last_error()
        raise OocsError(rc, msg.decode() if msg else "")
    return rc
