"""The C ABI library loads without a GPU and exports every function that
include/oocs.h declares; the Python binding covers exactly that set."""
import ctypes
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2109_05410_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oocs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oocs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("oocs_plan_create", "oocs_codec_encode", "oocs_codec_decode", "oocs_heat7_step_k",
                     "oocs_wave25_step_k", "oocs_run", "oocs_store_put", "oocs_store_get"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (oocs_[a-z0-9_]+)", out))
    assert set(declared_functions()) == exported


def test_binding_matches_header():
    assert set(L.SYMBOLS) == set(declared_functions())


def test_calls_without_gpu_work():
    lib = L.lib()
    assert lib.oocs_version() >= 1
    assert lib.oocs_codec_bytes(512, 512, 512, 8) == 512 ** 3 // 64 * 8 * 8
    assert lib.oocs_codec_bytes(510, 512, 512, 8) == 0
    assert lib.oocs_codec_bytes(512, 512, 512, 35) == 0
    # argument errors are reported before anything touches a device
    rc = lib.oocs_codec_encode(None, 8, 8, 8, 8, 64, 8, None, 0, None)
    assert rc == L.OOCS_E_ARG
    assert b"null" in lib.oocs_last_error()
    with pytest.raises(L.OocsError):
        L.check(rc)


def test_transfer_entry_points_check_arguments_without_gpu():
    """The SDMA switch, its availability query and the host-link probe
    reject null handles and buffers before touching a device."""
    lib = L.lib()
    assert lib.oocs_plan_set_sdma(None, 1) == L.OOCS_E_ARG
    assert lib.oocs_plan_sdma_available(None) == 0
    out = (ctypes.c_double * 4)()
    assert lib.oocs_link_probe(None, None, None, None, 1 << 20, 1 << 20, 1, 1, out) == L.OOCS_E_ARG
    assert lib.oocs_link_probe(1, 1, 1, 1, 0, 1 << 20, 1, 1, out) == L.OOCS_E_ARG      # zero bytes
    assert lib.oocs_link_probe(1, 1, 1, 1, 1 << 20, 0, 1, 1, out) == L.OOCS_E_ARG      # zero chunk
    assert lib.oocs_link_probe(1, 1, 1, 1, 1 << 20, 1 << 20, 0, 1, out) == L.OOCS_E_ARG  # no timed pass


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits with a message
    before anything is imported or launched."""
    r = subprocess.run(["python3", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_no_alloc_size_limit_is_checked_before_any_device_call():
    """Fields beyond the library-held scratch are refused up front (no HIP
    call is made, so this runs without a GPU)."""
    lib = L.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: the size check comes first
    n = L.OOCS_NOALLOC_MAX_CELLS
    assert lib.oocs_heat7_step_k_noalloc(fake, 4096, 4096, n // (4096 * 4096) + 1, C.c_float(0.1), 1, None) == L.OOCS_E_SIZE
    assert lib.oocs_heat7_step_k_noalloc(None, 4, 4, 4, C.c_float(0.1), 1, None) == L.OOCS_E_ARG
