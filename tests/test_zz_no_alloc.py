"""The allocation-free in-core heat step (library-held scratch) against the
entry point with a caller scratch buffer: same bits, on two calls in a row
(the second on a smaller field, so the shared scratch still holds the first
call's data), through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2109_05410_amd import _lib as L
from paper_2109_05410_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _with_scratch(u0, k):
    u = torch.from_numpy(u0).to(DEV)
    tmp = torch.empty_like(u)
    nz, ny, nx = u.shape
    stream = torch.cuda.current_stream().cuda_stream
    L.check(L.lib().oocs_heat7_step_k(C.c_void_p(u.data_ptr()), C.c_void_p(tmp.data_ptr()), nx, ny, nz,
                                      C.c_float(0.1), k, C.c_void_p(stream)))
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _no_alloc(u0, k):
    u = torch.from_numpy(u0).to(DEV)
    nz, ny, nx = u.shape
    stream = torch.cuda.current_stream().cuda_stream
    L.check(L.lib().oocs_heat7_step_k_noalloc(C.c_void_p(u.data_ptr()), nx, ny, nz, C.c_float(0.1), k,
                                              C.c_void_p(stream)))
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_no_alloc_matches_scratch_entry_point_twice():
    # first call: a field over 2^21 cells (the level job, one step per
    # launch); second: a small field (short-chunk launches) that reuses the
    # start of the scratch the first call left written
    cases = [((96, 256, 248), 7, 1), ((64, 64, 64), 10, 2)]
    assert 96 * 256 * 248 <= L.OOCS_NOALLOC_MAX_CELLS
    for shape, k, seed in cases:
        u0 = inputs.heat_uniform(shape, seed=seed)
        want = _with_scratch(u0, k)
        got = _no_alloc(u0, k)
        assert np.array_equal(got, want), shape


def test_no_alloc_refuses_oversized_fields():
    u = torch.zeros(4, device=DEV)
    rc = L.lib().oocs_heat7_step_k_noalloc(C.c_void_p(u.data_ptr()), 4096, 4096, 2, C.c_float(0.1), 1, None)
    assert rc == L.OOCS_E_SIZE
    assert b"scratch" in L.lib().oocs_last_error()
