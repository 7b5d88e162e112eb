"""Pins for the oracle's FP64 format (the paper's precision, Sec. VI; the
same fixed-rate method as the FP32 format with 64-bit integers, a 12-bit
header and 64 bit planes).

Checked against: Lindstrom's published forward matrix (exact on inputs
divisible by 16^3), inverse exactness with ten trailing zero bits, the
int64 range, the coder on integers whose high 32 planes are empty (which
must be 32 negative group tests followed by the FP32 coder's stream, itself
pinned by hand-worked streams), losslessness at full rate, zero and constant
blocks, the prefix property, chunk invariance, and error falling with rate."""
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lindstrom_M():
    rows = [l.split() for l in open(os.path.join(GOLD, "lindstrom2014_forward_matrix.txt")) if not l.startswith("#")]
    return np.array([[int(x) for x in r] for r in rows if r], dtype=np.int64)


def test_forward_transform_equals_published_matrix_on_all_deltas():
    M = lindstrom_M()
    S = 1 << 52
    for idx in range(64):
        i0, j0, l0 = idx & 3, (idx >> 2) & 3, idx >> 4
        q = np.zeros(64, dtype=np.int64)
        q[idx] = S
        t = O.fwd_xform64(q)
        expect = np.array([(S // 4096) * M[k & 3, i0] * M[(k >> 2) & 3, j0] * M[k >> 4, l0] for k in range(64)],
                          dtype=np.int64)
        assert np.array_equal(t, expect), idx


def test_inverse_undoes_forward_with_ten_trailing_zero_bits():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        q = rng.integers(-(1 << 52), 1 << 52, 64, dtype=np.int64) << 10
        assert np.array_equal(O.inv_xform64(O.fwd_xform64(q)), q)


def test_transform_stays_inside_int64():
    """|q| < 2^62 (the float cast's bound): no intermediate of either pass
    leaves int64 (the oracle checks with 128-bit arithmetic and reports)."""
    rng = np.random.default_rng(1)
    lim = (1 << 62) - 1
    for _ in range(2000):
        kind = rng.integers(0, 3)
        if kind == 0:
            q = rng.integers(-lim, lim, 64, dtype=np.int64)
        elif kind == 1:
            q = np.where(rng.random(64) < 0.5, lim, -lim).astype(np.int64)
        else:
            q = np.full(64, lim if rng.random() < 0.5 else -lim, dtype=np.int64)
        O.inv_xform64(O.fwd_xform64(q))


def test_coder_on_32_bit_integers_is_the_fp32_coder_after_32_empty_planes():
    """For coefficients whose digits above plane 31 are zero, planes 63..32
    each cost one negative group test (a 0 bit), and planes 31..0 are coded
    exactly as by the FP32 coder."""
    rng = np.random.default_rng(2)
    for budget in (40, 200, 777, 2100):
        for _ in range(30):
            u32 = rng.integers(0, 1 << 32, 64, dtype=np.uint64).astype(np.uint32)
            u32[rng.random(64) < 0.3] = 0
            w64, used64 = O.code_ints64(u32.astype(np.uint64), budget + 32)
            w32, used32 = O.code_ints(u32, budget)
            bits64 = np.unpackbits(w64.view(np.uint8), bitorder="little")[:budget + 32]
            bits32 = np.unpackbits(w32.view(np.uint8), bitorder="little")[:budget]
            assert not bits64[:32].any()
            assert np.array_equal(bits64[32:], bits32)
            assert used64 == used32 + 32


def test_integer_coder_lossless_at_full_budget():
    rng = np.random.default_rng(3)
    for _ in range(300):
        u = rng.integers(0, np.iinfo(np.uint64).max, 64, dtype=np.uint64, endpoint=True)
        u[rng.random(64) < 0.2] = 0
        budget = 64 * O.MAX_RATE64 - 12
        w, used = O.code_ints64(u, budget)
        assert used <= 12 + 64 * 64 + 64 + 64
        assert np.array_equal(O.decode_ints64(w, budget), u)


def test_float_codec_lossless_on_representable_blocks():
    """Values that are integers times 2^(emax - 52) keep their ten trailing
    zero bits through the cast, so at full rate the codec is exact."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        s = int(rng.integers(-60, 60))
        x = rng.integers(-(1 << 51), 1 << 51, 64).astype(np.float64) * 2.0 ** s
        words, _ = O.encode_block64(x, O.MAX_RATE64)
        y, _ = O.decode_block64(words, O.MAX_RATE64)
        assert np.array_equal(y, x)


def test_zero_and_constant_blocks():
    w, st = O.encode_block64(np.zeros(64), 4)
    assert st["bits_used"] == 1 and not w.any()
    y, _ = O.decode_block64(w, 4)
    assert not y.any()
    for c in (0.75, -3.25, 1e-300, 6.0e307, 1234.5):
        for rate in (3, 8, 24):
            w, _ = O.encode_block64(np.full(64, c), rate)
            y, _ = O.decode_block64(w, rate)
            assert np.all(y == c), (c, rate)


def test_prefix_property():
    rng = np.random.default_rng(5)
    for _ in range(100):
        x = rng.standard_normal(64) * np.exp(3 * rng.standard_normal(64))
        w_hi, _ = O.encode_block64(x, 40)
        for r in (1, 7, 24, 32):
            w_lo, _ = O.encode_block64(x, r)
            assert np.array_equal(w_lo, w_hi[:r])


def test_chunk_invariance_and_layout():
    rng = np.random.default_rng(6)
    f = rng.standard_normal((24, 12, 16))
    w = O.codec64_encode(f, 24)
    per_layer = (12 // 4) * (16 // 4) * 24
    for z0, z1 in ((0, 8), (8, 20), (20, 24)):
        assert np.array_equal(O.codec64_encode(f[z0:z1], 24), w[z0 // 4 * per_layer: z1 // 4 * per_layer])
    b = 1 + 4 * (2 + 3 * 1)  # block (x=1, y=2, z=1)
    blk = f[4:8, 8:12, 4:8].reshape(-1)  # (l, j, i) -> i + 4j + 16l
    want, _ = O.encode_block64(blk, 24)
    assert np.array_equal(w[b * 24:(b + 1) * 24], want)


def test_error_falls_with_rate():
    rng = np.random.default_rng(7)
    z, y, x = np.meshgrid(*(np.linspace(0, 1, 16),) * 3, indexing="ij")
    f = np.sin(3 * x + 1) * np.cos(2 * y) * np.exp(-z) + 1e-6 * rng.standard_normal(x.shape)
    errs = [np.abs(O.codec64_roundtrip(f, r) - f).max() for r in (8, 16, 24, 32, 48)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-12 * np.abs(f).max()
