"""GPU codec parity: every stage of the HIP encoder and decoder (block
exponent, block-floating-point integers, transform, sequency order +
negabinary, bit planes, coded words) must equal the oracle's bit for bit;
the whole-field calls must produce the oracle's streams and values."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2109_05410_amd import api

pytestmark = pytest.mark.gpu
DEV = "cuda"
RATES = [1, 2, 3, 8, 12, 16, 24, 34]


def block_zoo(n_random=600, seed=0):
    rng = np.random.default_rng(seed)
    blocks = [
        np.zeros(64), np.full(64, -0.0), np.full(64, 0.75), np.full(64, -3.25),
        np.eye(64)[0], np.eye(64)[63] * -1e-3, np.eye(64)[21] * 7.0,
        np.full(64, 3.0e38), np.full(64, 1e-40), rng.random(64) * 1e-39,      # huge, subnormal
        np.concatenate([rng.standard_normal(32) * 1e30, rng.standard_normal(32) * 1e-30]),
        np.where(np.arange(64) % 2 == 0, 1.0, -1.0),
        np.arange(64, dtype=np.float64) - 31.5,
    ]
    for _ in range(n_random):
        kind = rng.integers(0, 4)
        if kind == 0:
            b = rng.random(64)
        elif kind == 1:
            b = rng.standard_normal(64) * np.exp(3 * rng.standard_normal(64))
        elif kind == 2:
            x, y, z = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
            b = (np.sin(0.3 * x + rng.random()) * np.cos(0.2 * y) + 0.1 * z).transpose(2, 1, 0).ravel() * rng.random()
        else:
            b = np.where(rng.random(64) < 0.8, 0.0, rng.standard_normal(64))
        blocks.append(b)
    return np.stack(blocks).astype(np.float32)


@pytest.mark.parametrize("rate", RATES)
def test_encode_stages_bit_exact(rate):
    blocks = block_zoo(seed=rate)
    st = api.codec_encode_stages(torch.from_numpy(blocks).to(DEV), rate)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in st.items()}
    for b in range(blocks.shape[0]):
        words, o = O.encode_block(blocks[b], rate)
        assert g["emax"][b] == o["emax"], b
        if o["emax"] != O.EMAX_ZERO:
            assert np.array_equal(g["q"][b], o["q"]), b
            assert np.array_equal(g["t"][b], o["t"]), b
            assert np.array_equal(g["u"][b].view(np.uint32), o["u"]), b
            assert np.array_equal(g["plane"][b].view(np.uint64), o["plane"]), b
        assert g["bits_used"][b] == o["bits_used"], b
        assert np.array_equal(g["words"][b].view(np.uint64), words), b


@pytest.mark.parametrize("rate", RATES)
def test_decode_stages_bit_exact(rate):
    blocks = block_zoo(seed=100 + rate)
    words = np.stack([O.encode_block(b, rate)[0] for b in blocks])
    st = api.codec_decode_stages(torch.from_numpy(words.view(np.int64)).to(DEV), rate)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in st.items()}
    for b in range(blocks.shape[0]):
        vals, o = O.decode_block(words[b], rate)
        assert g["emax"][b] == o["emax"], b
        assert np.array_equal(g["plane"][b].view(np.uint64), o["plane"]), b
        assert np.array_equal(g["u"][b].view(np.uint32), o["u"]), b
        if o["emax"] != O.EMAX_ZERO:
            assert np.array_equal(g["q"][b], o["q"]), b
        assert np.array_equal(g["out"][b].view(np.uint32), vals.view(np.uint32)), b


@pytest.mark.parametrize("shape", [(20, 36, 68), (4, 4, 4), (8, 12, 260)])
@pytest.mark.parametrize("rate", [1, 8, 16, 34])
def test_field_codec_matches_oracle(shape, rate):
    """Several workgroups, a ragged last group of x-blocks, several layers."""
    f = np.random.default_rng(rate).standard_normal(shape).astype(np.float32)
    d = torch.from_numpy(f).to(DEV)
    words = api.codec_encode(d, rate)
    torch.cuda.synchronize()
    want = O.codec_encode(f, rate)
    assert np.array_equal(words.cpu().numpy().view(np.uint64), want)
    dec = api.codec_decode(torch.from_numpy(want.view(np.int64)).to(DEV), shape, rate)
    torch.cuda.synchronize()
    assert np.array_equal(dec.cpu().numpy().view(np.uint32), O.codec_decode(want, shape, rate).view(np.uint32))


def test_strided_field():
    from paper_2109_05410_amd import _lib as L
    import ctypes as C
    nz, ny, nx, rate = 8, 12, 16, 9
    ld_y, ld_z = nx + 8, (nx + 8) * ny + 16
    big = torch.randn(nz * ld_z, device=DEV)
    dense = torch.empty((nz, ny, nx), device=DEV)
    for z in range(nz):
        for y in range(ny):
            dense[z, y] = big[z * ld_z + y * ld_y: z * ld_z + y * ld_y + nx]
    out = torch.empty(api.codec_bytes(nx, ny, nz, rate) // 8, dtype=torch.int64, device=DEV)
    L.check(L.lib().oocs_codec_encode(C.c_void_p(big.data_ptr()), nx, ny, nz, ld_y, ld_z, rate,
                                      C.c_void_p(out.data_ptr()), out.numel() * 8,
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    ref = api.codec_encode(dense.contiguous(), rate)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_garbage_stream_decodes_in_bounds():
    """Any bit pattern decodes: each block reads only its own rate words."""
    rate = 8
    rng = np.random.default_rng(5)
    w = torch.from_numpy(rng.integers(-2**62, 2**62, 16 * 16 * 16 // 64 * rate, dtype=np.int64)).to(DEV)
    out = api.codec_decode(w, (16, 16, 16), rate)
    torch.cuda.synchronize()
    assert out.shape == (16, 16, 16)


def test_argument_errors():
    from paper_2109_05410_amd import _lib as L
    d = torch.zeros((8, 8, 8), device=DEV)
    with pytest.raises(L.OocsError) as e:
        api.codec_encode(d, 0)
    assert e.value.code == L.OOCS_E_RATE
    small = torch.zeros(3, dtype=torch.int64, device=DEV)
    with pytest.raises(L.OocsError) as e:
        api.codec_encode(d, 8, out=small)
    assert e.value.code == L.OOCS_E_SIZE


def test_full_size_sampled_blocks():
    """512^3 field at rate 8 (the benchmark's size): sampled blocks of the
    GPU stream equal the oracle's encoding of the same blocks."""
    shape = (512, 512, 512)
    from paper_2109_05410_amd import inputs
    f = inputs.heat_uniform(shape, seed=0)
    d = torch.from_numpy(f).to(DEV)
    rate = 8
    words = api.codec_encode(d, rate).cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(1)
    nb = 128
    for b in np.concatenate([[0, nb ** 3 - 1], rng.integers(0, nb ** 3, 300)]):
        bx, by, bz = b % nb, (b // nb) % nb, b // (nb * nb)
        blk = f[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4].reshape(64)
        want, _ = O.encode_block(blk, rate)
        assert np.array_equal(words[b * rate:(b + 1) * rate], want), b


@pytest.mark.parametrize("rate", RATES)
def test_midpoint_decode_stages_bit_exact(rate):
    """Mid-point reconstruction: the digits read are the same, and the
    integers after the inverse transform and the values equal the oracle's
    bit for bit (the stop plane and known prefix decide every offset)."""
    blocks = block_zoo(seed=200 + rate)
    words = np.stack([O.encode_block(b, rate)[0] for b in blocks])
    st = api.codec_decode_stages(torch.from_numpy(words.view(np.int64)).to(DEV), rate, mid=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in st.items()}
    changed = 0
    for b in range(blocks.shape[0]):
        vals, o = O.decode_block(words[b], rate, mid=True)
        zf, _ = O.decode_block(words[b], rate)
        assert np.array_equal(g["u"][b].view(np.uint32), o["u"]), b
        if o["emax"] != O.EMAX_ZERO:
            assert np.array_equal(g["q"][b], o["q"]), b
        assert np.array_equal(g["out"][b].view(np.uint32), vals.view(np.uint32)), b
        changed += int(not np.array_equal(vals, zf))
    if rate < 34:
        assert changed > 0


@pytest.mark.parametrize("shape", [(20, 36, 68), (8, 12, 260)])
@pytest.mark.parametrize("rate", [1, 8, 12, 16])
def test_midpoint_field_decode_matches_oracle(shape, rate):
    f = np.random.default_rng(rate + 7).standard_normal(shape).astype(np.float32)
    want_w = O.codec_encode(f, rate)
    dec = api.codec_decode(torch.from_numpy(want_w.view(np.int64)).to(DEV), shape, rate, mid=True)
    torch.cuda.synchronize()
    assert np.array_equal(dec.cpu().numpy().view(np.uint32),
                          O.codec_decode(want_w, shape, rate, mid=True).view(np.uint32))
