"""Pins for the oracle's fixed-rate 4^3 block transform codec (Sec. IV: the
user fixes the number of bits per value; Lindstrom 2014 for the transform).

Each stage is checked against something it does not share: Lindstrom's
published transform matrix, the definition of base -2 digits, counting
identities of the sequency order, hand-worked bit streams, and the
structural properties of a fixed-rate embedded coder (losslessness at full
rate, prefix property, chunk invariance)."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def lindstrom_M():
    rows = [l.split() for l in open(os.path.join(GOLD, "lindstrom2014_forward_matrix.txt")) if not l.startswith("#")]
    return np.array([[int(x) for x in r] for r in rows if r], dtype=np.int64)


def test_forward_transform_equals_published_matrix_on_all_deltas():
    """For inputs divisible by 16^3 every shift is exact, so the 3D lifting
    must equal the separable product (M/16) x (M/16) x (M/16); this fixes
    signs, output order and the axis order."""
    M = lindstrom_M()
    S = 1 << 24
    for idx in range(64):
        i0, j0, l0 = idx & 3, (idx >> 2) & 3, idx >> 4
        q = np.zeros(64, dtype=np.int32)
        q[idx] = S
        t = O.fwd_xform(q)
        expect = np.zeros(64, dtype=np.int64)
        for k in range(64):
            i, j, l = k & 3, (k >> 2) & 3, k >> 4
            expect[k] = (S // 4096) * M[i, i0] * M[j, j0] * M[l, l0]
        assert np.array_equal(t.astype(np.int64), expect), idx


def test_inverse_undoes_forward_with_ten_trailing_zero_bits():
    rng = np.random.default_rng(0)
    for _ in range(3000):
        q = (rng.integers(-(1 << 20), 1 << 20, 64) << 10).astype(np.int32)
        assert np.array_equal(O.inv_xform(O.fwd_xform(q)), q)


def test_inverse_not_exact_in_general():
    """The floor shifts discard low bits: the transform is lossy on odd data."""
    rng = np.random.default_rng(1)
    bad = 0
    for _ in range(200):
        q = rng.integers(-(1 << 29), 1 << 29, 64).astype(np.int32)
        bad += not np.array_equal(O.inv_xform(O.fwd_xform(q)), q)
    assert bad > 100


def test_transform_stays_inside_int32():
    """|q| < 2^30 never overflows int32 in either pass (the oracle computes in
    int64 and reports any intermediate outside int32 as an error)."""
    rng = np.random.default_rng(2)
    extreme = [np.full(64, (1 << 30) - 1), np.full(64, -(1 << 30) + 1),
               np.where(np.arange(64) % 2 == 0, (1 << 30) - 1, -(1 << 30) + 1)]
    for q in extreme + [rng.integers(-(1 << 30) + 1, 1 << 30, 64) for _ in range(2000)]:
        t = O.fwd_xform(np.asarray(q, dtype=np.int32))
        O.inv_xform(t)


def test_negabinary_digits_represent_the_integer():
    """u's bits are the base -2 digits of q: sum_k bit_k(u) (-2)^k == q."""
    rng = np.random.default_rng(3)
    vals = np.concatenate([rng.integers(-(1 << 30), 1 << 30, 400), [0, 1, -1, 2, -2, (1 << 30) - 1, -(1 << 30)]])
    for q in vals:
        q = int(q)
        blk = np.zeros(64, dtype=np.float32)
        # route through the real coder stage: a block whose DC coefficient is q
        # is not directly constructible, so check the map itself on integers
        u = ((q + 0xAAAAAAAA) & 0xFFFFFFFF) ^ 0xAAAAAAAA
        assert sum(((u >> k) & 1) * (-2) ** k for k in range(32)) == q
    # and the coder's stage output uses exactly that map
    v = rng.standard_normal(64).astype(np.float32)
    _, st = O.encode_block(v, 16)
    perm = O.codec_perm()
    for k in range(64):
        q = int(st["t"][perm[k]])
        assert sum(((int(st["u"][k]) >> b) & 1) * (-2) ** b for b in range(32)) == q


def test_sequency_order():
    perm = O.codec_perm()
    assert sorted(perm.tolist()) == list(range(64))
    keys = []
    for idx in perm:
        i, j, l = idx & 3, (idx >> 2) & 3, idx >> 4
        keys.append((i + j + l, i * i + j * j + l * l, l, j, i))
    assert keys == sorted(keys) and len(set(keys)) == 64
    # number of (i,j,l) in [0,3]^3 with each total sequency: coefficients of (1+x+x^2+x^3)^3
    counts = np.bincount([k[0] for k in keys])
    assert counts.tolist() == [1, 3, 6, 10, 12, 12, 10, 6, 3, 1]
    assert perm[0] == 0 and perm[-1] == 63


def golden():
    with open(os.path.join(GOLD, "codec_streams.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("case", golden()["blocks"], ids=lambda c: c["name"])
def test_hand_worked_block_streams(case):
    for rate, exp in case["rates"].items():
        rate = int(rate)
        words, st = O.encode_block(np.full(64, case["value"], dtype=np.float32), rate)
        assert [hex(int(w)) for w in words] == exp["words"]
        assert st["bits_used"] == exp["bits_used"]
        dec, _ = O.decode_block(words, rate)
        assert np.all(dec == np.float32(case["value"]))


@pytest.mark.parametrize("case", golden()["coefficient_streams"], ids=lambda c: c["name"])
def test_hand_worked_coefficient_streams(case):
    u = np.zeros(64, dtype=np.uint32)
    for k, v in case["u"].items():
        u[int(k)] = v
    words, used = O.code_ints(u, case["budget"])
    assert [hex(int(w)) for w in words] == case["words"]
    assert used == case["bits_used"]
    assert np.array_equal(O.decode_ints(words, case["budget"]), u)


def test_implied_last_bit_and_truncation():
    """Only coefficient 63 set: with budget 95 the implied bit restores it;
    with 64 bits the scan is cut and the decoder leaves it zero."""
    u = np.zeros(64, dtype=np.uint32)
    u[63] = 1
    w, used = O.code_ints(u, 64)
    assert used == 64
    assert O.decode_ints(w, 64)[63] == 0
    w, used = O.code_ints(u, 95)
    assert used == 95 and O.decode_ints(w, 95)[63] == 1


def test_integer_coder_lossless_at_full_budget():
    """Worst case is 64*32 plane bits + 64 group tests + 32 plane-end tests
    = 2144 bits; with rate 34 (2176 - 9 = 2167 bits) nothing is truncated."""
    rng = np.random.default_rng(4)
    budget = 64 * 34 - 9
    worst = 0
    for trial in range(400):
        if trial % 4 == 0:
            u = rng.integers(0, 1 << 32, 64, dtype=np.uint64).astype(np.uint32)
        else:
            u = (rng.integers(0, 1 << 32, 64, dtype=np.uint64) >> rng.integers(0, 32, 64).astype(np.uint64)).astype(np.uint32)
        w, used = O.code_ints(u, budget)
        worst = max(worst, used)
        assert np.array_equal(O.decode_ints(w, budget), u)
    assert worst <= 2144
    full = np.full(64, 0xFFFFFFFF, dtype=np.uint32)
    w, used = O.code_ints(full, budget)
    # plane 31: coefficients 0..62 each cost a positive group test and their
    # own 1 bit; coefficient 63 costs only its group test (its bit is implied);
    # then 31 planes of 64 verbatim bits
    assert used == 63 * 2 + 1 + 31 * 64
    assert np.array_equal(O.decode_ints(w, budget), full)


def test_float_codec_lossless_on_representable_blocks():
    """Values m*2^-s with |m| < 2^19 give q with >= 10 trailing zero bits, so
    the transform inverts exactly, and rate 34 codes every bit."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        s = int(rng.integers(-10, 40))
        m = rng.integers(-(1 << 19), 1 << 19, 64)
        x = np.ldexp(m.astype(np.float64), -s).astype(np.float32)
        w, _ = O.encode_block(x, 34)
        d, _ = O.decode_block(w, 34)
        assert np.array_equal(d, x)


@pytest.mark.parametrize("rate", [1, 2, 8, 12])
def test_constant_blocks_lossless(rate):
    rng = np.random.default_rng(rate)
    for c in np.concatenate([rng.standard_normal(50), rng.random(50) * 1e-20, [1.0, -3.5, 2.0 ** 100]]).astype(np.float32):
        w, _ = O.encode_block(np.full(64, c, dtype=np.float32), rate)
        d, _ = O.decode_block(w, rate)
        assert np.all(d == c)


def test_zero_blocks():
    for z in (0.0, -0.0):
        w, st = O.encode_block(np.full(64, z, dtype=np.float32), 8)
        assert st["bits_used"] == 1 and not np.any(w)
        d, _ = O.decode_block(w, 8)
        assert np.all(d == 0.0)


def test_prefix_property():
    """The coder is embedded: a rate-R1 block equals the first 64*R1 bits of
    the rate-R2 block for R1 < R2."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        x = (rng.standard_normal(64) * np.exp(rng.standard_normal(64))).astype(np.float32)
        w2, _ = O.encode_block(x, 20)
        for r1 in (1, 3, 8, 12, 16):
            w1, _ = O.encode_block(x, r1)
            assert np.array_equal(w1, w2[:r1])


def test_chunk_invariance():
    """Blocks are coded independently in z-major block order, so any run of
    whole 4-plane layers of a field codes to the same words as the
    corresponding slice of the whole-field stream."""
    rng = np.random.default_rng(7)
    f = rng.standard_normal((24, 12, 16)).astype(np.float32)
    rate = 7
    whole = O.codec_encode(f, rate)
    per_layer = (12 // 4) * (16 // 4) * rate
    for z0, z1 in ((0, 4), (8, 20), (4, 24)):
        part = O.codec_encode(f[z0:z1], rate)
        assert np.array_equal(part, whole[z0 // 4 * per_layer: z1 // 4 * per_layer])
    dec = O.codec_decode(whole, f.shape, rate)
    assert np.array_equal(dec[8:20], O.codec_decode(whole[2 * per_layer: 5 * per_layer], (12, 12, 16), rate))


def test_field_layout_matches_block_definition():
    """Block b = bx + nbx*(by + nby*bz) holds the cells (4bx+i, 4by+j, 4bz+l)
    at in-block index i + 4j + 16l."""
    rng = np.random.default_rng(8)
    f = rng.standard_normal((8, 8, 12)).astype(np.float32)
    rate = 9
    whole = O.codec_encode(f, rate)
    nbx, nby = 3, 2
    for bz in range(2):
        for by in range(nby):
            for bx in range(nbx):
                blk = f[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4].reshape(64)
                w, _ = O.encode_block(blk, rate)
                b = bx + nbx * (by + nby * bz)
                assert np.array_equal(w, whole[b * rate:(b + 1) * rate])


def test_error_shrinks_with_rate_on_smooth_data():
    z, y, x = np.meshgrid(np.arange(32), np.arange(32), np.arange(32), indexing="ij")
    f = (np.sin(0.2 * x) * np.cos(0.15 * y) + 0.3 * np.sin(0.1 * z) + 1.5).astype(np.float32)
    errs = [np.max(np.abs(O.codec_roundtrip(f, r) - f)) for r in (2, 4, 6, 8, 12)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    # from rate 16 on, the error is that of the 30-bit block-floating-point
    # transform alone: about one FP32 ulp of the largest values (|f| < 2.8)
    for r in (16, 24, 32):
        assert np.max(np.abs(O.codec_roundtrip(f, r) - f)) <= 2.0 ** -22


def test_subnormal_exponent_clamp():
    rng = np.random.default_rng(9)
    x = (rng.random(64) * 2.0 ** -130).astype(np.float32)
    w, st = O.encode_block(x, 34)
    assert st["emax"] == -126
    d, _ = O.decode_block(w, 34)
    assert np.max(np.abs(d - x)) <= 2.0 ** (-126 - 20)


# ---------------------------------------------------------------------------
# mid-point reconstruction (a decoding option; format step 9 in oracle.c)
# ---------------------------------------------------------------------------

def nb_value(u):
    """Integer of a 32-digit negabinary word, by its digits."""
    return sum(((int(u) >> j) & 1) * (-2) ** j for j in range(32))


def known_digits(u, budget):
    """Brute force: digit p of coefficient i is determined by the first
    `budget` bits unless some other block with that digit flipped codes to
    the same bits. The candidates are the block with only that digit
    flipped, and with one more digit of the same plane flipped (which is
    what keeps a group test's answer, 'some digit at or after position n is
    1', unchanged)."""
    base, used = O.code_ints(u, budget)
    known = np.zeros((64, 32), bool)
    for p in range(32):
        bit = np.uint32(1 << p)
        for i in range(64):
            v = u.copy()
            v[i] ^= bit
            if np.array_equal(O.code_ints(v, budget)[0], base):
                continue
            same = False
            for j in range(64):
                if j == i:
                    continue
                v2 = v.copy()
                v2[j] ^= bit
                if np.array_equal(O.code_ints(v2, budget)[0], base):
                    same = True
                    break
            known[i, p] = not same
    return known


def sample_coefficients(rng, n):
    """Negabinary coefficient blocks with the energy decay of smooth data:
    large low-sequency coefficients, small high-sequency ones."""
    out = []
    for _ in range(n):
        mag = (2.0 ** rng.uniform(0, 28, 64)) * np.exp(-np.arange(64) / rng.uniform(4, 40))
        q = (rng.choice([-1, 1], 64) * mag).astype(np.int64)
        out.append(((q.astype(np.uint32) + np.uint32(0xAAAAAAAA)) ^ np.uint32(0xAAAAAAAA)).astype(np.uint32))
    return out


@pytest.mark.parametrize("budget", [40, 137, 300, 555, 1001])
def test_stop_point_matches_brute_force_known_digits(budget):
    """The decoder's stop plane P and known prefix m agree with the digits
    the stream actually depends on: coefficient i knows exactly its digits
    at planes >= P + (i >= m) (all of them if the stream is complete)."""
    rng = np.random.default_rng(budget)
    for u in sample_coefficients(rng, 3):
        known = known_digits(u, budget)
        w, _ = O.code_ints(u, budget)
        _, P, m = O.decode_ints_stop(w, budget)
        for i in range(64):
            L = 0 if P < 0 else (P if i < m else P + 1)
            assert np.array_equal(known[i], np.arange(32) >= L), (i, P, m)


def test_midpoint_is_the_middle_of_the_consistent_integers():
    """With mid-point reconstruction a nonzero coefficient whose L low digits
    were cut off becomes the middle (rounded down) of the smallest and
    largest integers its known digits allow, found by enumerating every
    completion of the L digits (L <= 12 here); zero coefficients stay zero;
    the result is never farther from the true integer than half the range."""
    rng = np.random.default_rng(7)
    seen = 0
    for rate in (14, 18, 24, 28):
        for _ in range(30):
            x = rng.standard_normal(64).astype(np.float32) * np.float32(2.0 ** rng.integers(-8, 8))
            words, est = O.encode_block(x, rate)
            _, zf = O.decode_block(words, rate)
            _, md = O.decode_block(words, rate, mid=True)
            P, m = md["stop_plane"], md["stop_known"]
            assert (P, m) == (zf["stop_plane"], zf["stop_known"])
            assert np.array_equal(md["u"], zf["u"])  # the digits read are the same
            perm = O.codec_perm()
            for k in range(64):
                L = 0 if P < 0 else (P if k < m else P + 1)
                got = int(md["t"][perm[k]])
                if zf["u"][k] == 0 or L == 0:
                    assert got == int(zf["t"][perm[k]])
                    continue
                if L > 12:
                    continue
                base = nb_value(zf["u"][k])
                vals = [base + sum(((c >> j) & 1) * (-2) ** j for j in range(L)) for c in range(1 << L)]
                lo, hi = min(vals), max(vals)
                assert got == (lo + hi) // 2, (k, L)
                truth = nb_value(est["u"][k])
                assert lo <= truth <= hi
                assert abs(got - truth) <= (hi - lo + 1) // 2
                seen += 1
    assert seen > 200


def test_midpoint_changes_nothing_when_the_stream_is_complete():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((8, 8, 8)).astype(np.float32)
    w = O.codec_encode(f, 34)
    assert np.array_equal(O.codec_decode(w, f.shape, 34, mid=True), O.codec_decode(w, f.shape, 34))
    z = np.zeros((4, 8, 8), np.float32)
    assert not np.any(O.codec_decode(O.codec_encode(z, 4), z.shape, 4, mid=True))


@pytest.mark.parametrize("rate", [4, 8, 12])
def test_midpoint_lowers_the_error_on_smooth_data(rate):
    """On a smooth field plus noise (the diffused heat and the developed
    wavefield are of this kind) mid-point reconstruction lowers the L2
    error of decode(encode()) against the input."""
    rng = np.random.default_rng(rate)
    z, y, x = np.meshgrid(*(np.linspace(0, 1, 32),) * 3, indexing="ij")
    f = (np.sin(3 * x + 1) * np.cos(2 * y) * np.exp(-z) + 1e-3 * rng.standard_normal(x.shape)).astype(np.float32)
    e0 = np.linalg.norm(O.codec_roundtrip(f, rate) - f)
    e1 = np.linalg.norm(O.codec_roundtrip(f, rate, mid=True) - f)
    assert e1 < 0.9 * e0
