"""Pins for the oracle's replay of the compressed out-of-core schedule
(Sec. III halo + region sharing; Sec. V-A separate compression).

The replay claims: (1) decomposing z into blocks with halo h = r*k and
advancing each extended block k steps reproduces the plain stencil exactly;
(2) with compression, the host store after each residency is encode(F_k(
decode(store))), chunk by chunk (remainder R_i and common region C_i coded
separately). Both are checked here by simulating the block schedule
explicitly on the CPU, chunk by chunk, with the oracle's own stencil and
codec primitives."""
import numpy as np
import pytest

import oracle as O


def slab_bounds(nz, n):
    return [i * nz // n for i in range(n + 1)]


def chunks(nz, n, h):
    """Remainders R_i and common regions C_i as (kind, i, z0, z1), in z order."""
    a = slab_bounds(nz, n)
    out = []
    for i in range(n):
        r0 = 0 if i == 0 else a[i] + h
        r1 = nz if i == n - 1 else a[i + 1] - h
        out.append(("R", i, r0, r1))
        if i < n - 1:
            out.append(("C", i, a[i + 1] - h, a[i + 1] + h))
    return out


def test_chunks_partition_the_axis():
    for nz, n, h in ((512, 8, 4), (1024, 8, 48), (64, 4, 4)):
        cs = chunks(nz, n, h)
        assert cs[0][2] == 0 and cs[-1][3] == nz
        for (_, _, _, e), (_, _, s, _) in zip(cs, cs[1:]):
            assert e == s
        assert all(c[3] > c[2] for c in cs)


def advance_block_heat(u, z0, z1, h, steps, nz, fn):
    """Advance the extended block [z0-h, z1+h) (clipped to the grid) and
    return its valid part [z0, z1). Clipped ends are true boundaries."""
    e0, e1 = max(z0 - h, 0), min(z1 + h, nz)
    ext = fn(u[e0:e1], 0.1, steps)
    return ext[z0 - e0: z1 - e0]


@pytest.mark.parametrize("dtype,fn", [(np.float64, O.heat7_f64), (np.float32, O.heat7_f32)])
@pytest.mark.parametrize("n,k,steps", [(2, 1, 3), (2, 3, 7), (4, 4, 10), (3, 2, 5)])
def test_block_decomposition_is_exact_heat(dtype, fn, n, k, steps):
    rng = np.random.default_rng(n * 100 + k)
    nz, ny, nx = 24, 8, 8
    u0 = rng.random((nz, ny, nx)).astype(dtype)
    ref = fn(u0, 0.1, steps)
    h = 1 * k
    a = slab_bounds(nz, n)
    u = u0.copy()
    done = 0
    while done < steps:
        kk = min(k, steps - done)
        new = np.empty_like(u)
        for i in range(n):
            new[a[i]:a[i + 1]] = advance_block_heat(u, a[i], a[i + 1], h, kk, nz, fn)
        u = new
        done += kk
    assert np.array_equal(u, ref)


@pytest.mark.parametrize("n,k,steps", [(2, 1, 2), (2, 2, 5), (3, 3, 6)])
def test_block_decomposition_is_exact_wave(n, k, steps):
    rng = np.random.default_rng(k)
    nz, ny, nx = 48, 9, 10
    w = (0.02 + 0.1 * rng.random((nz, ny, nx))).astype(np.float32)
    p0 = rng.standard_normal((nz, ny, nx)).astype(np.float32)
    pm0 = rng.standard_normal((nz, ny, nx)).astype(np.float32)
    amps = rng.standard_normal(steps).astype(np.float32)
    sidx = 4 + nx * (5 + ny * 20)
    ref_p, ref_pm = O.wave25_f32(p0, pm0, w, steps, src=(amps, sidx))
    h = 4 * k
    a = slab_bounds(nz, n)
    p, pm = p0.copy(), pm0.copy()
    done = 0
    plane = nx * ny
    while done < steps:
        kk = min(k, steps - done)
        np_, npm = np.empty_like(p), np.empty_like(pm)
        for i in range(n):
            e0, e1 = max(a[i] - h, 0), min(a[i + 1] + h, nz)
            local = sidx - e0 * plane
            src = (amps[done:done + kk], local) if 0 <= local < (e1 - e0) * plane else None
            bp, bpm = O.wave25_f32(p[e0:e1], pm[e0:e1], w[e0:e1], kk, src=src)
            np_[a[i]:a[i + 1]] = bp[a[i] - e0:a[i + 1] - e0]
            npm[a[i]:a[i + 1]] = bpm[a[i] - e0:a[i + 1] - e0]
        p, pm = np_, npm
        done += kk
    assert np.array_equal(p, ref_p) and np.array_equal(pm, ref_pm)


def test_replay_rate0_is_plain():
    u0 = np.random.default_rng(0).random((16, 12, 8)).astype(np.float32)
    assert np.array_equal(O.replay_heat_f32(u0, 0.1, 9, 4, 0), O.heat7_f32(u0, 0.1, 9))


@pytest.mark.parametrize("nz,n,k,steps,rate", [(48, 4, 4, 10, 6), (32, 4, 4, 9, 8), (40, 2, 8, 17, 5)])
def test_separate_compression_schedule_equals_replay(nz, n, k, steps, rate):
    """The paper's schedule, simulated chunk by chunk: the host store holds
    every R_i and C_i as its own compressed chunk. Block i decodes R_i and C_i
    (C_{i-1} is still on the device from block i-1), advances k steps, and
    writes back R_i and C_{i-1}; C_i's lower half waits on the device for
    block i+1. The resulting store decodes to the replay, bit for bit."""
    rng = np.random.default_rng(1)
    ny, nx = 8, 8
    h = k
    u0 = rng.random((nz, ny, nx)).astype(np.float32)
    cs = chunks(nz, n, h)
    a = slab_bounds(nz, n)

    store = {(c[0], c[1]): O.codec_encode(u0[c[2]:c[3]], rate) for c in cs}
    rng_of = {(c[0], c[1]): (c[2], c[3]) for c in cs}

    def dec(key):
        z0, z1 = rng_of[key]
        return O.codec_decode(store[key], (z1 - z0, ny, nx), rate)

    done = 0
    while done < steps:
        kk = min(k, steps - done)
        dev_C_prev_in = None      # decoded C_{i-1}(t), kept from block i-1
        dev_C_prev_out_low = None  # C_{i-1}(t+k) lower half, from block i-1
        new_store = {}
        for i in range(n):
            # assemble [a_i - h, a_{i+1} + h) clipped, from C_{i-1}, R_i, C_i
            parts = []
            if i > 0:
                parts.append(dev_C_prev_in)
            parts.append(dec(("R", i)))
            if i < n - 1:
                c_in = dec(("C", i))
                parts.append(c_in)
            ext = np.concatenate(parts, axis=0)
            e0 = max(a[i] - h, 0)
            out = O.heat7_f32(ext, 0.1, kk)[a[i] - e0: a[i + 1] - e0]
            # write back R_i and C_{i-1}
            r0, r1 = rng_of[("R", i)]
            new_store[("R", i)] = O.codec_encode(out[r0 - a[i]: r1 - a[i]], rate)
            if i > 0:
                c_full = np.concatenate([dev_C_prev_out_low, out[:h]], axis=0)
                new_store[("C", i - 1)] = O.codec_encode(c_full, rate)
            if i < n - 1:
                dev_C_prev_in = c_in
                dev_C_prev_out_low = out[a[i + 1] - h - a[i]:]
        store = new_store
        done += kk

    final = np.concatenate([dec((c[0], c[1])) for c in cs], axis=0)
    assert np.array_equal(final, O.replay_heat_f32(u0, 0.1, steps, k, rate))


def test_compressed_error_shrinks_with_rate():
    z, y, x = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    u0 = (np.sin(np.pi * (x + 1) / 17) * np.sin(np.pi * (y + 1) / 17) * np.sin(np.pi * (z + 1) / 17)).astype(np.float32)
    ref = O.heat7_f64(u0.astype(np.float64), 0.1, 12)
    errs = [O.errors(O.replay_heat_f64(u0, 0.1, 12, 4, r), ref)["max_rel"] for r in (4, 8, 12, 16)]
    assert all(a > b for a, b in zip(errs, errs[1:]))


def test_error_metrics():
    ref = np.ones((4, 4, 4))
    ref[0, 0, 0] = 2.0
    a = ref.copy()
    a[1, 1, 1] += 0.5
    e = O.errors(a, ref, per_plane=16, seed=0)
    assert e["max_rel"] == pytest.approx(0.25)
    assert e["l2_rel"] == pytest.approx(0.5 / np.sqrt(63 + 4))
    assert O.errors(ref, ref)["pointwise_mean_rel"] == 0.0


def test_sample_points_layout_without_replacement():
    """Sec. VI-C samples a fixed number of points in every plane: each plane
    gets exactly per_plane distinct cells of its own, and asking for the
    whole plane returns every cell of it once."""
    shape = (6, 5, 4)
    full = O.sample_points(shape, per_plane=20, seed=3).reshape(6, 20)
    for z in range(6):
        assert sorted(full[z].tolist()) == list(range(20 * z, 20 * z + 20))
    part = O.sample_points(shape, per_plane=7, seed=4).reshape(6, 7)
    for z in range(6):
        assert len(set(part[z].tolist())) == 7
        assert all(20 * z <= i < 20 * z + 20 for i in part[z])
    # 100 per plane on a large plane: still distinct
    big = O.sample_points((3, 64, 64), per_plane=100, seed=0).reshape(3, 100)
    assert all(len(set(r.tolist())) == 100 for r in big)


def test_pointwise_mean_hand_computed():
    """A field whose relative error is a known constant e_z on each plane
    z: the point-wise mean is the plain average of the e_z (equal counts
    per plane), measured against |ref| (against |a| it would be the
    average of e/(1+e)); planes whose reference is at most 1e-30 of the
    largest magnitude are left out, one just above that is kept."""
    nz, ny, nx = 6, 8, 8
    rng = np.random.default_rng(11)
    ref = rng.uniform(0.5, 1.0, (nz, ny, nx))
    ref[0, 0, 0] = 1.0                       # largest magnitude
    ref[2] = 1e-31                            # skipped: <= 1e-30 * max
    ref[3] = -2e-30                           # kept (negative: |ref| is the divisor)
    e = np.array([0.01, 0.02, 0.5, 0.04, 0.05, 0.06])
    a = ref * (1.0 + e)[:, None, None]
    r = O.errors(a, ref, per_plane=10, seed=5)
    kept = [0, 1, 3, 4, 5]
    assert r["sampled_points"] == 60
    assert r["sampled_used"] == 50
    assert r["pointwise_mean_rel"] == pytest.approx(e[kept].mean(), rel=1e-12)
    assert abs(r["pointwise_mean_rel"] - (e[kept] / (1 + e[kept])).mean()) > 1e-4
    # normwise figures of the same field, written out
    d = a - ref
    assert r["max_rel"] == pytest.approx(np.abs(d).max() / 1.0, rel=1e-12)
    assert r["l2_rel"] == pytest.approx(np.sqrt((d ** 2).sum() / (ref ** 2).sum()), rel=1e-12)
    # one plane with a larger error moves the mean by (its change) / (planes kept)
    a2 = a.copy()
    a2[4] = ref[4] * 1.25
    r2 = O.errors(a2, ref, per_plane=10, seed=5)
    assert r2["pointwise_mean_rel"] - r["pointwise_mean_rel"] == pytest.approx((0.25 - 0.05) / 5, rel=1e-9)

