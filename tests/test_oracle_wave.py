"""Pins for the oracle's 25-point acoustic wave stencil (Sec. VI: 25 points,
HALO = 4 in Table I; 8th-order central second difference on each axis,
leapfrog with two time levels).

Checked against: the exactness of an 8th-order central difference on
polynomials of degree <= 9 (which fixes all five coefficients), a dense
Kronecker-sum operator built from a banded 1D matrix, the closed-form
response to the source with no propagation, light cone and symmetry."""
import numpy as np
import pytest

import oracle as O

C = [-205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560]


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("deg", list(range(0, 10)))
def test_second_derivative_exact_on_polynomials(axis, deg):
    """In the interior L f = f'' exactly for polynomials of degree <= 9 along
    any axis (grid-index units)."""
    shape = (17, 15, 13)  # (nz, ny, nx)
    n = shape[axis]
    x = (np.arange(n) - n / 2) / 4.0
    f1 = x ** deg
    d2 = deg * (deg - 1) * x ** (deg - 2) / 16.0 if deg >= 2 else np.zeros(n)
    sh = [1, 1, 1]
    sh[axis] = n
    f = np.broadcast_to(f1.reshape(sh), shape).copy()
    L = O.lap25_f64(f)
    sl = [slice(4, -4)] * 3
    expect = np.broadcast_to(d2.reshape(sh), shape)[tuple(sl)]
    got = L[tuple(sl)]
    scale = max(1.0, np.max(np.abs(f)))
    assert np.max(np.abs(got - expect)) < 1e-10 * scale


def test_degree_10_not_exact():
    """The scheme is exactly 8th order: degree 10 leaves the truncation term."""
    n = 21
    x = (np.arange(n) - n // 2).astype(np.float64)
    f = np.broadcast_to(x ** 10, (9, 9, n)).copy()
    L = O.lap25_f64(f)
    expect = 90 * x ** 8
    assert np.max(np.abs(L[4, 4, 4:-4] - expect[4:-4])) > 1.0


def banded_1d(n):
    B = C[0] * np.eye(n)
    for m in range(1, 5):
        B += C[m] * (np.eye(n, k=m) + np.eye(n, k=-m))
    return B


def dense_L(nx, ny, nz):
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, banded_1d(nx))) + np.kron(Iz, np.kron(banded_1d(ny), Ix))
            + np.kron(banded_1d(nz), np.kron(Iy, Ix)))


def test_laplacian_dense_brute_force():
    nz, ny, nx = 7, 9, 6
    p = np.random.default_rng(5).standard_normal((nz, ny, nx))
    assert np.max(np.abs(O.lap25_f64(p).ravel() - dense_L(nx, ny, nz) @ p.ravel())) < 1e-12


def test_leapfrog_dense_brute_force_with_source():
    nz, ny, nx = 6, 5, 7
    rng = np.random.default_rng(7)
    w = 0.05 + 0.1 * rng.random((nz, ny, nx))
    p0 = rng.standard_normal((nz, ny, nx))
    pm0 = rng.standard_normal((nz, ny, nx))
    steps = 6
    amps = rng.standard_normal(steps)
    src_idx = 2 + nx * (3 + ny * 4)
    Lm = dense_L(nx, ny, nz)
    W = np.diag(w.ravel())
    a, b = pm0.ravel().copy(), p0.ravel().copy()
    for s in range(steps):
        c = 2 * b - a + W @ (Lm @ b)
        c[src_idx] += amps[s]
        a, b = b, c
    p, pm = O.wave25_f64(p0, pm0, w, steps, src=(amps, src_idx))
    assert np.max(np.abs(p.ravel() - b)) < 1e-11
    assert np.max(np.abs(pm.ravel() - a)) < 1e-11


def test_source_only_closed_form():
    """With w = 0 nothing propagates: from rest p(n) = sum_{j<n} (n-j) s_j at
    the source cell, zero elsewhere."""
    shape = (8, 8, 8)
    steps = 7
    amps = np.arange(1, steps + 1, dtype=np.float64) * 0.5
    idx = 3 + 8 * (4 + 8 * 5)
    z = np.zeros(shape)
    p, pm = O.wave25_f64(z, z, z, steps, src=(amps, idx))
    expect = sum((steps - j) * amps[j] for j in range(steps))
    assert p.ravel()[idx] == expect
    assert np.count_nonzero(p) == 1


def test_light_cone_and_symmetry():
    """An impulse spreads at most 4 cells per step along the stencil arms, so
    after n steps the support lies within L1 distance 4n; a centred impulse
    stays mirror-symmetric in each axis, bit for bit."""
    n = 25
    c = n // 2
    w = np.full((n, n, n), 0.1)
    p0 = np.zeros((n, n, n))
    p0[c, c, c] = 1.0
    for steps in (1, 2):
        for fn, dt in ((O.wave25_f64, np.float64), (O.wave25_f32, np.float32)):
            p, pm = fn(p0.astype(dt), np.zeros_like(p0, dtype=dt), w.astype(dt), steps)
            l, j, i = np.nonzero(p)
            assert np.max(np.abs(l - c) + np.abs(j - c) + np.abs(i - c)) <= 4 * steps
            assert np.array_equal(p, p[::-1, :, :])
            assert np.array_equal(p, p[:, ::-1, :])
            assert np.array_equal(p, p[:, :, ::-1])
            # x <-> y swap only reorders a commutative pair in the fixed order
            assert np.array_equal(p, np.swapaxes(p, 1, 2))


def test_fp32_order_tracks_fp64():
    rng = np.random.default_rng(2)
    shape = (20, 18, 16)
    w = 0.02 + 0.1 * rng.random(shape)
    p0 = rng.standard_normal(shape)
    pm0 = rng.standard_normal(shape)
    w32, p32, pm32 = (a.astype(np.float32) for a in (w, p0, pm0))
    a, _ = O.wave25_f32(p32, pm32, w32, 8)
    b, _ = O.wave25_f64(p32.astype(np.float64), pm32.astype(np.float64), w32.astype(np.float64), 8)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-5


def test_constant_field_stays_in_interior():
    """L of a constant is 0 where the stencil does not reach the ghosts, so
    p(n+1) = 2p - p(n-1) = the constant there."""
    n = 20
    p0 = np.full((n, n, n), 0.5)
    p, pm = O.wave25_f64(p0, p0, np.full((n, n, n), 0.1), 1)
    assert np.max(np.abs(p[4:-4, 4:-4, 4:-4] - 0.5)) < 1e-15
