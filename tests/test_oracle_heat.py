"""Pins for the oracle's 7-point heat stencil (Sec. III, the 3D analogue of the
five-point Laplace example), each checked against mathematics the oracle does
not share: the closed-form Dirichlet eigenmodes, a dense Kronecker-sum matrix,
exact invariants."""
import numpy as np
import pytest

import oracle as O


def eigenmode(shape, p):
    nz, ny, nx = shape
    ix = np.sin(np.pi * p[0] * (np.arange(nx) + 1) / (nx + 1))
    iy = np.sin(np.pi * p[1] * (np.arange(ny) + 1) / (ny + 1))
    iz = np.sin(np.pi * p[2] * (np.arange(nz) + 1) / (nz + 1))
    return iz[:, None, None] * iy[None, :, None] * ix[None, None, :]


def decay_factor(shape, p, alpha):
    nz, ny, nx = shape
    s = sum(np.sin(np.pi * pd / (2 * (n + 1))) ** 2 for pd, n in zip(p, (nx, ny, nz)))
    return 1.0 - 4.0 * alpha * s


@pytest.mark.parametrize("shape,p", [((8, 8, 8), (1, 2, 1)), ((10, 6, 8), (2, 1, 3)), ((7, 9, 5), (3, 4, 2))])
def test_eigenmode_decays_by_closed_form(shape, p):
    """sin-product modes are eigenvectors of I + alpha*Laplacian with zero
    Dirichlet ghosts; eigenvalue 1 - 4 alpha sum sin^2(pi p_d / (2(N_d+1)))."""
    alpha, steps = 0.1, 10
    u0 = eigenmode(shape, p)
    lam = decay_factor(shape, p, alpha)
    u = O.heat7_f64(u0, alpha, steps)
    assert np.max(np.abs(u - lam ** steps * u0)) < 1e-14


def kron_laplacian(nx, ny, nz):
    def d1(n):
        return -2 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    # flat index = i + nx*(j + ny*l): x is the fastest (rightmost Kronecker factor)
    return np.kron(Iz, np.kron(Iy, d1(nx))) + np.kron(Iz, np.kron(d1(ny), Ix)) + np.kron(d1(nz), np.kron(Iy, Ix))


def test_dense_matrix_power_brute_force():
    nz, ny, nx = 7, 5, 6
    alpha, steps = 0.1, 5
    rng = np.random.default_rng(11)
    u0 = rng.random((nz, ny, nx))
    A = np.eye(nx * ny * nz) + alpha * kron_laplacian(nx, ny, nz)
    ref = np.linalg.matrix_power(A, steps) @ u0.ravel()
    u = O.heat7_f64(u0, alpha, steps)
    assert np.max(np.abs(u.ravel() - ref)) < 1e-13


def test_constant_field_light_cone_exact():
    """A constant stays exactly constant at cells more than t cells away from
    every face after t steps (the zero ghosts have not reached them)."""
    n, t = 14, 4
    u0 = np.full((n, n, n), 0.75)
    for fn in (O.heat7_f64, O.heat7_f32):
        u = fn(u0, 0.1, t)
        inner = u[t:n - t, t:n - t, t:n - t]
        assert np.all(inner == 0.75)
        # and the boundary layer did change
        assert u[0, 0, 0] < 0.75


def test_maximum_principle():
    """1 - 6 alpha >= 0 makes each update a convex combination with the zero
    ghosts, so values stay in [0, max u0]."""
    rng = np.random.default_rng(3)
    u0 = rng.random((12, 10, 9))
    u = O.heat7_f64(u0, 0.1, 20)
    assert u.min() >= 0.0 and u.max() <= u0.max()


def test_fp32_order_tracks_fp64():
    rng = np.random.default_rng(0)
    u0 = rng.random((16, 16, 16)).astype(np.float32)
    a = O.heat7_f32(u0, 0.1, 10)
    b = O.heat7_f64(u0.astype(np.float64), 0.1, 10)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 2e-6


def test_zero_steps_is_identity():
    u0 = np.random.default_rng(1).random((4, 5, 6))
    assert np.array_equal(O.heat7_f64(u0, 0.1, 0), u0)
