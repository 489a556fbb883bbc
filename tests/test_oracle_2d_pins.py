"""Pins of the oracle of the paper's 2D Laplace jacobi benchmark (CPU only):
discrete eigenmodes, a closed-form residual, harmonic fixed points, and a
dense brute-force operator built from the 5-point definition."""
import math

import numpy as np

import oracle

PI = math.pi


def mode(nx, ny, a, b, ld_extra=0):
    si = np.sin(a * PI * np.arange(nx + 2) / (nx + 1))
    sj = np.sin(b * PI * np.arange(ny + 2) / (ny + 1))
    u = np.zeros((ny + 2, nx + 2 + ld_extra))
    u[:, : nx + 2] = sj[:, None] * si[None, :]
    u[0, :] = u[-1, :] = 0
    u[:, 0] = 0
    u[:, nx + 1:] = 0
    return u


def test_eigenmode_one_sweep():
    for (nx, ny, a, b) in [(13, 7, 2, 3), (20, 31, 1, 5), (9, 9, 4, 1)]:
        u = mode(nx, ny, a, b)
        lam = (math.cos(a * PI / (nx + 1)) + math.cos(b * PI / (ny + 1))) / 2
        got = oracle.jacobi2d(u, 1)
        assert np.max(np.abs(got - lam * u)) <= 4e-16 * np.max(np.abs(u)) * 4
        # and after five sweeps lam^5 (linearity, ping-pong placement)
        got5 = oracle.jacobi2d(u, 5)
        assert np.max(np.abs(got5 - lam ** 5 * u)) <= 1e-14


def test_residual_closed_form():
    nx, ny, a, b = 15, 11, 3, 2
    h = 1.0 / 16
    u = mode(nx, ny, a, b)
    lam_op = (4 - 2 * math.cos(a * PI / (nx + 1)) - 2 * math.cos(b * PI / (ny + 1))) / (h * h)
    want = lam_op * math.sqrt((nx + 1) * (ny + 1) / 4.0)
    assert abs(oracle.laplace2d_resid_l2(u, h) - want) <= 1e-12 * want


def test_harmonic_and_constant_fields_are_fixed_points():
    nx, ny = 12, 9
    i = np.arange(nx + 2)[None, :] / 8.0
    j = np.arange(ny + 2)[:, None] / 8.0
    lin = np.ascontiguousarray(i + 2 * j + 0 * i * j)  # discrete harmonic, dyadic values
    assert np.array_equal(oracle.jacobi2d(lin, 7), lin)
    assert oracle.laplace2d_resid_l2(lin, 0.1) == 0.0
    c = np.full((ny + 2, nx + 2), 0.75)
    assert np.array_equal(oracle.jacobi2d(c, 3), c)


def test_dense_brute_force():
    nx, ny = 4, 5
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, (ny + 2, nx + 2))
    n = nx * ny
    idx = lambda i, j: (j - 1) * nx + (i - 1)
    N = np.zeros((n, n))
    g = np.zeros(n)
    for j in range(1, ny + 1):
        for i in range(1, nx + 1):
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 1 <= ii <= nx and 1 <= jj <= ny:
                    N[idx(i, j), idx(ii, jj)] = 1.0
                else:
                    g[idx(i, j)] += u[jj, ii]
    x = u[1:-1, 1:-1].reshape(-1)
    want = (N @ x + g) / 4.0
    got = oracle.jacobi2d(u, 1)[1:-1, 1:-1].reshape(-1)
    assert np.max(np.abs(got - want)) <= 1e-15
    # the residual is (N x + g - 4 x) / h^2
    h = 0.25
    r = (N @ x + g - 4 * x) / (h * h)
    assert abs(oracle.laplace2d_resid_l2(u, h) - np.linalg.norm(r)) <= 1e-13 * np.linalg.norm(r)


def test_padded_leading_dimension_and_halo_untouched():
    nx, ny = 10, 6
    rng = np.random.default_rng(4)
    tight = rng.uniform(0, 1, (ny + 2, nx + 2))
    padded = np.full((ny + 2, nx + 2 + 5), -9.0)
    padded[:, : nx + 2] = tight
    a = oracle.jacobi2d(tight, 4)
    b = oracle.jacobi2d(padded, 4, nx=nx)
    assert np.array_equal(a, b[:, : nx + 2])
    assert np.all(b[:, nx + 2:] == -9.0)
    assert np.array_equal(a[0], tight[0]) and np.array_equal(a[:, 0], tight[:, 0])
