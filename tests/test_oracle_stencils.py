"""Pins of the oracle's isotropic stencils (Eqs. (22)-(23)) against exact
polynomial and Fourier results."""
import numpy as np
import pytest


def _grid(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1).astype(float), y.reshape(-1).astype(float), z.reshape(-1).astype(float)


def _interior(shape, m=1):
    nx, ny, nz = shape
    x, y, z = _grid(shape)
    return (x >= m) & (x < nx - m) & (y >= m) & (y < ny - m) & (z >= m) & (z < nz - m)


def test_gradient_exact_on_linear(orc):
    shape = (7, 6, 5)
    x, y, z = _grid(shape)
    psi = 0.3 + 1.5 * x - 0.7 * y + 2.25 * z
    G = orc.grad_iso(psi, shape).reshape(3, -1)
    m = _interior(shape)
    np.testing.assert_allclose(G[0, m], 1.5, atol=1e-13)
    np.testing.assert_allclose(G[1, m], -0.7, atol=1e-13)
    np.testing.assert_allclose(G[2, m], 2.25, atol=1e-13)


def test_laplacian_exact_on_quadratic(orc):
    shape = (7, 6, 5)
    x, y, z = _grid(shape)
    psi = x ** 2 + 2 * y ** 2 - 0.5 * z ** 2 + 3 * x * y - y * z + 0.1 * x
    L = orc.lap_iso(psi, shape)
    m = _interior(shape)
    np.testing.assert_allclose(L[m], 2 + 4 - 1, atol=1e-12)


def test_gradient_fourier_symbol(orc):
    """For psi = sin(k x) on a periodic grid the isotropic gradient is the
    central difference sin(k) cos(k x) (the transverse weights sum to 1/6)."""
    shape = (16, 4, 4)
    x, y, z = _grid(shape)
    k = 2 * np.pi * 3 / 16
    G = orc.grad_iso(np.sin(k * x), shape).reshape(3, -1)
    np.testing.assert_allclose(G[0], np.sin(k) * np.cos(k * x), atol=1e-14)
    np.testing.assert_allclose(G[1:], 0, atol=1e-14)


def test_laplacian_fourier_symbol(orc):
    """Symbol of the isotropic Laplacian: -4 sin^2(k/2) for a 1-D wave and
    -52/9 at the checkerboard mode k = (pi, pi, pi)."""
    shape = (16, 4, 4)
    x, y, z = _grid(shape)
    k = 2 * np.pi * 5 / 16
    L = orc.lap_iso(np.cos(k * x), shape)
    np.testing.assert_allclose(L, -4 * np.sin(k / 2) ** 2 * np.cos(k * x), atol=1e-14)
    shape = (4, 4, 4)
    x, y, z = _grid(shape)
    cb = (-1.0) ** (x + y + z)
    np.testing.assert_allclose(orc.lap_iso(cb, shape), -52.0 / 9.0 * cb, atol=1e-13)


def test_divergence_free_sums(orc):
    """Both stencils are antisymmetric/zero-sum: on a periodic grid the
    gradient and the Laplacian of any field sum to zero."""
    rng = np.random.default_rng(0)
    shape = (6, 5, 4)
    psi = rng.normal(size=6 * 5 * 4)
    assert abs(orc.lap_iso(psi, shape).sum()) < 1e-12
    np.testing.assert_allclose(orc.grad_iso(psi, shape).reshape(3, -1).sum(axis=1), 0, atol=1e-12)
