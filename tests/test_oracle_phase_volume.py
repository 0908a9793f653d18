"""Pins of the oracle's CAC update (Sec. II A 1) and volume correction
(Sec. II C) against conservation laws, the TVD property, exact transport of
linear profiles and the equilibrium of the planar tanh profile."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W


def _grid(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1).astype(float), y.reshape(-1).astype(float), z.reshape(-1).astype(float)


def _uniform_u(N, u):
    return np.concatenate([np.full(N, u[0]), np.full(N, u[1]), np.full(N, u[2])])


def test_phase_conservative_periodic(orc):
    """Advection (flux differences), diffusion and compression (isotropic
    divergence) all conserve sum(phi) on a periodic box, for any velocity."""
    shape = (10, 9, 8)
    N = 10 * 9 * 8
    solid = np.zeros(N, np.uint8)
    for seed in range(3):
        phi = W.random_smooth_field(shape, seed)
        u = np.concatenate([W.random_smooth_field(shape, 10 + seed + d, -0.1, 0.1) for d in range(3)])
        ps = orc.phase(orc.Params(), shape, solid, phi, u)
        assert ps.sum() == pytest.approx(phi.sum(), rel=1e-13)
        assert np.abs(ps - phi).max() > 1e-4


def test_advection_no_flux_through_walls(orc):
    """With D = kappa = 0 the update is pure flux differencing with zero flux on
    faces that touch a solid: the fluid sum is conserved with walls present."""
    shape = (8, 8, 10)
    N = 8 * 8 * 10
    solid = W.random_geometry(shape, 4)
    phi = W.random_smooth_field(shape, 1)
    u = np.concatenate([W.random_smooth_field(shape, 20 + d, -0.15, 0.15) for d in range(3)])
    ps = orc.phase(orc.Params(D=0.0), shape, solid, phi, u)
    fl = solid == 0
    assert ps[fl].sum() == pytest.approx(phi[fl].sum(), rel=1e-13)
    np.testing.assert_array_equal(ps[~fl], phi[~fl])  # solid nodes untouched


def test_muscl_linear_profile_exact(orc):
    """A linear profile under uniform velocity is transported exactly by the
    MUSCL-minmod fluxes (both slopes equal the profile slope): phi* = phi - u.grad(phi),
    for either sign of each velocity component (upwind selection)."""
    shape = (12, 12, 12)
    N = 12 ** 3
    x, y, z = _grid(shape)
    phi = 0.2 + 0.01 * x + 0.02 * y - 0.015 * z
    m = (x >= 2) & (x <= 9) & (y >= 2) & (y <= 9) & (z >= 2) & (z <= 9)
    for u in ((0.1, 0.05, -0.07), (-0.1, -0.05, 0.07)):
        ps = orc.phase(orc.Params(D=0.0), shape, np.zeros(N, np.uint8), phi, _uniform_u(N, u))
        exp = phi - (u[0] * 0.01 + u[1] * 0.02 - u[2] * 0.015)
        np.testing.assert_allclose(ps[m], exp[m], atol=1e-15)


def test_muscl_tvd(orc):
    """Maximum principle of the limited scheme: a discontinuous pattern in
    [0, 1] advected by a uniform velocity (CFL 0.2) creates no new extrema."""
    shape = (12, 10, 8)
    N = 12 * 10 * 8
    rng = np.random.default_rng(7)
    phi = (rng.uniform(size=N) > 0.5).astype(float)
    phi = 0.5 * phi + 0.5 * np.roll(phi, 1)
    for u in ((0.1, 0.05, 0.05), (-0.08, 0.06, -0.06)):
        ps = orc.phase(orc.Params(D=0.0), shape, np.zeros(N, np.uint8), phi, _uniform_u(N, u))
        assert ps.min() >= phi.min() - 1e-15
        assert ps.max() <= phi.max() + 1e-15


def test_minmod_extremum_first_order(orc):
    """At a local maximum minmod slopes vanish: the face value is the cell value
    (first-order upwind).  Single spike advected along +x."""
    shape = (9, 4, 4)
    N = 9 * 16
    x, y, z = _grid(shape)
    phi = np.where(x == 4, 1.0, 0.0)
    u = 0.2
    ps = orc.phase(orc.Params(D=0.0), shape, np.zeros(N, np.uint8), phi, _uniform_u(N, (u, 0, 0)))
    np.testing.assert_allclose(ps[x == 4], 1.0 - u, atol=1e-15)
    np.testing.assert_allclose(ps[x == 5], u, atol=1e-15)
    np.testing.assert_allclose(ps[(x != 4) & (x != 5)], 0.0, atol=1e-15)


def test_planar_tanh_is_cac_equilibrium(orc):
    """At rest the planar profile (1 - tanh(2 s/delta))/2 balances diffusion and
    compression exactly in the continuum when kappa = 4 D/delta (Eq. (26)).  The
    discrete residual relative to the diffusion term is small and falls at
    second order in 1/delta (a wrong kappa or sign leaves an O(1) residual)."""
    rel = []
    for delta in (4.0, 8.0, 16.0):
        shape = (4, 4, 128)
        N = 4 * 4 * 128
        x, y, z = _grid(shape)
        phi = 0.5 * (1 - np.tanh(2 * (z - 63.7) / delta))
        p = orc.Params(delta=delta, D=0.1)
        ps = orc.phase(p, shape, np.zeros(N, np.uint8), phi, np.zeros(3 * N))
        lap = orc.lap_iso(phi, shape)
        m = (z > 10) & (z < 118)  # away from the periodic seam of the profile
        rel.append(np.abs(ps - phi)[m].max() / np.abs(p.D * lap)[m].max())
    assert rel[0] < 0.12
    assert rel[1] < rel[0] / 3 and rel[2] < rel[1] / 3


def test_volume_correction_exact(orc):
    shape = (8, 8, 10)
    N = 8 * 8 * 10
    solid = W.flat_walls(shape)
    rng = np.random.default_rng(3)
    phis = np.clip(W.random_smooth_field(shape, 5, -0.1, 1.1), 0.0, 1.0)
    phis[rng.integers(0, N, 20)] = 0.0005  # below the band
    M_t = orc.mass(shape, solid, phis) + 0.37
    new, lam = orc.volume(orc.Params(), shape, solid, phis, M_t)
    fl = solid == 0
    assert new[fl].sum() == pytest.approx(M_t, rel=1e-14)
    np.testing.assert_array_equal(new[~fl], phis[~fl])
    band = fl & (phis > 1e-3) & (phis < 1 - 1e-3)
    np.testing.assert_array_equal(new[fl & ~band], phis[fl & ~band])
    # the correction is proportional to phi*(1-phi*) with one multiplier
    ratio = (new - phis)[band] / (phis * (1 - phis))[band]
    np.testing.assert_allclose(ratio, lam, rtol=1e-9)
    assert lam > 0


def test_volume_degenerate(orc):
    shape = (4, 4, 6)
    N = 96
    solid = W.flat_walls(shape)
    phis = np.where(np.arange(N) % 3 == 0, 1.0, 0.0)
    new, lam = orc.volume(orc.Params(), shape, solid, phis, 100.0)
    assert lam == 0.0
    np.testing.assert_array_equal(new, phis)  # W = 0: nothing to redistribute
    phis = W.random_smooth_field(shape, 2)
    new, lam = orc.volume(orc.Params(volume_correction=0), shape, solid, phis, 100.0)
    np.testing.assert_array_equal(new, phis)
