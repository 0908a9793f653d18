"""Pins of the oracle's node-level arithmetic against closed forms.

D3Q27 quadrature (Sec. II A), the third-order Hermite equilibrium (Eq. (11)),
the Guo forcing term (Eq. (17)) and the regularised non-equilibrium part
(Eqs. (14), (16)) have moment identities that follow from Hermite
orthogonality; each test sums the oracle's populations and compares the
moments with those identities, so a wrong weight, sign, index or prefactor
anywhere in the oracle fails one of them.
"""
import itertools

import numpy as np
import pytest

CS2 = 1.0 / 3.0
I3 = np.eye(3)


@pytest.fixture(scope="module")
def lat(orc):
    return orc.lattice()


def test_velocity_set(lat):
    c, w, opp = lat
    assert c.shape == (27, 3)
    assert len({tuple(v) for v in c}) == 27
    assert set(np.unique(c)) == {-1, 0, 1}
    assert tuple(c[0]) == (0, 0, 0)
    for i in range(27):
        np.testing.assert_array_equal(c[opp[i]], -c[i])
    # canonical order: opposite of odd i is i+1
    for i in range(1, 27, 2):
        assert opp[i] == i + 1


def test_weights_textbook(lat):
    c, w, _ = lat
    # D3Q27 weights are the tensor product of the D1Q3 weights (2/3, 1/6, 1/6)
    w1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
    for i in range(27):
        assert w[i] == pytest.approx(w1[c[i, 0]] * w1[c[i, 1]] * w1[c[i, 2]], abs=1e-16)


def test_isotropy(lat):
    c, w, _ = lat
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(w @ c, 0, atol=1e-16)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    np.testing.assert_allclose(M2, CS2 * I3, atol=1e-15)
    M3 = np.einsum("i,ia,ib,ig->abg", w, c, c, c)
    np.testing.assert_allclose(M3, 0, atol=1e-15)
    M4 = np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c)
    iso4 = CS2 ** 2 * (np.einsum("ab,gd->abgd", I3, I3) + np.einsum("ag,bd->abgd", I3, I3) +
                       np.einsum("ad,bg->abgd", I3, I3))
    np.testing.assert_allclose(M4, iso4, atol=1e-15)


def _rand_u(rng, scale=0.1):
    return rng.uniform(-scale, scale, 3)


def test_feq_moments(orc, lat):
    """Moments of the third-order equilibrium: p*, u, p* c_s^2 I + uu, and the
    third-order moments carried by D3Q27 (all but the aaa components)."""
    c, w, _ = lat
    rng = np.random.default_rng(1)
    for _ in range(20):
        ps = rng.uniform(-0.5, 0.5)
        u = _rand_u(rng)
        f = orc.feq(ps, u)
        assert f.sum() == pytest.approx(ps, abs=1e-15)
        np.testing.assert_allclose(f @ c, u, atol=1e-15)
        M2 = np.einsum("i,ia,ib->ab", f, c, c)
        np.testing.assert_allclose(M2, ps * CS2 * I3 + np.outer(u, u), atol=1e-15)
        M3 = np.einsum("i,ia,ib,ig->abg", f, c, c, c)
        for a, b, g in itertools.product(range(3), repeat=3):
            if a == b == g:
                continue  # H3_aaa vanishes on D3Q27 (c_a^3 = c_a, 3 c_s^2 = 1)
            exp = CS2 * (u[a] * I3[b, g] + u[b] * I3[a, g] + u[g] * I3[a, b]) + u[a] * u[b] * u[g]
            assert M3[a, b, g] == pytest.approx(exp, abs=1e-15)


def test_feq_rest_state_is_weights(orc, lat):
    c, w, _ = lat
    np.testing.assert_allclose(orc.feq(0.7, np.zeros(3)), 0.7 * w, atol=1e-16)


def test_guo_moments(orc, lat):
    """Guo forcing: zero mass source, momentum source a, stress source ua + au."""
    c, w, _ = lat
    rng = np.random.default_rng(2)
    for _ in range(20):
        u, a = _rand_u(rng), _rand_u(rng, 1e-2)
        S = orc.guo(u, a)
        assert S.sum() == pytest.approx(0.0, abs=1e-16)
        np.testing.assert_allclose(S @ c, a, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", S, c, c), np.outer(u, a) + np.outer(a, u), atol=1e-16)


def test_fneq_reg_moments(orc, lat):
    """The regularised part carries exactly A2 and A3 = S(u A2) (Hermite
    projection) and no mass or momentum."""
    c, w, _ = lat
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = _rand_u(rng)
        B = rng.normal(size=(3, 3)) * 1e-3
        A2 = B + B.T
        f = orc.fneq_reg(u, A2)
        assert f.sum() == pytest.approx(0.0, abs=1e-16)
        np.testing.assert_allclose(f @ c, 0, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, c, c), A2, atol=1e-16)
        M3 = np.einsum("i,ia,ib,ig->abg", f, c, c, c)
        A3 = np.einsum("a,bg->abg", u, A2) + np.einsum("b,ag->abg", u, A2) + np.einsum("g,ab->abg", u, A2)
        for a, b, g in itertools.product(range(3), repeat=3):
            if a == b == g:
                continue
            assert M3[a, b, g] == pytest.approx(A3[a, b, g], abs=1e-16)


def _params(orc, **kw):
    return orc.Params(**kw)


def test_collide_equilibrium_fixed_point(orc):
    """A population at equilibrium, with a flat phase field (no force), is a
    fixed point of the collision at any p*, u and viscosity."""
    rng = np.random.default_rng(4)
    for nu in (0.01, 0.04, 0.24):
        p = _params(orc, nu_l=nu, nu_g=nu)
        ps, u = rng.uniform(-0.2, 0.2), _rand_u(rng)
        f = orc.feq(ps, u)
        fp, uo, pso = orc.collide_node(p, 0.3, np.zeros(3), 0.0, f)
        np.testing.assert_allclose(fp, f, atol=1e-15)
        np.testing.assert_allclose(uo, u, atol=1e-15)
        assert pso == pytest.approx(ps, abs=1e-15)


def test_collide_moments(orc, lat):
    """Post-collision moments: p* unchanged; momentum j + a (u + a/2); the
    non-equilibrium stress relaxes by (1 - omega), omega from the viscosity
    relation nu = c_s^2 (1/omega - 1/2) (Eq. (4)).  The pure phases phi = 0
    and phi = 1 select the gas and liquid viscosities (mixture laws, Eqs. (8)-(10))."""
    c, w, _ = lat
    rng = np.random.default_rng(5)
    for rho_l, rho_g in ((1.0, 1.0), (1.2, 0.9)):
        p = _params(orc, rho_l=rho_l, rho_g=rho_g, nu_l=0.031, nu_g=0.24, g=(0.0, 0.0, -1e-5))
        for phi, nu in ((0.0, 0.24), (1.0, 0.031)):
            f = orc.feq(0.01, _rand_u(rng, 0.05)) + rng.normal(size=27) * 1e-4
            G, L = rng.normal(size=3) * 0.05, 0.01
            fp, u, ps = orc.collide_node(p, phi, G, L, f)
            assert fp.sum() == pytest.approx(ps, abs=1e-15)
            assert ps == pytest.approx(f.sum(), abs=1e-15)
            j = f @ c
            a = 2.0 * (u - j)
            np.testing.assert_allclose(fp @ c, j + a, atol=1e-15)
            omega = 1.0 / (nu / CS2 + 0.5)
            Pin = np.einsum("i,ia,ib->ab", f, c, c)
            Pout = np.einsum("i,ia,ib->ab", fp, c, c)
            sym = 0.5 * (np.outer(u, a) + np.outer(a, u))
            neq_in = Pin - ps * CS2 * I3 - np.outer(u, u) + sym
            neq_out = Pout - ps * CS2 * I3 - np.outer(u, u) - sym
            np.testing.assert_allclose(neq_out, (1.0 - omega) * neq_in, atol=1e-14)


def test_capillary_force_direction(orc, lat):
    """With rho_l = rho_g the only force is mu_phi grad(phi); at phi = 1/2,
    L = 0 the chemical potential vanishes, so no momentum is injected."""
    c, _, _ = lat
    p = _params(orc)
    f = orc.feq(0.0, np.zeros(3))
    fp, u, _ = orc.collide_node(p, 0.5, np.array([0.1, 0.0, 0.0]), 0.0, f)
    np.testing.assert_allclose(u, 0, atol=1e-17)
    # phi = 1/4 lies between the gas root 0 and the interface root 1/2 of the
    # double well, where mu_phi > 0 (L = 0): the force points along +grad(phi)
    fp, u, _ = orc.collide_node(p, 0.25, np.array([0.1, 0.0, 0.0]), 0.0, f)
    assert u[0] > 0 and abs(u[1]) < 1e-18 and abs(u[2]) < 1e-18
    fp, u, _ = orc.collide_node(p, 0.75, np.array([0.1, 0.0, 0.0]), 0.0, f)
    assert u[0] < 0
