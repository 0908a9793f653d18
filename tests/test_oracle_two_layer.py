"""Pin of the viscous-correction force F_nu (Eq. (21)) and of the mixture laws
of density and viscosity (Eqs. (8)-(10)): force-driven two-layer channel flow.

Liquid (phi = 1, rho_l, nu_l) fills the lower half of a channel between two
solid walls and gas (phi = 0, rho_g, nu_g) the upper half, with a flat tanh
interface of width delta at mid-height; x and y are periodic.  The body force
drives the liquid along x (F_ext = (rho(phi) - rho_g) g).  In the steady state
u = u_x(z), and the momentum balance of a fluid with the dynamic viscosity
mu = rho nu interpolated linearly in phi (Eq. (9)) is

    d/dz (mu du/dz) = -f,   f = (rho(phi) - rho_g) g,   u = 0 at the half-links,

whose sharp-interface limit is the two-layer parabola with continuous velocity
and continuous shear stress mu du/dz at the interface.  The lattice Boltzmann
step recovers nu (grad u + grad u^T) from its populations; without F_nu it
would satisfy d/dz (nu du/dz) = -f/rho instead, and F_nu =
nu (grad u + grad u^T) . grad rho is exactly the term that turns the one into
the other (rho d(nu u')/dz + nu rho' u' = (mu u')').  The steady profile
therefore fixes the sign and the factor nu omega / c_s^2 of Eq. (21), and the
linear law for mu rather than for nu.

The reference profile is computed here by quadrature of the continuum problem
(independent of the oracle), and is itself pinned against the closed-form
two-layer parabola as delta -> 0.  Planted mistakes in a copy of the oracle
must fail the pin.
"""
import os

import numpy as np
import pytest
from scipy.integrate import cumulative_trapezoid

import oracle.oracle as O

RHO_L, RHO_G, NU_L, NU_G, G = 1.2, 0.4, 0.05, 0.15, 1e-6


def _phi_profile(z, zi, delta):
    return 0.5 * (1.0 - np.tanh(2.0 * (z - zi) / delta))


def _reference(H, zi, delta, zq, npts=400001):
    """u(zq) of d/dz(mu u') = -f on [1/2, H + 1/2] with u = 0 at both ends."""
    z = np.linspace(0.5, H + 0.5, npts)
    phi = _phi_profile(z, zi, delta)
    mu = RHO_G * NU_G + (RHO_L * NU_L - RHO_G * NU_G) * phi
    f = (RHO_L - RHO_G) * phi * G
    F = cumulative_trapezoid(f, z, initial=0.0)          # integral of f from the bottom wall
    A = cumulative_trapezoid(1.0 / mu, z, initial=0.0)
    B = cumulative_trapezoid(F / mu, z, initial=0.0)
    tau0 = B[-1] / A[-1]                                 # shear stress at the bottom wall
    return np.interp(zq, z, tau0 * A - B)


def _two_layer_parabola(H, s):
    """Sharp interface at s = H/2 (s = distance from the bottom wall): liquid
    below with mu1 and force density f, gas above with mu2 and no force."""
    mu1, mu2 = RHO_L * NU_L, RHO_G * NU_G
    f = (RHO_L - RHO_G) * G
    h1 = H / 2.0
    B = f * h1 * h1 / (2.0 * mu1 * (H - h1) + 2.0 * mu2 * h1)
    A = (f * h1 - mu2 * B) / mu1
    return np.where(s <= h1, -f * s * s / (2.0 * mu1) + A * s, B * (H - s))


def test_reference_tends_to_the_two_layer_parabola():
    H = 16
    s = np.linspace(0.0, H, 33)
    exact = _two_layer_parabola(H, s)
    e = [np.abs(_reference(H, 0.5 + H / 2, d, s + 0.5) - exact).max() / exact.max() for d in (0.2, 0.1, 0.05)]
    assert e[2] < 2e-3, e
    assert e[0] > e[1] > e[2], e
    # shear stress continuity: the kink of the profile at the interface
    mu1, mu2 = RHO_L * NU_L, RHO_G * NU_G
    h = 1e-6
    dl = (_two_layer_parabola(H, np.array([H / 2 - h])) - _two_layer_parabola(H, np.array([H / 2 - 2 * h]))) / h
    du = (_two_layer_parabola(H, np.array([H / 2 + 2 * h])) - _two_layer_parabola(H, np.array([H / 2 + h]))) / h
    assert mu1 * dl[0] == pytest.approx(mu2 * du[0], rel=1e-4)


def _channel_error(H, delta_per_H=0.25):
    """Max deviation of the oracle's steady u_x from the reference, relative to
    its maximum (H fluid layers, walls at z = 0 and H + 1)."""
    nz = H + 2
    shape = (2, 2, nz)
    N = 4 * nz
    solid = np.zeros((nz, 2, 2), np.uint8)
    solid[0] = solid[-1] = 1
    zi = 0.5 + H / 2.0
    delta = delta_per_H * H
    z = np.arange(nz, dtype=np.float64)
    phi0 = np.broadcast_to(_phi_profile(z, zi, delta)[:, None, None], (nz, 2, 2)).reshape(-1)
    prm = O.Params(rho_l=RHO_L, rho_g=RHO_G, nu_l=NU_L, nu_g=NU_G, delta=delta, sigma=0.02, g=(G, 0.0, 0.0))
    s = O.OracleSim.create(shape, solid.reshape(-1), np.full(N, np.pi / 2), prm, np.ascontiguousarray(phi0))
    s.step(int(8 * H * H / min(NU_L, NU_G)))
    zq = np.arange(1, H + 1, dtype=np.float64)
    u = s.u.reshape(3, nz, 2, 2)[0, 1:H + 1, 0, 0]
    ref = _reference(H, zi, delta, zq)
    return np.abs(u - ref).max() / np.abs(ref).max()


def test_two_layer_channel_converges_at_second_order():
    e8, e16 = _channel_error(8), _channel_error(16)
    assert e16 < 1e-2, (e8, e16)
    assert 3.0 < e8 / e16 < 5.0, (e8, e16)


# Planted mistakes: each must move the steady profile far outside the bound.
_F_NU_LINE = "        Fnu *= -nu * omega / CS2;\n"
_NU_LINE = "    const double nu = mu / rho;\n"
PLANTED = {
    "F_nu sign": [(_F_NU_LINE, "        Fnu *= nu * omega / CS2;\n")],
    "F_nu without nu omega / c_s^2": [(_F_NU_LINE, "        Fnu *= -1.0;\n")],
    "no F_nu": [(_F_NU_LINE, "        Fnu *= 0.0;\n")],
    "nu (not mu) linear in phi": [(_NU_LINE, "    const double nu = p->nu_g + (p->nu_l - p->nu_g) * phi;\n")],
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_mistakes_fail_the_pin(name, tmp_path):
    path = O.build_variant(os.path.join(str(tmp_path), "liboracle_planted.so"), PLANTED[name])
    with O.using_library(path):
        e = _channel_error(16)
    assert e > 3e-2, (name, e)  # three times the bound the correct step meets
