"""Static contact angle of the geometric wetting condition (Sec. II B,
Eqs. (36)-(47)), as in the test of Sec. III A at a smaller radius: a
hemispherical droplet (R = 16, interface width 4, rho = 1, nu = 0.04,
sigma = 0.02) relaxes on a flat wall until its fitted angle is stationary.

What the paper fixes and what is checked:
* theta = 90 degrees is recovered within 1 degree at R = 24 (the ghost equals
  its donor; the fitted angle exceeds 90 by about 0.35 cells / R radians:
  1.3 degrees at R = 16, 0.9 at R = 24, 0.5 at R = 40);
* for the other angles the step does not recover the imposed angle within
  1 degree; the residual follows the localisation factor lambda_s of Eq. (47),
  which scales the imposed normal derivative -|grad_par phi| cot(theta_c) by
  sqrt(4 phi_f (1 - phi_f)) <= 1 across the diffuse contact line.  Its mean over
  the contact line, weighted by the gradient that sets the wall flux, is
  pi/4 ~ 0.79 for a tanh profile, so the measured angles obey
  cot(theta_measured) = k cot(theta_imposed) with k well below 1 and the same
  for hydrophilic and hydrophobic angles;
* the diagnostic reading lambda_s = 1 (ghost_localization = 0) removes that
  factor: the measured cotangent is then at least the imposed one.
The table of the paper's own setup (256^3, R0 = 40) comes from
`bench.py --angle-study`."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W
from tests import diagnostics as dg

pytestmark = pytest.mark.gpu

def _stationary_angle(theta_deg, ghost_localization=1, R=16.0, every=2000, max_steps=40000, tol=0.05):
    from paper_2607_25444_amd import capi, tuning
    shape = (int(5 * R), int(5 * R), int(2 * R + 8))
    w = W.sessile(shape, R, theta_deg)
    prm = dict(w.params, ghost_localization=ghost_localization)
    s = capi.Sim(shape, prm)
    s.set_launch(*tuning.launch_for(shape))
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0)
    hist, steps = [], 0
    while steps < max_steps:
        s.step(every)
        steps += every
        phi, _, _ = s.fields()
        a, _, _ = dg.contact_angle_sphere(phi.cpu().numpy().astype(np.float64), shape)
        hist.append(a)
        if steps >= 16000 and max(hist[-3:]) - min(hist[-3:]) < tol:
            break
    s.sync()
    s.close()
    print(f"theta {theta_deg} R {R} (ghost_localization {ghost_localization}): {hist[-1]:.2f} after {steps} steps",
          flush=True)
    return hist[-1]


def _cot(deg):
    return 1.0 / np.tan(np.deg2rad(deg))


def test_neutral_wetting_within_one_degree():
    assert abs(_stationary_angle(90.0, R=24.0, max_steps=60000) - 90.0) < 1.0


def test_residual_follows_the_localisation_factor():
    ratios = {th: _cot(_stationary_angle(th)) / _cot(th) for th in (30.0, 60.0, 120.0)}
    print("cot ratios", ratios)
    for th, k in ratios.items():
        assert 0.6 < k < 0.9, (th, k)
    # one factor for hydrophilic and hydrophobic angles alike
    assert max(ratios.values()) - min(ratios.values()) < 0.2


def test_plain_extrapolation_removes_the_factor():
    for th in (60.0, 120.0):
        k = _cot(_stationary_angle(th, ghost_localization=0)) / _cot(th)
        assert k > 0.95, (th, k)
