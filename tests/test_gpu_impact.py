"""Droplet impact at liquid-to-gas density ratio 1000 (Sec. III C) on the GPU
(FP32, through the C ABI).

* Parity with the FP64 oracle after 100 steps: max |dphi| <= 1e-5 and max |du|
  <= 1e-4 max |u| over fluid nodes (the plain step's bar), from the same initial
  velocity field.
* A longer run stays finite, keeps the phase-field volume (FP64 correction) and
  spreads the droplet beyond its initial diameter on the 130 degree wall."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w):
    from paper_2607_25444_amd import capi
    s = capi.Sim(w.shape, w.params)
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0, w.meta["u0"])
    return s


def test_impact_parity(orc):
    w = W.impact((40, 40, 36), R=9.0, We=10.0)
    steps = 100
    print(f"[impact] parity {w.name} U0={w.meta['U0']:.4f} steps={steps}", flush=True)
    s = _sim(w)
    s.step(steps)
    phi, u, _ = s.fields()
    s.sync()
    phi = phi.cpu().numpy().astype(np.float64)
    u = u.cpu().numpy().astype(np.float64).reshape(3, -1)
    s.close()
    o = orc.OracleSim.create(w.shape, w.solid, w.theta.astype(np.float64), orc.Params(**w.params),
                             w.phi0.astype(np.float64), u0=w.meta["u0"].astype(np.float64))
    o.step(steps)
    fl = w.solid == 0
    uo = o.u.reshape(3, -1)
    e_phi = float(np.abs(phi - o.phi)[fl].max())
    umax = float(np.abs(uo[:, fl]).max())
    e_u = float(np.abs(u - uo)[:, fl].max()) / umax
    print(f"[impact] max|dphi| = {e_phi:.2e}, max|du|/max|u| = {e_u:.2e} (max|u| = {umax:.2e})")
    assert e_phi <= 1e-5
    assert e_u <= 1e-4


def test_impact_long_run_spreads_and_conserves():
    w = W.impact((96, 96, 48), R=14.0, We=30.0)
    nx, ny, nz = w.shape
    print(f"[impact] long run {w.name} U0={w.meta['U0']:.4f}", flush=True)
    s = _sim(w)
    v0 = s.volume()
    widths = []
    for _ in range(20):
        s.step(100)
        phi = s.fields()[0].cpu().numpy().reshape(nz, ny, nx)
        widths.append(int((phi[1:4].max(axis=(0, 1)) > 0.5).sum()))
    v1 = s.volume()
    s.sync()
    s.close()
    beta = max(widths) / (2 * 14.0)
    print(f"[impact] lateral extension per 100 steps {widths}; beta_max ~ {beta:.2f}; volume drift {(v1 - v0) / v0:.1e}")
    assert abs(v1 - v0) <= 1e-6 * v0
    assert beta > 1.0
