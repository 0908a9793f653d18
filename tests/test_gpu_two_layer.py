"""The viscous-correction force F_nu (Eq. (21)) and the mixture laws (Eqs.
(8)-(10)) on the GPU: force-driven two-layer channel flow (liquid below gas,
density 1.2/0.4, viscosity 0.05/0.15) to its steady state, against the
quadrature of d/dz(mu du/dz) = -f used to pin the oracle, and against the
oracle's own steady profile."""
import numpy as np
import pytest

from tests import test_oracle_two_layer as T

pytestmark = pytest.mark.gpu


def _setup(H):
    nz = H + 2
    shape = (4, 4, nz)
    solid = np.zeros((nz, 4, 4), np.uint8)
    solid[0] = solid[-1] = 1
    zi = 0.5 + H / 2.0
    delta = 0.25 * H
    z = np.arange(nz, dtype=np.float64)
    phi0 = np.broadcast_to(T._phi_profile(z, zi, delta)[:, None, None], (nz, 4, 4)).reshape(-1)
    prm = dict(rho_l=T.RHO_L, rho_g=T.RHO_G, nu_l=T.NU_L, nu_g=T.NU_G, delta=delta, sigma=0.02,
               g=(T.G, 0.0, 0.0))
    steps = int(8 * H * H / min(T.NU_L, T.NU_G))
    return shape, solid.reshape(-1), np.ascontiguousarray(phi0), prm, zi, delta, steps


@pytest.mark.parametrize("H", [8, 16])
def test_two_layer_channel_gpu(orc, H):
    from paper_2607_25444_amd import capi
    from paper_2607_25444_amd import workloads as W
    shape, solid, phi0, prm, zi, delta, steps = _setup(H)
    nz = shape[2]
    N = int(np.prod(shape))
    p = W.default_params(**prm)
    s = capi.Sim(shape, p)
    s.set_launch(16, 4, 4, 1, 0)
    s.set_geometry(solid, np.full(N, np.pi / 2, np.float32))
    s.set_state(phi0.astype(np.float32))
    s.step(steps)
    _, u, _ = s.fields()
    s.sync()
    ug = u.cpu().numpy().astype(np.float64).reshape(3, nz, 4, 4)[0, 1:H + 1, 0, 0]
    s.close()
    zq = np.arange(1, H + 1, dtype=np.float64)
    ref = T._reference(H, zi, delta, zq)
    err = np.abs(ug - ref).max() / np.abs(ref).max()
    o = orc.OracleSim.create(shape, solid, np.full(N, np.pi / 2), orc.Params(**p), phi0.astype(np.float32))
    o.step(steps)
    uo = o.u.reshape(3, nz, 4, 4)[0, 1:H + 1, 0, 0]
    print(f"H={H}: GPU vs reference {err:.3e}, GPU vs oracle {np.abs(ug - uo).max() / np.abs(uo).max():.3e}")
    assert err < (3e-2 if H == 8 else 1e-2)
    assert np.abs(ug - uo).max() <= 1e-4 * np.abs(uo).max()
