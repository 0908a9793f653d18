"""Pins of the oracle on curved, rough and porous voxel solids (the outlook of
Sec. IV; wall geometry of Sec. II B applied to arbitrary masks).

* The reconstructed wall normal at wall nodes of a voxelised sphere points
  into the sphere (cosine with the inward radius close to 1 on average).
* On a cylinder whose axis runs along y, the mask is invariant under y
  shifts, so the integer normal has no y component at all.
* Every donor of every wall node is a fluid node.
* A uniform rest state stays uniform and at rest on every geometry (the
  gradient vanishes, so the ghosts copy their donors and bounce-back keeps the
  rest equilibrium).
* The phase-field volume is conserved to FP64 rounding (Eqs. (48)-(55))."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

Q = 27
CASES = {
    "sphere": lambda: W.sphere_substrate(),
    "cylinder": lambda: W.cylinder_substrate(),
    "rough": lambda: W.rough_wall(seed=3),
    "porous": lambda: W.porous_packing(seed=4),
}


def _coords(idx, shape):
    nx, ny, nz = shape
    return idx % nx, (idx // nx) % ny, idx // (nx * ny)


def test_sphere_wall_normals_point_into_the_solid(orc):
    w = W.sphere_substrate()
    nx, ny, nz = w.shape
    idx, n6, q = orc.wall_nodes(w.solid, w.shape)
    x, y, z = _coords(idx, w.shape)
    cx, cy, cz = w.meta["centre"]
    r = np.stack([x - cx, y - cy, z - cz], 1).astype(float)
    on = (z >= 2) & (z < nz - 1) & (np.linalg.norm(r, axis=1) <= w.meta["Rs"] + 1.0)
    assert on.sum() > 1000
    cos = (n6 * r).sum(1) / np.linalg.norm(n6, axis=1) / np.linalg.norm(r, axis=1)
    assert cos[on].mean() < -0.95
    assert cos[on].max() < -0.6


def test_cylinder_normals_have_no_axial_component(orc):
    w = W.cylinder_substrate()
    idx, n6, q = orc.wall_nodes(w.solid, w.shape)
    assert len(idx) > 0
    np.testing.assert_array_equal(n6[:, 1], 0)


@pytest.mark.parametrize("case", sorted(CASES))
def test_donors_are_fluid(orc, case):
    w = CASES[case]()
    nx, ny, nz = w.shape
    c, _, _ = orc.lattice()
    idx, n6, q = orc.wall_nodes(w.solid, w.shape)
    assert (q >= 0).all()
    x, y, z = _coords(idx, w.shape)
    dx, dy, dz = (x + c[q, 0]) % nx, (y + c[q, 1]) % ny, (z + c[q, 2]) % nz
    assert (w.solid[dx + nx * (dy + ny * dz)] == 0).all()


@pytest.mark.parametrize("case", sorted(CASES))
def test_uniform_rest_state_invariant(orc, case):
    w = CASES[case]()
    N = w.N
    fl = w.solid == 0
    for phi_c in (0.3, 1.0):
        s = orc.OracleSim.create(w.shape, w.solid, w.theta.astype(np.float64), orc.Params(**w.params),
                                 np.full(N, phi_c))
        f0 = s.f.copy()
        s.step(3)
        np.testing.assert_allclose(s.phi[fl], phi_c, atol=1e-14)
        np.testing.assert_allclose(s.f.reshape(Q, N)[:, fl], f0.reshape(Q, N)[:, fl], atol=1e-15)
        np.testing.assert_allclose(s.u.reshape(3, N)[:, fl], 0.0, atol=1e-15)


@pytest.mark.parametrize("case", ["rough", "porous"])
def test_volume_conserved(orc, case):
    w = CASES[case]()
    s = orc.OracleSim.create(w.shape, w.solid, w.theta.astype(np.float64), orc.Params(**w.params),
                             w.phi0.astype(np.float64))
    m0 = s.mass()
    s.step(20)
    assert abs(s.mass() - m0) <= 1e-12 * m0
