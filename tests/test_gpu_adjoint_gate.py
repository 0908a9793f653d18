"""The adjoint at the stated length of the contact-angle inversion workload:
128 x 128 x 64 lattice, bottom-wall angle field from four Gaussian bumps,
hemispherical droplet R = 24, 1000 steps, checkpoints every K = 50.  The
target is the final phase field of the run at theta_seed (here the GPU's own
run), the gradient is taken at theta_{seed + 1000}.

Reference: central differences (h = 1e-4 rad) of the FP64 C oracle's loss,
stored in tests/golden/adjoint_fd_128x128x64.json by
tests/golden/adjoint_fd.py (which calls only oracle/): one per sampled wall
node (16 nodes drawn from the annulus around the initial contact line) and
one along a random direction over those 16 nodes.  Bound: 1e-3 relative per
node (on a node whose derivative is below 1% of the largest component, the
absolute error allowed at that threshold) and along the direction; the 4
far-field wall nodes, never reached by the interface, have a zero
derivative.

Measured: the FP32 reverse sweep misses that bound at 1000 steps by two orders
of magnitude on this drop.  Its error grows with the rollout
length (test_error_growth_large_drop: 1e-6 after 12 steps, 1e-3 after
100-200, a blow-up between 500 and 1000); on a drop small enough that FP32
resolves its whole liquid phase the same code agrees with central differences
at 1000 steps (test_small_drop_1000_steps).  The cause: where 1 - phi is below
2^-24 (the inside of the R = 24 drop), the FP32 phase field is flat to within
round-off, so the unit normal of the compressive flux, and the factor
phi (1 - phi) / |grad phi| of its derivative, are set by round-off; the exact
FP64 derivative carries O(1) terms through those normals, the FP32 one
amplifies noise through them."""
import json
import os

import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_fd_128x128x64.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="finite-difference reference not generated yet")
@pytest.mark.xfail(strict=True, reason="FP32 reverse sweep: the error grows with the rollout on the R = 24 drop, whose "
                                       "liquid phase FP32 cannot resolve (measured 1e2 relative at 1000 steps)")
def test_gradient_matches_oracle_finite_differences_at_1000_steps():
    from paper_2607_25444_amd import capi, tuning
    d = json.load(open(GOLDEN))
    steps, K = d["steps"], 50
    w = W.adjoint_128(seed=d["theta_seed_gradient"])
    theta_t = W.adjoint_128(seed=d["theta_seed_target"]).theta
    s = capi.Sim(w.shape, w.params)
    s.set_launch(*tuning.launch_for(w.shape))
    # target: the run at theta_seed
    s.set_geometry(w.solid, theta_t)
    s.set_state(w.phi0)
    s.step(steps)
    target, _, _ = s.fields()
    target = target.clone()
    # gradient at theta_{seed + 1000}
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0)
    L, dth = s.adjoint(steps, K, target)
    idx, _, _ = s.wall_nodes()
    s.sync()
    s.close()
    g = dth.cpu().numpy()
    pos = {int(k): i for i, k in enumerate(idx)}
    gn = np.array([g[pos[k]] for k in d["nodes"]])
    fd = np.array(d["fd"])
    gmax = float(np.abs(g).max())
    # relative bound 1e-3 on nodes that carry at least 1% of the largest gradient component; on a node below
    # that (the derivative nearly vanishes there) the same absolute error as at the 1% threshold
    scale = np.maximum(np.abs(fd), 1e-2 * gmax)
    err = np.abs(gn - fd) / scale
    print("loss", L, "max |dL/dtheta|", gmax)
    for k, a, b, r in zip(d["nodes"], gn, fd, err):
        print(f"wall node {k}: adjoint {a:.6e} fd {b:.6e} rel {abs(a - b) / abs(b):.2e}, error over its scale {r:.2e}")
    v = np.array(d["direction"])
    gd = float(np.dot(v, gn))
    print(f"direction: adjoint {gd:.6e} fd {d['fd_direction']:.6e}")
    assert np.sum(np.abs(fd) >= 1e-2 * gmax) >= 12  # most sampled nodes are well inside the gradient's support
    assert np.all(err <= 1e-3), err
    assert abs(gd - d["fd_direction"]) <= 1e-3 * abs(d["fd_direction"])
    far = np.array([g[pos[k]] for k in d["far_nodes"]])
    assert np.abs(far).max() <= 1e-6 * gmax


GROWTH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_fd_growth.json")


def _gpu_grad(w, theta_t, nodes, n, K):
    from paper_2607_25444_amd import capi, tuning
    s = capi.Sim(w.shape, w.params)
    s.set_launch(*tuning.launch_for(w.shape))
    s.set_geometry(w.solid, theta_t)
    s.set_state(w.phi0)
    s.step(n)
    target, _, _ = s.fields()
    target = target.clone()
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0)
    _, dth = s.adjoint(n, K, target)
    idx, _, _ = s.wall_nodes()
    s.sync()
    s.close()
    g = dth.cpu().numpy()
    pos = {int(k): i for i, k in enumerate(idx)}
    return np.array([g[pos[k]] for k in nodes])


def _err(gn, fd):
    """Largest error on the sampled nodes relative to the largest sampled derivative."""
    fd = np.asarray(fd)
    return float(np.abs(gn - fd).max() / np.abs(fd).max())


@pytest.mark.skipif(not os.path.exists(GROWTH), reason="finite-difference reference not generated yet")
def test_error_growth_large_drop():
    """The 128 x 128 x 64 workload after 12 to 200 steps (K = 50) against central
    differences of the FP64 oracle on three sampled wall nodes: agreement to
    1e-5 after 12 steps and 1e-3 after 50, then errors of about 1e-3 after 100
    and 200 steps (bound 1e-2); the gradient blows up between 500 and 1000
    steps (the expected failure above)."""
    d = json.load(open(GROWTH))["cases"]["adjoint_128x128x64"]
    w = W.adjoint_128(seed=1000)
    theta_t = W.adjoint_128(seed=0).theta
    errs = {}
    for n, fd in sorted(d["fd"].items(), key=lambda kv: int(kv[0])):
        gn = _gpu_grad(w, theta_t, d["nodes"], int(n), min(50, int(n)))
        errs[int(n)] = _err(gn, fd)
        print(f"{n} steps: adjoint {gn} fd {fd} error {errs[int(n)]:.2e}", flush=True)
    assert errs[12] <= 1e-5
    assert errs[50] <= 1e-3
    assert max(errs.values()) <= 1e-2


@pytest.mark.skipif(not os.path.exists(GROWTH), reason="finite-difference reference not generated yet")
def test_small_drop_1000_steps():
    """A drop of radius 9 on a 48 x 48 x 24 lattice (same angle fields and
    loss; 1 - phi stays above 1e-4, which FP32 resolves): the gradient agrees
    with central differences of the FP64 oracle to 1e-3 after 200 and 1000
    steps, with K = 50."""
    d = json.load(open(GROWTH))["cases"]["adjoint_small_48x48x24"]
    nx, ny, nz = 48, 48, 24
    R = 9.0
    phi0 = W.tanh_droplet((nx, ny, nz), ((nx - 1) / 2 - 0.3, (ny - 1) / 2 - 0.7, 0.5), R, 4.0).astype(np.float32)
    w = W.Workload("adjoint_small_48x48x24", (nx, ny, nz), W.flat_walls((nx, ny, nz)),
                   W.gaussian_bump_theta((nx, ny, nz), 1000), phi0, W.default_params(), 1000, dict(R=R))
    theta_t = W.gaussian_bump_theta((nx, ny, nz), 0)
    for n, fd in sorted(d["fd"].items(), key=lambda kv: int(kv[0])):
        gn = _gpu_grad(w, theta_t, d["nodes"], int(n), 50)
        e = _err(gn, fd)
        print(f"{n} steps: adjoint {gn} fd {fd} error {e:.2e}", flush=True)
        assert e <= 1e-3
