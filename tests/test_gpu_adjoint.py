"""Adjoint of the step on the GPU (libcac reverse sweep through its C ABI)
against the oracle's own adjoint and against finite differences.

* Oracle adjoint: oracle/literal.py differentiated by torch autograd in FP64,
  the exact gradient of the discrete step (its forward agrees with the C
  oracle to round-off, and its gradient with central differences of the C
  oracle; see test_oracle_adjoint.py).
* Finite differences: central differences of the FP64 C oracle,
  h = 1e-4 rad, on the wall nodes with the largest gradients.
Tolerance: the GPU computes forward and reverse in FP32; gradients must agree
with the oracle within 2e-5 of the largest gradient component (FP32 round-off
carried through ten steps each way; measured about 6e-7), and with the
finite differences within 1e-3 relative per sampled node.  Inputs avoid
exactly mirror-symmetric states, where minmod ties make the gradient
one-sided."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu


def _droplet_case(shape, seed, **pkw):
    """Sessile droplet slightly off the lattice symmetry planes, random angles."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    solid = W.flat_walls(shape)
    R = 0.3 * min(nx, ny)
    phi0 = W.tanh_droplet(shape, (nx / 2 - 0.3, ny / 2 - 0.7, 0.5), R, 4.0).astype(np.float32)
    theta = np.deg2rad(rng.uniform(40.0, 140.0, nx * ny * nz)).astype(np.float32)
    target = np.clip(W.tanh_droplet(shape, (nx / 2 + 0.4, ny / 2 - 0.2, 0.5), R * 0.95, 4.0), 0, 1).astype(np.float32)
    return solid, phi0, theta, target, W.default_params(**pkw)


def _blocks_case(shape, seed, **pkw):
    """Flat walls plus solid blocks, smooth random phase field, random angles."""
    rng = np.random.default_rng(seed)
    solid = W.random_geometry(shape, seed=seed)
    phi0 = W.random_smooth_field(shape, seed=seed).astype(np.float32)
    theta = rng.uniform(0.6, 2.5, int(np.prod(shape))).astype(np.float32)
    target = W.random_smooth_field(shape, seed=seed + 100).astype(np.float32)
    return solid, phi0, theta, target, W.default_params(**pkw)


CASES = {
    "droplet": lambda s: _droplet_case(s, 1),
    "droplet-nowallflux": lambda s: _droplet_case(s, 2, wall_compression=0),
    "blocks-density-gravity": lambda s: _blocks_case(s, 3, rho_l=4.0, nu_l=0.05, nu_g=0.03, sigma=0.01,
                                                     g=(1e-4, -2e-4, -3e-4)),
    "blocks-nocorrection": lambda s: _blocks_case(s, 4, volume_correction=0, wall_compression=0),
}


def gpu_grad(shape, solid, phi0, theta, target, params, nsteps, K, launch=None):
    from paper_2607_25444_amd import capi
    s = capi.Sim(shape, params)
    if launch:
        s.set_launch(*launch)
    s.set_geometry(solid, theta)
    s.set_state(phi0)
    s.tape_forward(nsteps, K)
    L, seed = s.loss(target)
    dth, dphi0 = s.tape_backward(seed)
    s.sync()
    idx, _, donor = s.wall_nodes()
    out = (L, dth.cpu().numpy(), dphi0.cpu().numpy().astype(np.float64), idx, donor)
    s.close()
    return out


def oracle_grad(shape, solid, phi0, theta, target, params, nsteps):
    from oracle import literal
    th_w = np.asarray(theta, dtype=np.float64)
    lit = literal.LiteralSim(shape, solid, params, phi0)
    sim_idx = lit.wall_linear_index()
    return literal.rollout_grad(shape, solid, params, phi0, th_w[sim_idx], nsteps, target), sim_idx


@pytest.mark.parametrize("name", list(CASES))
def test_gradient_matches_oracle_adjoint(name):
    shape = (20, 18, 16)
    solid, phi0, theta, target, params = CASES[name](shape)
    nsteps, K = 10, 4
    L, dth, dphi0, idx, donor = gpu_grad(shape, solid, phi0, theta, target, params, nsteps, K)
    (Lo, gth, gphi), oidx = oracle_grad(shape, solid, phi0, theta, target, params, nsteps)
    assert np.array_equal(idx, oidx)
    print(f"{name}: L gpu {L:.9e} oracle {Lo:.9e}; max|dL/dtheta| {np.abs(gth).max():.3e}, "
          f"max|dL/dphi0| {np.abs(gphi).max():.3e}")
    assert abs(L - Lo) <= 1e-5 * Lo
    eth = np.abs(dth - gth).max() / np.abs(gth).max()
    eph = np.abs(dphi0 - gphi).max() / np.abs(gphi).max()
    print(f"  rel err dtheta {eth:.2e}, dphi0 {eph:.2e}")
    assert np.all(dth[donor < 0] == 0.0)
    assert eth <= 2e-5
    assert eph <= 2e-5


def test_checkpoint_interval_does_not_change_the_gradient():
    """Segment replay reproduces the recorded sweep exactly, so any K gives the
    same bits."""
    shape = (20, 18, 16)
    solid, phi0, theta, target, params = CASES["droplet"](shape)
    ref = None
    for K in (1, 3, 7, 9, 20):
        L, dth, dphi0, _, _ = gpu_grad(shape, solid, phi0, theta, target, params, 9, K)
        if ref is None:
            ref = (L, dth, dphi0)
        else:
            assert L == ref[0]
            assert np.array_equal(dth, ref[1])
            assert np.array_equal(dphi0, ref[2])


@pytest.mark.parametrize("K", [4, 9, 20])
def test_recorded_sweep_leaves_the_state_of_plain_steps(K):
    """The recorded sweep runs its last segment through the rings (K = 4: one step,
    K >= 9: all nine) and hands the end state back to the handle.  The saved state
    (populations, phi in both buffers with their ghosts, velocity, step count)
    must equal that of nine plain steps bit for bit, and so must the state three
    plain steps later."""
    from paper_2607_25444_amd import capi
    shape = (20, 18, 16)
    solid, phi0, theta, target, params = CASES["droplet"](shape)

    def run(record):
        s = capi.Sim(shape, params)
        s.set_geometry(solid, theta)
        s.set_state(phi0)
        if record:
            s.tape_forward(9, K)
        else:
            s.step(9)
        a = s.save_state().cpu().numpy()
        s.step(3)
        b = s.save_state().cpu().numpy()
        s.sync()
        s.close()
        return a, b

    def where(x, y):
        """Sections of the saved state (64-byte header, then float planes) that differ."""
        n = int(np.prod(shape))
        bounds = [("header", 0, 64), ("populations", 64, 64 + 108 * n), ("phi", 64 + 108 * n, 64 + 112 * n),
                  ("phi previous", 64 + 112 * n, 64 + 116 * n), ("u", 64 + 116 * n, 64 + 128 * n),
                  ("p*0", 64 + 128 * n, 64 + 132 * n)]
        return [name for name, lo, hi in bounds if not np.array_equal(x[lo:hi], y[lo:hi])]

    a0, b0 = run(False)
    a1, b1 = run(True)
    assert a0.size == a1.size == 64 + 132 * int(np.prod(shape))
    assert np.array_equal(a0, a1), where(a0, a1)
    assert np.array_equal(b0, b1), where(b0, b1)


@pytest.mark.parametrize("K", [3, 9])
def test_reverse_sweep_can_be_repeated(K):
    """A second reverse sweep of the same recording gives the same bits: with one
    segment (K = 9) the rings still hold it; with several (K = 3) the last
    segment, overwritten by the first sweep, is replayed from its checkpoint."""
    from paper_2607_25444_amd import capi
    shape = (20, 18, 16)
    solid, phi0, theta, target, params = CASES["droplet"](shape)
    s = capi.Sim(shape, params)
    s.set_geometry(solid, theta)
    s.set_state(phi0)
    s.tape_forward(9, K)
    _, seed = s.loss(target)
    out = []
    for _ in range(2):
        dth, dphi0 = s.tape_backward(seed)
        s.sync()
        out.append((dth.cpu().numpy(), dphi0.cpu().numpy()))
    s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.abs(out[0][0]).max() > 0.0


def test_gradient_matches_oracle_finite_differences(orc):
    """dL/dtheta at the wall nodes with the largest gradients against central
    differences of the FP64 C oracle (h = 1e-4 rad)."""
    shape = (24, 20, 16)
    solid, phi0, theta, target, params = CASES["droplet"](shape)
    nsteps, K = 20, 6
    L, dth, _, idx, donor = gpu_grad(shape, solid, phi0, theta, target, params, nsteps, K)
    order = np.argsort(-np.abs(dth))
    sample = list(order[:6]) + list(np.random.default_rng(0).choice(order[:60], 2, replace=False))
    fl = np.asarray(solid).reshape(-1) == 0
    h = 1e-4

    def loss(th):
        s = orc.OracleSim.create(shape, solid, th, orc.Params(**params), phi0)
        s.step(nsteps)
        d = (s.phi - np.asarray(target, np.float64))[fl]
        return 0.5 * float(np.dot(d, d))

    th0 = np.asarray(theta, dtype=np.float64)
    for k in sample:
        tp, tm = th0.copy(), th0.copy()
        tp[idx[k]] += h
        tm[idx[k]] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        print(f"wall node {idx[k]}: adjoint {dth[k]:.6e} fd {fd:.6e}")
        assert abs(dth[k] - fd) <= 1e-3 * abs(fd) + 1e-6 * np.abs(dth).max()


def test_autograd_function_and_entry_points():
    """CACStep.backward equals tape_backward, and cac_adjoint equals the
    tape_forward / loss / tape_backward sequence."""
    import torch
    from paper_2607_25444_amd import capi
    shape = (20, 18, 16)
    solid, phi0, theta, target, params = CASES["blocks-density-gravity"](shape)
    nsteps, K = 8, 3
    L, dth, dphi0, idx, _ = gpu_grad(shape, solid, phi0, theta, target, params, nsteps, K)

    s = capi.Sim(shape, params)
    s.set_geometry(solid, theta)
    th = torch.tensor(np.asarray(theta)[idx], device="cuda", requires_grad=True)
    p0 = torch.tensor(phi0, device="cuda", requires_grad=True)
    tgt = torch.tensor(target, device="cuda")
    fl = torch.tensor(np.asarray(solid).reshape(-1) == 0, device="cuda")
    step = capi.cac_step_function()
    phi = step.apply(th, p0, s, nsteps, K)
    loss = 0.5 * (torch.where(fl, phi - tgt, torch.zeros_like(phi)) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) <= 1e-5 * L
    assert np.allclose(th.grad.cpu().numpy(), dth.astype(np.float32), rtol=0, atol=1e-6 * np.abs(dth).max())
    assert np.array_equal(p0.grad.cpu().numpy(), dphi0.astype(np.float32))

    s.set_contact_angles(th.detach())
    s.set_state(phi0)
    L2, dth2 = s.adjoint(nsteps, K, target)
    assert L2 == L
    assert np.array_equal(dth2.cpu().numpy(), dth)
    s.close()


def test_full_size_gradient_is_deterministic_and_matches_finite_differences(orc):
    """128 x 128 x 64 contact-angle inversion workload (bump angle field):
    two reverse sweeps give the same bits; on the two wall nodes with the
    largest gradient dL/dtheta agrees with central differences of the C oracle."""
    w = W.adjoint_128(seed=0)
    nx, ny, nz = w.shape
    nsteps, K = 12, 5
    # target shape: a slightly wider cap, off the lattice symmetry planes
    target = W.tanh_droplet(w.shape, ((nx - 1) / 2 + 0.6, (ny - 1) / 2 - 0.4, 0.5), 25.0, 4.0).astype(np.float32)
    L, dth, _, idx, _ = gpu_grad(w.shape, w.solid, w.phi0, w.theta, target, w.params, nsteps, K)
    L2, dth2, _, _, _ = gpu_grad(w.shape, w.solid, w.phi0, w.theta, target, w.params, nsteps, K)
    assert L == L2 and np.array_equal(dth, dth2)
    assert np.all(np.isfinite(dth)) and np.abs(dth).max() > 0
    fl = w.solid == 0
    h = 1e-4

    def loss(th):
        o = orc.OracleSim.create(w.shape, w.solid, th, orc.Params(**w.params), w.phi0)
        o.step(nsteps)
        d = (o.phi - target.astype(np.float64))[fl]
        return 0.5 * float(np.dot(d, d))

    th0 = np.asarray(w.theta, dtype=np.float64)
    for k in np.argsort(-np.abs(dth))[:2]:
        tp, tm = th0.copy(), th0.copy()
        tp[idx[k]] += h
        tm[idx[k]] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        print(f"wall node {idx[k]}: adjoint {dth[k]:.6e} fd {fd:.6e}")
        assert abs(dth[k] - fd) <= 1e-3 * abs(fd)
