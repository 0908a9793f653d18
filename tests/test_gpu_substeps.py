"""Per-substep parity (GPU through the C ABI test hooks against the FP64
oracle's substep functions) and checkpoint / resume.

Each substep of one step is run alone on the GPU (cac_debug_substep) and its
output buffer compared with the oracle's function for that substep, the oracle
chaining its own outputs (no oracle input comes from the GPU):
  W ghosts and wall compressive flux (Sec. II B), H post-collision populations
  and velocity (Sec. II A), P phase field before the correction (Sec. II A 1),
  V corrected phase field (Sec. II C).
Inputs: random blocks on flat walls, smooth random phase field, velocity and
p*, random angles per node, density contrast and gravity.  Bound: 1e-6 absolute
on phase-field values and 1e-6 of the field maximum on populations and
velocity (FP32 rounding of one substep)."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu

Q = 27


def _inputs(shape, seed, **pkw):
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    solid = W.random_geometry(shape, seed=seed)
    phi0 = W.random_smooth_field(shape, seed=seed).astype(np.float32)
    u0 = np.concatenate([0.03 * (W.random_smooth_field(shape, seed=seed + 10 + d) - 0.5) for d in range(3)])
    u0 = u0.astype(np.float32)
    ps0 = (0.01 * W.random_smooth_field(shape, seed=seed + 20)).astype(np.float32)
    theta = rng.uniform(0.6, 2.5, N).astype(np.float32)
    params = W.default_params(**pkw)
    return solid, phi0, u0, ps0, theta, params


@pytest.mark.parametrize("wc", [1, 0])
def test_each_substep_matches_the_oracle(orc, wc):
    from paper_2607_25444_amd import capi
    shape = (24, 20, 18)
    solid, phi0, u0, ps0, theta, params = _inputs(shape, 5 + wc, rho_l=3.0, nu_l=0.05, nu_g=0.03, sigma=0.01,
                                                  g=(0.0, 2e-5, -4e-5), wall_compression=wc)
    N = int(np.prod(shape))
    fl = np.asarray(solid).reshape(-1) == 0
    P = orc.Params(**params)
    o = orc.OracleSim.create(shape, solid, theta, P, phi0, pstar0=ps0, u0=u0)
    s = capi.Sim(shape, params)
    s.set_geometry(solid, theta)
    s.set_state(phi0, u0, ps0)

    # W
    s.debug_substep(0)
    ph_g = s.debug_buffer(0).cpu().numpy().astype(np.float64)
    aw_g = s.debug_buffer(5).cpu().numpy().astype(np.float64)
    ph_o, aw_o = orc.ghost(P, shape, solid, theta, o.phi, with_flux=True)
    e_w = np.abs(ph_g - ph_o).max()
    e_a = np.abs(aw_g - aw_o).max()
    # H
    s.debug_substep(1)
    fp_g = s.debug_buffer(4).cpu().numpy().astype(np.float64).reshape(Q, N)
    u_g = s.debug_buffer(2).cpu().numpy().astype(np.float64).reshape(3, N)
    fp_o, _, u_o, _ = orc.hydro(P, shape, solid, ph_o, o.f)
    fp_o = fp_o.reshape(Q, N)
    u_o = u_o.reshape(3, N)
    e_f = np.abs(fp_g - fp_o)[:, fl].max() / np.abs(fp_o[:, fl]).max()
    e_u = np.abs(u_g - u_o)[:, fl].max() / np.abs(u_o[:, fl]).max()
    # P
    s.debug_substep(2)
    pst_g = s.debug_buffer(1).cpu().numpy().astype(np.float64)
    pst_o = orc.phase(P, shape, solid, ph_o, u_o.reshape(-1), a_wall=aw_o)
    e_p = np.abs(pst_g - pst_o)[fl].max()
    # cac_step is refused in the middle of a step
    with pytest.raises(capi.CacError):
        s.step(1)
    # V
    s.debug_substep(3)
    phi_g = s.fields()[0].cpu().numpy().astype(np.float64)
    phi_o, lam = orc.volume(P, shape, solid, pst_o, orc.mass(shape, solid, phi0))
    e_v = np.abs(phi_g - phi_o)[fl].max()
    s.sync()
    print(f"wc={wc}: W {e_w:.2e} a {e_a:.2e} H f {e_f:.2e} u {e_u:.2e} P {e_p:.2e} V {e_v:.2e} (lambda {lam:.3e})")
    assert e_w <= 1e-6
    assert e_a <= 1e-6
    assert e_f <= 1e-6
    assert e_u <= 1e-6
    assert e_p <= 1e-6
    assert e_v <= 1e-6
    # out of order
    with pytest.raises(capi.CacError):
        s.debug_substep(2)
    s.close()


def test_save_and_load_resume_bit_for_bit():
    from paper_2607_25444_amd import capi
    shape = (24, 20, 18)
    solid, phi0, u0, ps0, theta, params = _inputs(shape, 9, rho_l=2.0, g=(0.0, 0.0, -3e-5))

    fl = np.asarray(solid).reshape(-1) == 0

    def snapshot(s):
        # populations are defined on fluid nodes only
        phi, u, ps = s.fields()
        f = s.populations()
        s.sync()
        return [t.cpu().numpy() for t in (phi, u, ps)] + [f.cpu().numpy().reshape(27, -1)[:, fl]]

    s = capi.Sim(shape, params)
    s.set_geometry(solid, theta)
    s.set_state(phi0, u0, ps0)
    s.step(7)
    buf = s.save_state()
    s.step(9)
    a = snapshot(s)
    s.load_state(buf)
    s.step(9)
    b = snapshot(s)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # a second handle with the same geometry resumes from the same buffer
    t = capi.Sim(shape, params)
    t.set_geometry(solid, theta)
    t.load_state(buf)
    t.step(9)
    c = snapshot(t)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)
    # a buffer of the wrong size is refused
    with pytest.raises(capi.CacError):
        t.load_state(buf[:100])
    s.close()
    t.close()
