"""GPU (FP32, libcac through its C ABI) against the FP64 oracle.

Tolerances: after one step every field within 2e-6 absolute (phi) or 1e-5 of
its maximum (u, p*, populations); after 200 steps of the 32^3 sessile
droplet max |phi_gpu - phi_oracle| <= 1e-5 and max |u_gpu - u_oracle| <=
1e-4 max |u_oracle| over fluid nodes.  Both sides start from the same FP32
inputs (the oracle widens them to FP64)."""
import numpy as np
import pytest

from paper_2607_25444_amd import workloads as W

pytestmark = pytest.mark.gpu

Q = 27


def _params(w, **kw):
    p = dict(w.params)
    p.update(kw)
    return p


def gpu_run(w, steps, launch=None, **kw):
    from paper_2607_25444_amd import capi
    s = capi.Sim(w.shape, _params(w, **kw))
    if launch:
        s.set_launch(*launch)
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0, w.meta.get("u0"))
    s.step(steps)
    phi, u, ps = s.fields()
    f = s.populations()
    s.sync()
    out = dict(phi=phi.cpu().numpy().astype(np.float64), u=u.cpu().numpy().astype(np.float64),
               pstar=ps.cpu().numpy().astype(np.float64), f=f.cpu().numpy().astype(np.float64),
               volume=s.volume())
    s.close()
    return out


def oracle_run(orc, w, steps, **kw):
    p = orc.Params(**_params(w, **kw))
    u0 = w.meta.get("u0")
    s = orc.OracleSim.create(w.shape, w.solid, w.theta.astype(np.float64), p, w.phi0.astype(np.float64),
                             u0=None if u0 is None else u0.astype(np.float64))
    fpost = np.zeros(Q * w.N)
    if steps:
        s.step(steps, fpost=fpost)
    return dict(phi=s.phi, u=s.u, pstar=s.pstar, f=fpost, M=s.M_target)


def _masks(w, orc):
    fl = w.solid == 0
    idx, _, _ = orc.wall_nodes(w.solid, w.shape)
    wall = np.zeros(w.N, bool)
    wall[idx] = True
    return fl, wall


def _cmp(g, o, w, orc, phi_tol, rel_tol, with_f=True):
    fl, wall = _masks(w, orc)
    N = w.N
    dphi = np.abs(g["phi"] - o["phi"])
    assert dphi[fl].max() <= phi_tol, f"phi fluid {dphi[fl].max():.3e}"
    assert dphi[wall].max() <= phi_tol, f"phi ghosts {dphi[wall].max():.3e}"
    uo, ug = o["u"].reshape(3, N)[:, fl], g["u"].reshape(3, N)[:, fl]
    assert np.abs(ug - uo).max() <= rel_tol * max(np.abs(uo).max(), 1e-12), \
        f"u {np.abs(ug - uo).max():.3e} vs max {np.abs(uo).max():.3e}"
    # p* is the zeroth moment of populations of size ~ max(|p*|, |u|) (f^eq of Eq. (11)),
    # so its FP32 rounding scales with that size
    po, pg = o["pstar"][fl], g["pstar"][fl]
    assert np.abs(pg - po).max() <= rel_tol * max(np.abs(po).max(), np.abs(uo).max(), 1e-4), \
        f"p* {np.abs(pg - po).max():.3e}"
    if with_f:
        fo, fg = o["f"].reshape(Q, N)[:, fl], g["f"].reshape(Q, N)[:, fl]
        assert np.abs(fg - fo).max() <= rel_tol * max(np.abs(fo).max(), 1e-6), \
            f"f {np.abs(fg - fo).max():.3e} vs max {np.abs(fo).max():.3e}"


def _variable_density_case(shape=(20, 12, 14), seed=3):
    solid = W.random_geometry(shape, seed, n_blocks=3)
    nx, ny, nz = shape
    phi0 = W.tanh_droplet(shape, (nx / 2, ny / 2, nz / 2), 4.5, 4.0).astype(np.float32)
    rng = np.random.default_rng(seed)
    theta = np.deg2rad(rng.uniform(30, 150, size=nx * ny * nz)).astype(np.float32)
    prm = W.default_params(rho_l=1.2, rho_g=0.9, nu_l=0.031, nu_g=0.24, sigma=0.025, g=(1e-5, -2e-5, -1e-4))
    return W.Workload("vardens", shape, solid, theta, phi0, prm, 0)


@pytest.mark.parametrize("wc", [0, 1])
def test_one_step_all_fields(orc, wc):
    """One step on a random voxel geometry with per-node angles, density and
    viscosity contrast and a body force: every term of the step is live."""
    w = _variable_density_case()
    o = oracle_run(orc, w, 1, wall_compression=wc)
    g = gpu_run(w, 1, wall_compression=wc)
    _cmp(g, o, w, orc, 2e-6, 1e-5)


@pytest.mark.parametrize("wc", [0, 1])
def test_plain_ghost_extrapolation_reading(orc, wc):
    """The diagnostic reading ghost_localization = 0 (lambda_s = 1 in the ghost
    of Eq. (46)) on the sessile droplet: 1 and 50 steps against the oracle."""
    w = W.sessile_32(60.0)
    fl, wall = _masks(w, orc)
    for steps, tol_phi, tol_rel in ((1, 2e-6, 1e-5), (50, 1e-5, 1e-4)):
        o = oracle_run(orc, w, steps, wall_compression=wc, ghost_localization=0)
        g = gpu_run(w, steps, wall_compression=wc, ghost_localization=0)
        _cmp(g, o, w, orc, tol_phi, tol_rel)
        # another reading: its ghosts differ from those of Eq. (47)
        d = oracle_run(orc, w, steps, wall_compression=wc)
        assert np.abs(d["phi"][wall] - o["phi"][wall]).max() > 1e-3


@pytest.mark.parametrize("steps", [0, 1, 5])
def test_sessile_initial_steps(orc, steps):
    w = W.sessile_32(60.0)
    o = oracle_run(orc, w, steps)
    g = gpu_run(w, steps)
    _cmp(g, o, w, orc, 2e-6, 1e-5, with_f=steps > 0)


@pytest.mark.parametrize("wc", [1, 0])
def test_sessile_200_steps(orc, wc):
    """Static sessile droplet 32^3, theta = 60 deg, 200 steps: phi within 1e-5,
    u within 1e-4 of max|u| (FP32 against FP64)."""
    w = W.sessile_32(60.0)
    o = oracle_run(orc, w, 200, wall_compression=wc)
    g = gpu_run(w, 200, wall_compression=wc)
    fl, wall = _masks(w, orc)
    N = w.N
    dphi = np.abs(g["phi"] - o["phi"])
    print("phi err fluid", dphi[fl].max(), "ghost", dphi[wall].max(), flush=True)
    assert dphi[fl].max() <= 1e-5
    assert dphi[wall].max() <= 1e-5
    uo, ug = o["u"].reshape(3, N)[:, fl], g["u"].reshape(3, N)[:, fl]
    print("u err", np.abs(ug - uo).max(), "max u", np.abs(uo).max())
    assert np.abs(ug - uo).max() <= 1e-4 * np.abs(uo).max()
    assert g["volume"] == pytest.approx(o["M"], rel=1e-6)


@pytest.mark.parametrize("launch", [None, (16, 4, 4, 0, 5), (32, 2, 4, 1, 3), (16, 8, 4, 0, 2), (64, 2, 2, 0, 1),
                                    (128, 2, 1, 0, 6), (32, 4, 4, 0, 4), (256, 2, 1, 0, 1), (512, 1, 1, 1, 3)])
def test_ragged_tiles(orc, launch):
    """A grid that fills no tile exactly (70 x 37 x 19), random solids, 20 steps."""
    shape = (70, 37, 19)
    nx, ny, nz = shape
    solid = W.random_geometry(shape, 11, n_blocks=6)
    phi0 = W.tanh_droplet(shape, (30.2, 17.7, 7.1), 6.0, 4.0).astype(np.float32)
    w = W.Workload("ragged", shape, solid, W.uniform_theta(shape, 75.0), phi0, W.default_params(), 0)
    o = oracle_run(orc, w, 20)
    g = gpu_run(w, 20, launch=launch)
    _cmp(g, o, w, orc, 5e-6, 5e-5)


@pytest.mark.parametrize("launch", [(128, 2, 1, 0, 1), (128, 1, 2, 1, 3)])
def test_row_wide_tiles(orc, launch):
    """A lattice exactly one 128-wide tile across (non-temporal population loads
    in the hardware workgroup order), random solids, 20 steps."""
    shape = (128, 10, 12)
    solid = W.random_geometry(shape, 13, n_blocks=5)
    phi0 = W.tanh_droplet(shape, (60.3, 4.6, 5.2), 5.0, 4.0).astype(np.float32)
    w = W.Workload("row_wide", shape, solid, W.uniform_theta(shape, 70.0), phi0, W.default_params(), 0)
    o = oracle_run(orc, w, 20)
    g = gpu_run(w, 20, launch=launch)
    _cmp(g, o, w, orc, 5e-6, 5e-5)


def test_deterministic_and_graph_replay():
    """Two identical runs are bitwise equal, and graph replay equals eager launches."""
    w = W.sessile((40, 36, 20), 7.0, 110.0)
    a = gpu_run(w, 15, launch=(16, 4, 4, 0))
    b = gpu_run(w, 15, launch=(16, 4, 4, 0))
    c = gpu_run(w, 15, launch=(16, 4, 4, 1))
    for k in ("phi", "u", "f"):
        np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(a[k], c[k])


def test_uniform_state_invariant_gpu():
    """Rest state, constant phi, walls: nothing moves (exact in FP32)."""
    shape = (24, 20, 16)
    N = 24 * 20 * 16
    w = W.Workload("rest", shape, W.random_geometry(shape, 2), W.uniform_theta(shape, 40.0),
                   np.full(N, 0.3, np.float32), W.default_params(), 0)
    g = gpu_run(w, 10)
    fl = w.solid == 0
    assert np.abs(g["phi"][fl] - 0.3).max() < 1e-7
    assert np.abs(g["u"]).max() < 1e-9


def test_volume_conserved_gpu():
    """Phase-field volume after 300 steps equals the initial one up to FP32
    storage rounding of phi."""
    w = W.sessile((48, 48, 24), 9.0, 45.0)
    g = gpu_run(w, 300)
    M0 = float(w.phi0.astype(np.float64)[w.solid == 0].sum())
    assert g["volume"] == pytest.approx(M0, rel=2e-7)


def test_full_size_spreading_one_step(orc):
    """Spreading workload at its full size (256 x 256 x 128), one step: every
    fluid node of phi, u and p* against the oracle, in the launch configuration
    the benchmark uses."""
    from paper_2607_25444_amd import tuning
    w = W.spreading_256(0)
    o = oracle_run(orc, w, 1)
    g = gpu_run(w, 1, launch=tuning.launch_for(w.shape))
    _cmp(g, o, w, orc, 2e-6, 1e-5, with_f=False)


@pytest.mark.parametrize("name", ["orifice", "porous", "impact"])
def test_full_size_one_step(orc, name):
    """The other full-size workloads of the benchmark (orifice 192 x 192 x 768,
    porous packing 256 x 256 x 128, impact 256^3 at density ratio 1000), one
    step: every fluid node of phi, u and p* and every ghost against the oracle,
    in the launch configuration the benchmark uses."""
    from paper_2607_25444_amd import tuning
    w = {"orifice": lambda: W.orifice_192(0), "porous": lambda: W.porous_256(0),
         "impact": lambda: W.impact_256()}[name]()
    print(f"[full size] {w.name} N={w.N}", flush=True)
    o = oracle_run(orc, w, 1)
    g = gpu_run(w, 1, launch=tuning.launch_for(w.shape))
    _cmp(g, o, w, orc, 2e-6, 1e-5, with_f=False)


@pytest.mark.parametrize("name", ["spreading", "porous", "impact"])
def test_full_size_20_steps(orc, name):
    """The full-size workloads besides the orifice (spreading 256 x 256 x 128,
    porous packing 256 x 256 x 128, impact 256^3 at density ratio 1000), 20
    steps in the launch the benchmark uses: phi within 1e-5 and u within 1e-4
    of its maximum on every fluid node, p* and every ghost as well."""
    from paper_2607_25444_amd import tuning
    w = {"spreading": lambda: W.spreading_256(0), "porous": lambda: W.porous_256(0),
         "impact": lambda: W.impact_256()}[name]()
    print(f"[full size] {w.name} N={w.N}, 20 steps", flush=True)
    o = oracle_run(orc, w, 20)
    g = gpu_run(w, 20, launch=tuning.launch_for(w.shape))
    fl, wall = _masks(w, orc)
    N = w.N
    dphi = np.abs(g["phi"] - o["phi"])
    uo, ug = o["u"].reshape(3, N)[:, fl], g["u"].reshape(3, N)[:, fl]
    print("phi err fluid", dphi[fl].max(), "ghost", dphi[wall].max(), "u err", np.abs(ug - uo).max(),
          "max u", np.abs(uo).max(), flush=True)
    _cmp(g, o, w, orc, 1e-5, 1e-4, with_f=False)


def test_scaled_orifice_200_steps(orc):
    """The orifice workload scaled down (48 x 48 x 96, plate 4 cells thick with
    a hole of diameter 12, droplet R = 10 just above it, the paper's orifice
    fluids, g = 2e-4 so that the drop moves within the run, angle 110
    degrees): 200 steps with F_p, F_nu and F_ext live, phi within 1e-5 and u
    within 1e-4 of its maximum."""
    shape = (48, 48, 96)
    nx, ny, nz = shape
    solid = W.orifice_plate_mask(shape, 46, 4, 12.0)
    phi0 = W.tanh_droplet(shape, ((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, 49.5 + 2.0 + 10.0), 10.0, 6.0)
    prm = W.default_params(rho_l=1.2, rho_g=0.9, nu_l=0.031, nu_g=0.24, sigma=0.025, delta=6.0,
                           g=(0.0, 0.0, -2e-4))
    w = W.Workload("orifice_48x48x96", shape, solid, W.uniform_theta(shape, 110.0), phi0.astype(np.float32), prm, 200)
    o = oracle_run(orc, w, 200)
    g = gpu_run(w, 200)
    fl, wall = _masks(w, orc)
    N = w.N
    dphi = np.abs(g["phi"] - o["phi"])
    uo, ug = o["u"].reshape(3, N)[:, fl], g["u"].reshape(3, N)[:, fl]
    print("phi err fluid", dphi[fl].max(), "ghost", dphi[wall].max(), "u err", np.abs(ug - uo).max(),
          "max u", np.abs(uo).max(), flush=True)
    assert np.abs(uo).max() > 1e-3  # the drop falls and deforms
    _cmp(g, o, w, orc, 1e-5, 1e-4, with_f=False)


def test_full_size_orifice_20_steps(orc):
    """The benchmark workload, orifice 192 x 192 x 768 (density and viscosity
    contrast, body force: F_p, F_nu and F_ext live), 20 steps in the launch the
    benchmark times: phi within 1e-5 and u within 1e-4 of its maximum on every
    fluid node, p* and every ghost as well."""
    from paper_2607_25444_amd import tuning
    w = W.orifice_192(0)
    print(f"[full size] {w.name} N={w.N}, 20 steps", flush=True)
    o = oracle_run(orc, w, 20)
    g = gpu_run(w, 20, launch=tuning.launch_for(w.shape))
    fl, wall = _masks(w, orc)
    dphi = np.abs(g["phi"] - o["phi"])
    N = w.N
    uo, ug = o["u"].reshape(3, N)[:, fl], g["u"].reshape(3, N)[:, fl]
    print("phi err fluid", dphi[fl].max(), "ghost", dphi[wall].max(), "u err", np.abs(ug - uo).max(),
          "max u", np.abs(uo).max(), flush=True)
    _cmp(g, o, w, orc, 1e-5, 1e-4, with_f=False)


def test_512_cubed_lattice():
    """The paper's 512^3 spreading lattice (27 N above 2^31: population indices
    use the full unsigned 32-bit range): two steps in the launch the benchmark
    uses (256 x 2 tiles, ordinary loads) and in row-wide 512 x 1 tiles
    (non-temporal loads, hardware workgroup order) agree on every node
    (the per-node arithmetic is the same; only the FP64 order of the volume
    sums differs), stay finite and keep the phase-field volume."""
    from paper_2607_25444_amd import capi, tuning
    w = W.spreading_512()
    assert 27 * w.N > 2 ** 31
    fl = w.solid == 0
    M0 = float(w.phi0.astype(np.float64)[fl].sum())
    out = []
    for launch in (tuning.launch_for(w.shape), (512, 1, 1, 0, 0)):
        print(f"[512^3] launch {launch}", flush=True)
        s = capi.Sim(w.shape, w.params)
        s.set_launch(*launch)
        s.set_geometry(w.solid, w.theta)
        s.set_state(w.phi0)
        s.step(2)
        phi, u, _ = s.fields()
        vol = s.volume()
        s.sync()
        out.append((phi.cpu().numpy(), u.cpu().numpy(), vol))
        s.close()
        del phi, u
    (pa, ua, va), (pb, ub, vb) = out
    assert np.isfinite(pa).all() and np.isfinite(ua).all()
    assert np.abs(pa - pb)[fl].max() <= 2e-6
    assert np.abs(ua - ub).max() <= 2e-5 * max(np.abs(ua).max(), 1e-9)
    assert va == pytest.approx(M0, rel=2e-7) and vb == pytest.approx(M0, rel=2e-7)


def test_watchdog_reports_non_finite_values():
    """A NaN forced into the initial phase field, and a velocity too large for
    the collision, raise CAC_ERR_NONFINITE at the next synchronising call."""
    from paper_2607_25444_amd import capi
    w = W.sessile((24, 20, 16), R=5.0, theta_deg=60.0)
    fl = np.flatnonzero(w.solid == 0)
    phi = w.phi0.copy()
    phi[fl[len(fl) // 2]] = np.nan
    s = capi.Sim(w.shape, w.params)
    s.set_geometry(w.solid, w.theta)
    s.set_state(phi)
    s.step(1)
    with pytest.raises(capi.CacError) as e:
        s.sync()
    assert e.value.status == capi.CAC_ERR_NONFINITE
    u0 = np.zeros(3 * w.N, np.float32)
    u0[fl] = 1e30
    s.set_state(w.phi0, u0)
    s.step(2)
    with pytest.raises(capi.CacError) as e:
        s.volume()
    assert e.value.status == capi.CAC_ERR_NONFINITE
    # a clean state clears the flag
    s.set_state(w.phi0)
    s.step(2)
    s.sync()
    s.close()
