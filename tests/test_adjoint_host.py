"""The library's hand-written reverse step, run on the CPU.

tests/host_emu/adj_emu.cpp compiles the reverse-step node bodies of libcac
(adjoint_device.hpp) for the host.  Fed with the forward state of each step
(taken from the FP64 literal oracle, rounded to FP32), it must reproduce the
oracle's autograd gradient (dL/dtheta per wall node, dL/dphi at the start of
the window) to FP32 accuracy: 2e-6 of the largest component.  Window of 1 and
3 steps after 3 warm-up steps, on asymmetric states (exact mirror symmetry
puts minmod arguments on a tie, where the gradient is one-sided)."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from paper_2607_25444_amd import capi
from paper_2607_25444_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2607_25444_amd", "csrc")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("emu") / "adj_emu.so")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-fPIC", "-shared",
                    "-I", CSRC, os.path.join(HERE, "host_emu", "adj_emu.cpp"), "-o", out], check=True)
    return C.CDLL(out)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.float32)


def _ptr(a, t=C.c_float):
    return a.ctypes.data_as(C.POINTER(t))


def run_window(emu, shape, solid, phi0, theta_field, params, nwarm, nsteps, seed):
    from oracle import literal as Lt
    nx, ny, nz = shape
    N = nx * ny * nz
    perm = [Lt.C_LIST.index(tuple(c)) for c in Lt._CANON]  # library order -> literal order
    sim = Lt.LiteralSim(shape, solid, params, phi0)
    p = sim.p
    th_w = sim.wall_theta_from_field(theta_field)
    fpost = torch.zeros((27, nz, ny, nx), dtype=torch.float64)
    with torch.no_grad():
        for _ in range(nwarm):
            ph, aw = Lt.ghost_update(p, sim.geo, th_w, sim.phi)
            fpost, fnew, u, _ = Lt.hydro(p, sim.solid, ph, sim.f)
            sim.phi = Lt.volume(p, sim.solid, Lt.phase(p, sim.solid, ph, u, aw), sim.M_target)
            sim.f = fnew
    rng = np.random.default_rng(seed)
    target = torch.as_tensor(np.clip(sim.phi.numpy() + 0.05 * rng.standard_normal(sim.phi.shape), 0, 1))
    phi_start = sim.phi.detach().clone().requires_grad_(True)
    thv = th_w.detach().clone().requires_grad_(True)
    phi, f, fprev, rec = phi_start, sim.f.detach(), fpost.detach(), []
    for _ in range(nsteps):
        ph, aw = Lt.ghost_update(p, sim.geo, thv, phi)
        fp, fnew, u, _ = Lt.hydro(p, sim.solid, ph, f)
        pst = Lt.phase(p, sim.solid, ph, u, aw)
        rec.append((fprev, ph.detach(), phi.detach(), u.detach(), pst.detach()))
        fprev = fp.detach()
        phi, f = Lt.volume(p, sim.solid, pst, sim.M_target), fnew
    fl = ~sim.solid
    L = 0.5 * (torch.where(fl, phi - target, torch.zeros_like(phi)) ** 2).sum()
    gth, gphi = torch.autograd.grad(L, [thv, phi_start])

    solid_u8 = np.ascontiguousarray(np.asarray(solid).reshape(-1), dtype=np.uint8)
    widx, n6, donor = capi.wall_tables(solid_u8, shape)
    assert np.array_equal(widx, sim.wall_linear_index())
    prm = np.array([p["rho_l"], p["rho_g"], p["nu_l"], p["nu_g"], p["sigma"], p["delta"], p["D"], *p["g"],
                    p["eps_phi"], p["eps_n"], p["sin_tol"], p["cot_max"], p["volume_correction"],
                    p["wall_compression"]], dtype=np.float64)
    widx32, n632, don32 = (np.ascontiguousarray(a, dtype=np.int32) for a in (widx, n6, donor))
    theta32 = _f32(thv.detach().numpy())
    pb = _f32(torch.where(fl, phi - target, torch.zeros_like(phi)).detach().numpy().reshape(-1))
    mb = np.zeros(10 * N, np.float32)
    thb = np.zeros(len(widx), np.float64)
    for j in reversed(range(nsteps)):
        fpv, ph, pold, u, pst = rec[j]
        arrs = [_f32(fpv.numpy().reshape(27, -1)[perm].reshape(-1)), _f32(ph.numpy().reshape(-1)),
                _f32(pold.numpy().reshape(-1)), _f32(u.numpy().reshape(-1)), _f32(pst.numpy().reshape(-1))]
        pbo, mbo = np.zeros(N, np.float32), np.zeros(10 * N, np.float32)
        emu.emu_reverse_step(nx, ny, nz, _ptr(prm, C.c_double), _ptr(solid_u8, C.c_uint8), len(widx),
                             _ptr(widx32, C.c_int32), _ptr(n632, C.c_int32), _ptr(don32, C.c_int32), _ptr(theta32),
                             C.c_double(float(sim.M_target)), *[_ptr(a) for a in arrs], _ptr(pb), _ptr(mb),
                             _ptr(pbo), _ptr(mbo), _ptr(thb, C.c_double))
        pb, mb = pbo, mbo
    gth, gphi = gth.numpy(), gphi.numpy().reshape(-1)
    return (np.abs(thb - gth).max() / np.abs(gth).max(), np.abs(pb - gphi).max() / np.abs(gphi).max())


def _cases():
    shape = (12, 11, 10)
    x, y, z = W.grid(shape)
    d = np.sqrt((x - 5.3) ** 2 + (y - 4.8) ** 2 + (z - 0.7) ** 2)
    drop = (0.5 * (1 - np.tanh(2 * (d - 3.5) / 4.0))).reshape(-1)
    rng = np.random.default_rng(7)
    out = {"droplet": (shape, W.flat_walls(shape), drop, rng.uniform(0.7, 2.4, drop.size), W.default_params())}
    for k, pk in ((1, dict(nu_l=0.05, nu_g=0.03, sigma=0.01, wall_compression=1)),
                  (2, dict(rho_l=5.0, nu_l=0.05, nu_g=0.03, sigma=0.01, g=(1e-4, -2e-4, 3e-4), wall_compression=0)),
                  (3, dict(rho_l=5.0, sigma=0.01, g=(0.0, 0.0, -3e-4), volume_correction=0))):
        out[f"blocks{k}"] = (shape, W.random_geometry(shape, seed=k), W.random_smooth_field(shape, seed=k),
                             np.random.default_rng(k).uniform(0.5, 2.6, int(np.prod(shape))), W.default_params(**pk))
    return out


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nsteps", [1, 3])
def test_host_reverse_step_matches_oracle_adjoint(emu, name, nsteps):
    shape, solid, phi0, theta, params = CASES[name]
    eth, eph = run_window(emu, shape, solid, phi0, theta, params, nwarm=3, nsteps=nsteps, seed=1)
    print(f"{name} {nsteps}: rel err dtheta {eth:.2e} dphi {eph:.2e}")
    assert eth <= 2e-6
    assert eph <= 2e-6
