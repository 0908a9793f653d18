#!/usr/bin/env python3
"""Throughput of the coupled CAC lattice Boltzmann wetting step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload orifice]

Workload (N = 1): the gravity-driven passage through a sharp-edged orifice,
192 x 192 x 768 lattice (28.3 M nodes), plate 8 cells thick with a hole of
diameter 48, droplet R = 40, density and viscosity contrast (1.2/0.9,
0.031/0.24) and a body force, FP32 state, seed 0 (synthetic input, see
paper_2607_25444_amd/workloads.py): the largest plain-step lattice and the
one where every force term of the step is live.  Inputs are resident in HBM
before the timed region; K steps are timed with HIP events on the stream the
library launches on, bracketed by device synchronisation.  Prints one JSON
line:
  value      fluid-node MLUPS of the plain step (whole job, one GPU)
  roofline   the dominant kernel (hydrodynamic collide-stream) against the
             HBM peak: algorithmic bytes (27 populations read and written +
             phi read = 220 B per fluid node) x fluid nodes / its average launch
             time, timed live with per-kernel HIP events; `step` gives the
             whole step against the same peak (224 B per fluid node)
  spreading  the same for the 256 x 256 x 128 spreading workload
  r1, batched, adjoint   the gradient-form collision, the 64-domain batch and
             the reverse-mode sweep, each beside the plain step
  adjoint_resident   the same reverse-mode sweep with the whole rollout kept in
             HBM (one segment, no replay), when the device has the room
  cpu_baseline  the FP64 oracle timed on the host on a bounded sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HYDRO_BYTES_PER_LU = 27 * 4 * 2 + 4
STEP_BYTES_PER_LU = 28 * 4 * 2
METRIC = "MLUPS and % HBM roofline, 1 MI355X: plain vs batched vs adjoint step"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


HYDRO_SOURCES = ("kernels.hip", "step_device.hpp", "cac_internal.hpp")


def kernel_source_hash():
    """sha256[:16] over the sources that define the hydrodynamic kernel."""
    h = hashlib.sha256()
    for name in HYDRO_SOURCES:
        with open(os.path.join(ROOT, "paper_2607_25444_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, key="bytes_per_launch"):
    """HBM bytes per hydro launch (key "bytes_per_launch") or per whole step
    (key "step_bytes") from the committed rocprofv3 counter summary for this
    workload, if there is one and it was taken on the current kernel source;
    else None."""
    p = os.path.join(ROOT, "profiles", f"hydro_traffic_{workload_name}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("workload") != workload_name or d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get(key)


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps, W, capi=None, launch=None):
    """The FP64 oracle on the host: `steps` steps of the benchmark workload on
    all threads, and one step of the 256x256x128 spreading workload on one
    thread (a bounded sample each).  With the GPU binding given, the oracle's
    state after those steps is also the accuracy gate of the benchmark: the
    GPU path runs the same steps from the same state in the benchmark's launch
    and must agree on every fluid node (phi within 1e-5, u within 1e-4 of
    its maximum)."""
    import numpy as np
    import oracle

    def timed(wl, n):
        p = oracle.Params(**wl.params)
        s = oracle.OracleSim.create(wl.shape, wl.solid, wl.theta.astype(np.float64), p, wl.phi0.astype(np.float64),
                                    u0=wl.meta.get("u0"))
        t0 = time.perf_counter()
        s.step(n)
        return time.perf_counter() - t0, s

    threads = oracle.num_threads()
    dt, o = timed(w, steps)
    rec = dict(value=round(w.n_fluid * steps / dt / 1e6, 4), unit="MLUPS", cores=threads, kind="oracle",
               sample=f"{steps} full steps of the {w.name} workload ({w.n_fluid} fluid nodes), FP64, "
                      f"{dt:.1f} s wall on {threads} threads")
    if capi is not None:
        sim = capi.Sim(w.shape, w.params)
        sim.set_launch(*launch)
        sim.set_geometry(w.solid, w.theta)
        sim.set_state(w.phi0, w.meta.get("u0"))
        sim.step(steps)
        phi, u, _ = sim.fields()
        phi, u = phi.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64)
        sim.sync()
        sim.close()
        fl = w.solid.reshape(-1) == 0
        uo, ug = o.u.reshape(3, -1)[:, fl], u.reshape(3, -1)[:, fl]
        dphi = float(np.abs(phi[fl] - o.phi.reshape(-1)[fl]).max())
        du = float(np.abs(ug - uo).max() / max(np.abs(uo).max(), 1e-30))
        rec["gate"] = dict(steps=steps, max_abs_dphi=dphi, bound_phi=1e-5, max_rel_du=du, bound_u=1e-4,
                           passed=bool(dphi <= 1e-5 and du <= 1e-4))
    del o
    ws = W.spreading_256(0)
    oracle.set_threads(1)
    dt1, _ = timed(ws, 1)
    oracle.set_threads(threads)
    rec.update(value_1core=round(ws.n_fluid / dt1 / 1e6, 4),
               sample_1core=f"1 full step of the {ws.name} workload ({ws.n_fluid} fluid nodes) on 1 thread, "
                            f"{dt1:.1f} s wall",
               cpu_model=host_cpu_model(), nproc=os.cpu_count())
    return rec


def workload_of(W, name, seed):
    return {"spreading": lambda: W.spreading_256(seed), "orifice": lambda: W.orifice_192(seed),
            "porous": lambda: W.porous_256(seed), "impact": lambda: W.impact_256(),
            "spreading512": lambda: W.spreading_512(), "sessile": lambda: W.sessile_32(60.0)}[name]()


def plain_block(torch, capi, w, launch, steps, warmup, probes):
    """Plain step on workload w: `steps` steps timed with HIP events on the
    library's stream after `warmup` untimed ones, then per-kernel times (HIP
    events around every kernel) and, with probes, the live bandwidth ceilings."""
    sim = capi.Sim(w.shape, w.params)
    sim.set_launch(*launch)
    sim.set_geometry(w.solid, w.theta)
    sim.set_state(w.phi0, w.meta.get("u0"))
    M0 = sim.volume()
    sim.step(warmup)
    sim.sync()
    stream = sim.stream
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    sim.sync()
    ms_step = ms / max(steps, 1)
    kp = min(steps, 100)
    kavg = [v / kp for v in sim.profile_step(kp)]
    M1 = sim.volume()
    hydro_gbs = w.n_fluid * HYDRO_BYTES_PER_LU / (kavg[1] * 1e-3) / 1e9
    step_gbs = w.n_fluid * STEP_BYTES_PER_LU / (ms_step * 1e-3) / 1e9
    out = {
        "workload": w.name, "fluid_nodes": w.n_fluid, "launch": list(launch), "steps": steps,
        "ms_per_step": round(ms_step, 5), "value": round(w.n_fluid / (ms_step * 1e-3) / 1e6, 2), "unit": "MLUPS",
        "kernel_ms": {"W": round(kavg[0], 5), "H": round(kavg[1], 5), "P": round(kavg[2], 5), "V": round(kavg[3], 5)},
        "hydro_algorithmic_GBs": round(hydro_gbs, 1),
        "wall_nodes": sim.nwall,
        "step": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "bytes_per_lu": STEP_BYTES_PER_LU,
            "algorithmic_GBs": round(step_gbs, 1),
            "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4),
            "kernel_ms": {"W": round(kavg[0], 5), "H": round(kavg[1], 5), "P": round(kavg[2], 5),
                          "V": round(kavg[3], 5)},
            "mlups_all_nodes": round(w.N / (ms_step * 1e-3) / 1e6, 2),
            "volume_rel_drift": (M1 - M0) / M0,
        },
    }
    # measured HBM bytes of the whole step (W, H, P and V, rocprofv3 FETCH_SIZE + WRITE_SIZE), when the committed
    # counters match the kernel source
    sbytes = measured_traffic(w.name, "step_bytes")
    out["step"]["measured_bytes_per_step"] = sbytes
    out["step"]["measured_GBs"] = round(sbytes / (ms_step * 1e-3) / 1e9, 1) if sbytes else None
    out["step"]["measured_frac_of_peak"] = round(sbytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if sbytes else None
    if probes:
        # achievable ceilings, measured live after the timed region: the
        # collide-stream's memory access pattern without its arithmetic (27-plane
        # pull copy, 216 B per node over all nodes; leaves the handle without a
        # state) and a plain 1 GiB streaming copy
        pull_ms = sim.pull_copy_probe(20)
        pull_gbs = w.N * 216 / (pull_ms * 1e-3) / 1e9
        copy_gbs = copy_probe(torch, reps=10, quiet=True)
        out["ceilings"] = {"pull_copy_GBs": round(pull_gbs, 1), "pull_copy_ms": round(pull_ms, 5),
                           "plain_copy_GBs": round(copy_gbs, 1),
                           "hydro_algorithmic_over_pull_copy": round(hydro_gbs / pull_gbs, 4)}
        log(f"[bench] ceilings: pull copy {pull_gbs:.0f} GB/s ({pull_ms:.4f} ms), plain copy {copy_gbs:.0f} GB/s")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def copy_probe(torch, nbytes=1 << 30, reps=20, quiet=False):
    """Elementwise copy of nbytes (read nbytes, write nbytes) with torch's
    streaming kernel; returns (and unless quiet prints as JSON) the GB/s."""
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    if not quiet:
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": round(ms, 4),
                          "GBs": round(gbs, 1)}), flush=True)
    del src, dst
    return gbs


def bench_batch(torch, capi, W, steps, warmup, seed, singles=True, tune_cache=None):
    """Batched persistent step over 64 droplet domains (edges from {32,48,64,96,128},
    R = L/4, angle in [30, 150]); autotuned schedule, graph replay."""
    from paper_2607_25444_amd import tuning

    ws = W.batch_domains(seed)
    t0 = time.perf_counter()
    b = capi.Batch(ws)
    t_init = time.perf_counter() - t0
    ndom, ntot, nfl = b.info()
    tune_ms = b.autotune(tune_cache, trial_steps=6)
    sched = b.schedule()
    b.step(warmup)
    b.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    b.sync()
    kms = [v / 20 for v in b.profile_step(20)]
    vols = b.volumes()
    b.close()
    del b
    out = {"workload": f"{ndom} domains, edges {sorted(set(w.shape[0] for w in ws))}", "domains": ndom,
           "nodes": ntot, "fluid_nodes": nfl, "steps": steps, "ms_per_step": round(ms, 5),
           "value": round(nfl / (ms * 1e-3) / 1e6, 2), "unit": "MLUPS",
           "algorithmic_frac_of_peak": round(nfl * STEP_BYTES_PER_LU / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "schedule": {"hydro_tile": list(sched[:3]), "phase_tile": sched[3], "grid_mult": sched[4],
                        "order": sched[5], "graph": sched[6]},
           "autotune_best_ms": round(tune_ms, 5), "init_s": round(t_init, 2),
           "kernel_ms": {"W": round(kms[0], 5), "H": round(kms[1], 5), "P": round(kms[2], 5), "V": round(kms[3], 5)}}
    if singles:
        # the same domains advanced one after another, each by its own single-lattice handle
        tot = 0.0
        for w in ws:
            sim = capi.Sim(w.shape, w.params)
            sim.set_launch(*tuning.launch_for(w.shape))
            sim.set_geometry(w.solid, w.theta)
            sim.set_state(w.phi0)
            sim.step(3)
            sim.sync()
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(sim.stream)
            sim.step(20)
            a1.record(sim.stream)
            torch.cuda.synchronize()
            tot += a0.elapsed_time(a1) / 20
            sim.close()
        out["singles_ms_per_step"] = round(tot, 5)
        out["speedup_vs_singles"] = round(tot / ms, 3)
    return out


# Gradient-form hydrodynamic substep (two kernels): the rebuild pass reads the
# record (p*, a, omega: 20 B) and the velocity (12 B) and writes the 27
# post-collision populations (108 B); the stream pass reads the populations
# (108 B) and phi (4 B) and writes the record (20 B) and the velocity (12 B).
R1_HYDRO_BYTES_PER_LU = (5 + 3 + 27) * 4 + (27 + 1 + 5 + 3) * 4


def bench_r1(torch, capi, w, launch, steps, warmup):
    """The same workload with the gradient-form collision (collision = 1: no
    populations stored, Eq. (15) from the velocity field), timed like the plain
    step."""
    prm = dict(w.params)
    prm["collision"] = 1
    sim = capi.Sim(w.shape, prm)
    sim.set_launch(*launch)
    sim.set_geometry(w.solid, w.theta)
    sim.set_state(w.phi0, w.meta.get("u0"))
    sim.step(warmup)
    sim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sim.sync()
    kp = min(steps, 100)
    kavg = [v / kp for v in sim.profile_step(kp)]
    sim.close()
    achieved = w.n_fluid * R1_HYDRO_BYTES_PER_LU / (kavg[1] * 1e-3) / 1e9
    return {"path": "collision = 1 (gradient-form A2, moment-only state)", "steps": steps,
            "ms_per_step": round(ms, 5), "value": round(w.n_fluid / (ms * 1e-3) / 1e6, 2), "unit": "MLUPS",
            "kernel_ms": {"W": round(kavg[0], 5), "H": round(kavg[1], 5), "P": round(kavg[2], 5),
                          "V": round(kavg[3], 5)},
            "hydro_bytes_per_lu": R1_HYDRO_BYTES_PER_LU, "hydro_algorithmic_GBs": round(achieved, 1),
            "hydro_frac_of_peak": round(achieved / HBM_PEAK_GBS, 4)}


def bench_adjoint(torch, capi, tuning, W, steps, K, seed):
    """Reverse-mode sweep on the contact-angle inversion workload (128 x 128 x 64,
    bump angle field): cac_tape_forward (steps, checkpoints every K) + loss +
    cac_tape_backward, timed with HIP events on the library's stream, beside
    the plain step on the same lattice."""
    w = W.adjoint_128(seed)
    nx, ny, nz = w.shape
    launch = tuning.launch_for(w.shape)
    target = W.tanh_droplet(w.shape, ((nx - 1) / 2 + 0.6, (ny - 1) / 2 - 0.4, 0.5), 25.0, 4.0).astype("float32")
    sim = capi.Sim(w.shape, w.params)
    sim.set_launch(*launch)
    sim.set_geometry(w.solid, w.theta)
    stream = sim.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # plain step on the same lattice
    sim.set_state(w.phi0)
    sim.step(20)
    sim.sync()
    ev[0].record(stream)
    sim.step(steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    plain_ms = ev[0].elapsed_time(ev[1])
    # warm-up sweep (allocates checkpoints and rings)
    mem_before = torch.cuda.memory_allocated()
    sim.set_state(w.phi0)
    sim.tape_forward(steps, K)
    _, seed_t = sim.loss(target)
    sim.tape_backward(seed_t, want_phi0=False)
    sim.sync()
    mem0 = torch.cuda.memory_allocated()
    # timed sweep
    sim.set_state(w.phi0)
    sim.sync()
    ev[0].record(stream)
    sim.tape_forward(steps, K)
    ev[1].record(stream)
    L, seed_t = sim.loss(target)
    ev[2].record(stream)
    dth, _ = sim.tape_backward(seed_t, want_phi0=False)
    ev[3].record(stream)
    torch.cuda.synchronize()
    sim.sync()
    fwd_ms = ev[0].elapsed_time(ev[1])
    bwd_ms = ev[2].elapsed_time(ev[3])
    tot_ms = ev[0].elapsed_time(ev[3])
    n = w.n_fluid * steps
    out = {
        "workload": w.name,
        "steps": steps,
        "K": K,
        "launch": list(launch),
        "value": round(n / (tot_ms * 1e-3) / 1e6, 2),
        "unit": "MLUPS (forward record + reverse sweep, per step of the rollout)",
        "ms_per_step": round(tot_ms / steps, 5),
        "ms_per_step_forward_record": round(fwd_ms / steps, 5),
        "ms_per_step_reverse": round(bwd_ms / steps, 5),
        "plain_mlups_same_lattice": round(n / (plain_ms * 1e-3) / 1e6, 2),
        "ratio_to_plain": round(plain_ms / tot_ms, 4),
        "loss": L,
        "max_abs_dL_dtheta": float(dth.abs().max().item()),
        "tape_bytes": int(mem0 - mem_before),
    }
    sim.close()
    return out


def angle_study(args):
    """Static contact-angle test of Sec. III A on the GPU path: a droplet of
    radius R0 whose centre sits cz above the bottom solid layer (a cap at about
    90 degrees) relaxes on a flat wall (rho = 1, nu = 0.04, sigma = 0.02) until
    the fitted angle is stationary; the angle is measured by a sphere fit of
    the phi = 1/2 surface and by the paper's circle fit in the central xz plane
    (Eqs. (56)-(57)), both with the wall at z_w = 1/2.  Prints one JSON line per
    measurement and one per run."""
    import numpy as np
    import torch
    from paper_2607_25444_amd import capi
    from paper_2607_25444_amd import tuning
    from paper_2607_25444_amd import workloads as W
    from tests import diagnostics as dg

    shape = tuple(int(v) for v in args.angle_shape.split(","))
    nx, ny, nz = shape
    angles = [float(a) for a in args.angles.split(",")]
    readings = [(int(r), int(l)) for r in args.wall_compression.split(",")
                for l in args.ghost_localization.split(",")]
    solid = W.flat_walls(shape)
    centre = ((nx - 1) / 2, (ny - 1) / 2, args.angle_cz)
    phi_sphere = W.tanh_droplet(shape, centre, args.angle_R, args.delta).astype(np.float32)
    vol0 = float(phi_sphere[solid == 0].astype(np.float64).sum())
    launch = tuning.launch_for(shape)
    rows = []
    for wc, gl in readings:
        for th in angles:
            prm = W.default_params(delta=args.delta, D=args.D, wall_compression=wc, ghost_localization=gl,
                                   nu_l=args.nu, nu_g=args.nu, sigma=0.02)
            if args.angle_init == "cap":
                # spherical cap meeting the wall (z_w = 1/2) at the imposed angle, with the
                # liquid volume of the paper's initial droplet
                ct = np.cos(np.deg2rad(th))
                Rc = (3.0 * vol0 / (np.pi * (2.0 - 3.0 * ct + ct ** 3))) ** (1.0 / 3.0)
                phi0 = W.tanh_droplet(shape, (centre[0], centre[1], 0.5 - Rc * ct), Rc,
                                      args.delta).astype(np.float32)
            else:
                phi0 = phi_sphere
            slices = []
            sim = capi.Sim(shape, prm)
            sim.set_launch(*launch)
            sim.set_geometry(solid, W.uniform_theta(shape, th))
            sim.set_state(phi0)
            M0 = sim.volume()
            t0 = time.perf_counter()
            hist, steps, status = [], 0, "max_steps"
            while steps < args.angle_steps:
                sim.step(args.angle_every)
                steps += args.angle_every
                try:
                    sim.sync()
                except capi.CacError as e:
                    status = f"non-finite after {steps} steps"
                    break
                phi, u, _ = sim.fields()
                ph = phi.cpu().numpy().astype(np.float64)
                umax = float(u.abs().max().item())
                fluid = ph[solid == 0]
                if fluid.max() < 0.5:
                    status = "no liquid left"
                    break
                try:
                    a_sph, c, Rf = dg.contact_angle_sphere(ph, shape)
                    a_sec = dg.contact_angle_section(ph, shape, ny // 2)
                except Exception:  # no interface near the wall any more (detached drop)
                    status = f"fit failed after {steps} steps"
                    break
                zlow = dg.liquid_floor(ph, shape)
                hist.append(a_sph)
                if args.angle_dump:
                    slices.append(ph.reshape(nz, ny, nx)[:, ny // 2, :].astype(np.float32))
                print(json.dumps({"angle_study": "progress", "wall_compression": wc, "ghost_localization": gl,
                                  "theta_imposed": th,
                                  "steps": steps, "theta_sphere": round(a_sph, 3), "theta_section": round(a_sec, 3),
                                  "fit_R": round(float(Rf), 3), "fit_z0": round(float(c[2]), 3),
                                  "liquid_floor_z": zlow, "umax": umax}), flush=True)
                if zlow > 1:
                    status = f"detached after {steps} steps"
                    break
                if (steps >= args.angle_min_steps and len(hist) >= 3 and
                        max(hist[-3:]) - min(hist[-3:]) < args.angle_tol):
                    status = "stationary"
                    break
            M1 = sim.volume() if status != "non-finite" and not status.startswith("non-finite") else float("nan")
            row = {"angle_study": "result", "shape": list(shape), "R0": args.angle_R, "cz": args.angle_cz,
                   "init": args.angle_init, "delta": args.delta, "D": args.D, "nu": args.nu, "wall_compression": wc,
                   "ghost_localization": gl, "theta_imposed": th,
                   "theta_sphere": round(hist[-1], 3) if hist else None,
                   "theta_section": round(a_sec, 3) if hist else None,
                   "steps": steps, "status": status, "volume_rel_drift": (M1 - M0) / M0,
                   "wall_s": round(time.perf_counter() - t0, 1)}
            rows.append(row)
            print(json.dumps(row), flush=True)
            if args.angle_dump and slices:
                os.makedirs(args.angle_dump, exist_ok=True)
                np.savez_compressed(os.path.join(args.angle_dump, f"xz_wc{wc}_gl{gl}_th{int(th)}.npz"),
                                    slices=np.stack(slices), every=args.angle_every)
            sim.close()
            del sim
            torch.cuda.empty_cache()
    return rows


def rt_log(args):
    """Wetted radius of the short-time spreading workload (Sec. III B):
    r = sqrt(sum of phi over the first fluid layer / pi) every `every` steps,
    against t* = t / tau_i with tau_i = sqrt(rho R0^3 / sigma).  One JSON line
    per sample."""
    import torch
    from paper_2607_25444_amd import capi
    from paper_2607_25444_amd import tuning
    from paper_2607_25444_amd import workloads as W
    from tests import diagnostics as dg

    w = W.spreading_256(args.seed)
    R0 = 40.0
    tau = (w.params["rho_l"] * R0 ** 3 / w.params["sigma"]) ** 0.5
    sim = capi.Sim(w.shape, w.params)
    sim.set_launch(*tuning.launch_for(w.shape))
    sim.set_geometry(w.solid, w.theta)
    sim.set_state(w.phi0)
    steps = 0
    while True:
        phi, _, _ = sim.fields()
        r = dg.wetted_radius(phi.cpu().numpy(), w.shape)
        print(json.dumps({"rt_log": w.name, "theta_deg": w.meta.get("theta_deg"), "nu": w.params["nu_l"],
                          "step": steps, "t_star": round(steps / tau, 5), "r": round(r, 4),
                          "r_over_R0": round(r / R0, 5)}), flush=True)
        if steps >= args.rt_steps:
            break
        sim.step(args.rt_every)
        steps += args.rt_every
    sim.sync()
    sim.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="orifice",
                    choices=["spreading", "orifice", "porous", "impact", "spreading512", "sessile"])
    ap.add_argument("--no-spreading", action="store_true", help="skip the 256x256x128 spreading block")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None, help="bx,by,bz,graph,phase_tile")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=1000)
    ap.add_argument("--adjoint-K", type=int, default=50)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-adjoint-resident", action="store_true",
                    help="skip the adjoint run that keeps the whole rollout in HBM (K = adjoint steps)")
    ap.add_argument("--r1-steps", type=int, default=200)
    ap.add_argument("--no-r1", action="store_true", help="skip the gradient-form collision (collision = 1)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 1 GiB device copy (HBM ceiling; counter calibration)")
    ap.add_argument("--rt-log", action="store_true",
                    help="log the wetted radius r(t) of the spreading workload instead of the benchmark")
    ap.add_argument("--rt-steps", type=int, default=5000)
    ap.add_argument("--rt-every", type=int, default=50)
    ap.add_argument("--angle-study", action="store_true",
                    help="static contact-angle test of Sec. III A instead of the throughput benchmark")
    ap.add_argument("--angle-shape", default="256,256,256")
    ap.add_argument("--angle-R", type=float, default=40.0)
    ap.add_argument("--angle-cz", type=float, default=2.0, help="droplet centre height (node units)")
    ap.add_argument("--angle-init", default="sphere", choices=["sphere", "cap"],
                    help="sphere: the paper's start (about 90 degrees); cap: a cap at the imposed angle "
                         "with the same liquid volume")
    ap.add_argument("--angles", default="30,60,90,120,150,160")
    ap.add_argument("--wall-compression", default="1", help="comma list of readings of the wall flux")
    ap.add_argument("--ghost-localization", default="1",
                    help="comma list: 1 = lambda_s of Eq. (47) in the ghost, 0 = lambda_s = 1 (diagnostic)")
    ap.add_argument("--angle-dump", default=None, help="folder for the central xz slices of every checkpoint")
    ap.add_argument("--delta", type=float, default=4.0)
    ap.add_argument("--D", type=float, default=0.1)
    ap.add_argument("--nu", type=float, default=0.04)
    ap.add_argument("--angle-steps", type=int, default=60000)
    ap.add_argument("--angle-min-steps", type=int, default=20000)
    ap.add_argument("--angle-every", type=int, default=4000)
    ap.add_argument("--angle-tol", type=float, default=0.1)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (no sharding or collectives); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_25444_amd import capi
    from paper_2607_25444_amd import tuning
    from paper_2607_25444_amd import workloads as W

    if args.copy_probe:
        copy_probe(torch)
        return
    if args.angle_study:
        angle_study(args)
        return
    if args.rt_log:
        rt_log(args)
        return

    w = workload_of(W, args.workload, args.seed)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else tuning.launch_for(w.shape)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] workload {w.name} N={w.N} fluid={w.n_fluid} launch={launch}")
    blk = plain_block(torch, capi, w, launch, args.steps, args.warmup, probes=True)
    log(f"[bench] {w.name}: {blk['ms_per_step']:.4f} ms/step, {blk['value']:.1f} MLUPS, kernels {blk['kernel_ms']}")
    traffic = measured_traffic(w.name)
    rec = {
        "metric": METRIC,
        "value": blk["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": blk["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "path": "plain step (W ghosts, H collide-stream, P CAC update, V volume correction)",
            "nodes": w.N,
            "fluid_nodes": w.n_fluid,
            "wall_nodes": blk["wall_nodes"],
            "theta_deg": w.meta.get("theta_deg"),
            "seed": args.seed,
            "launch": list(launch),
            "precision": "FP32 populations and fields, FP64 volume reductions",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_hydro",
            "achieved": blk["hydro_algorithmic_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(blk["hydro_algorithmic_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_lu": HYDRO_BYTES_PER_LU,
            "units_per_launch": w.n_fluid,
            "kernel_ms": blk["kernel_ms"]["H"],
        },
        "step": blk["step"],
        "ceilings": blk["ceilings"],
    }
    if traffic:
        rec["ceilings"]["hydro_measured_over_pull_copy"] = round(
            traffic / (blk["kernel_ms"]["H"] * 1e-3) / 1e9 / blk["ceilings"]["pull_copy_GBs"], 4)
    if args.workload != "spreading" and not args.no_spreading:
        log("[bench] spreading 256x256x128 (plain step) ...")
        ws = W.spreading_256(args.seed)
        sb = plain_block(torch, capi, ws, tuning.launch_for(ws.shape), args.steps, args.warmup, probes=False)
        sb["roofline_frac"] = round(sb["hydro_algorithmic_GBs"] / HBM_PEAK_GBS, 4)
        sb["traffic"] = measured_traffic(ws.name)
        rec["spreading"] = sb
        log(f"[bench] spreading {sb['value']} MLUPS, {sb['ms_per_step']} ms/step")
    if not args.no_r1:
        log("[bench] gradient-form collision on the spreading workload ...")
        ws = W.spreading_256(args.seed)
        rec["r1"] = bench_r1(torch, capi, ws, tuning.launch_for(ws.shape), args.r1_steps, 20)
        plain = rec["spreading"]["value"] if "spreading" in rec else rec["value"]
        rec["r1"]["ratio_to_plain_same_workload"] = round(rec["r1"]["value"] / plain, 4)
        log(f"[bench] r1 {rec['r1']}")
    if not args.no_batch:
        log("[bench] batched workload ...")
        rec["batched"] = bench_batch(torch, capi, W, args.batch_steps, 10, args.seed)
        plain = rec["spreading"]["value"] if "spreading" in rec else rec["value"]
        rec["batched"]["ratio_to_plain_spreading"] = round(rec["batched"]["value"] / plain, 4)
        log(f"[bench] batched {rec['batched']}")
    if not args.no_adjoint:
        log("[bench] adjoint workload ...")
        rec["adjoint"] = bench_adjoint(torch, capi, tuning, W, args.adjoint_steps, args.adjoint_K, args.seed)
        log(f"[bench] adjoint {rec['adjoint']}")
    if not args.no_adjoint and not args.no_adjoint_resident:
        # the same rollout as one segment: the recorded sweep keeps every step
        # in the rings (about 128 B per node and step), and nothing is replayed
        torch.cuda.empty_cache()
        need = 128 * W.adjoint_128(args.seed).N * args.adjoint_steps * 1.05 + (4 << 30)
        free_b, _ = torch.cuda.mem_get_info()
        if free_b > need:
            log("[bench] adjoint workload, whole rollout resident in HBM ...")
            rec["adjoint_resident"] = bench_adjoint(torch, capi, tuning, W, args.adjoint_steps, args.adjoint_steps,
                                                    args.seed)
            log(f"[bench] adjoint_resident {rec['adjoint_resident']}")
        else:
            rec["adjoint_resident"] = {"skipped": f"needs {need / 2**30:.0f} GiB, {free_b / 2**30:.0f} GiB free"}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host ...")
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, W, capi, launch)
        log(f"[bench] cpu baseline {rec['cpu_baseline']}")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
