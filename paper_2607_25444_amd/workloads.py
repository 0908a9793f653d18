"""Seeded synthetic inputs for the CAC wetting step.

This module builds geometry masks, contact-angle fields, initial phase fields
and parameter sets.  It holds none of the method's arithmetic and is the only
code that the GPU path and the FP64 oracle both use (each side receives the
same arrays).  The recipes follow the paper's workloads (Sec. III): droplets
on flat walls with a tanh interface profile, and a sharp-edged orifice plate.

Conventions: node coordinates are integers 0..n-1, linear index
``n = x + nx * (y + ny * z)``, arrays are flattened in that order.  Solid
voxel layers sit at z = 0 and z = nz - 1 (the wall surface is at z = 1/2);
x and y are periodic.  The initial phase field is
``phi0 = (1 - tanh(2 (d - R) / delta)) / 2`` with d the distance to the
droplet centre, evaluated on every node (solid nodes included, where it is
the initial ghost value).
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict

import numpy as np


@dataclass
class Workload:
    name: str
    shape: tuple            # (nx, ny, nz)
    solid: np.ndarray       # uint8, N, 1 = solid
    theta: np.ndarray       # float32, N, radians, read at wall nodes
    phi0: np.ndarray        # float32, N
    params: dict            # physical parameters (lattice units)
    steps: int              # nominal run length of the workload
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    @property
    def n_fluid(self):
        return int(self.N - int(self.solid.sum()))


def default_params(**kw) -> dict:
    p = dict(rho_l=1.0, rho_g=1.0, nu_l=0.04, nu_g=0.04, sigma=0.02, delta=4.0, D=0.1,
             g=(0.0, 0.0, 0.0), eps_phi=1e-3, eps_n=1e-12, sin_tol=1e-6, cot_max=1e6,
             volume_correction=1, wall_compression=1, ghost_localization=1)
    p.update(kw)
    return p


def grid(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def flat_walls(shape) -> np.ndarray:
    """Solid layers at z = 0 and z = nz - 1; x, y periodic."""
    nx, ny, nz = shape
    s = np.zeros((nz, ny, nx), np.uint8)
    s[0] = 1
    s[nz - 1] = 1
    return s.reshape(-1)


def tanh_droplet(shape, centre, R, delta) -> np.ndarray:
    x, y, z = grid(shape)
    d = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    return (0.5 * (1.0 - np.tanh(2.0 * (d - R) / delta))).reshape(-1)


def flat_interface(shape, z0, delta, liquid_below=True) -> np.ndarray:
    x, y, z = grid(shape)
    s = 2.0 * (z - z0) / delta
    return (0.5 * (1.0 - np.tanh(s)) if liquid_below else 0.5 * (1.0 + np.tanh(s))).reshape(-1)


def uniform_theta(shape, theta_deg) -> np.ndarray:
    nx, ny, nz = shape
    return np.full(nx * ny * nz, np.deg2rad(theta_deg), np.float32)


# ------------------------------------------------------------------ workloads

def sessile_32(theta_deg=60.0, seed=0) -> Workload:
    """Static sessile droplet: 32^3, flat walls, hemispherical cap R = 8 centred on
    the wall, interface width 4, uniform angle, rho and nu ratios 1, fluid at rest."""
    shape = (32, 32, 32)
    nx, ny, nz = shape
    solid = flat_walls(shape)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, 0.5), 8.0, 4.0)
    return Workload("sessile_32x32x32", shape, solid, uniform_theta(shape, theta_deg),
                    phi0.astype(np.float32), default_params(), 200, dict(R=8.0, theta_deg=theta_deg))


def sessile(shape, R, theta_deg, delta=4.0, centre_z=0.5, **pkw) -> Workload:
    nx, ny, nz = shape
    solid = flat_walls(shape)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, centre_z), R, delta)
    return Workload(f"sessile_{nx}x{ny}x{nz}", shape, solid, uniform_theta(shape, theta_deg),
                    phi0.astype(np.float32), default_params(delta=delta, **pkw), 0,
                    dict(R=R, theta_deg=theta_deg))


def spreading_256(seed=0) -> Workload:
    """Short-time spreading: 256x256x128, flat walls, sphere R = 40 touching the wall
    surface, interface width 4; angle and Ohnesorge number drawn from the seed."""
    rng = np.random.default_rng(seed)
    shape = (256, 256, 128)
    nx, ny, nz = shape
    theta = float(rng.choice([30.0, 60.0, 90.0, 120.0, 150.0]))
    oh = float(rng.choice([0.02, 0.0395, 0.08]))
    R, sigma, rho = 40.0, 0.02, 1.0
    nu = oh * np.sqrt(sigma * R / rho)
    solid = flat_walls(shape)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, 0.5 + R), R, 4.0)
    return Workload("spreading_256x256x128", shape, solid, uniform_theta(shape, theta),
                    phi0.astype(np.float32), default_params(nu_l=nu, nu_g=nu, sigma=sigma), 5000,
                    dict(R=R, theta_deg=theta, Oh=oh, tau_i=float(np.sqrt(rho * R ** 3 / sigma))))


def spreading_512(theta_deg=90.0) -> Workload:
    """The paper's spreading lattice (Sec. III B): 512^3, R0 = 80 touching the
    wall, rho = 1, nu = 0.05, sigma = 0.02 (Oh_R0 = 3.95e-2), interface width 4."""
    shape = (512, 512, 512)
    nx, ny, nz = shape
    R = 80.0
    solid = flat_walls(shape)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, 0.5 + R), R, 4.0)
    return Workload("spreading_512x512x512", shape, solid, uniform_theta(shape, theta_deg),
                    phi0.astype(np.float32), default_params(nu_l=0.05, nu_g=0.05, sigma=0.02), 0,
                    dict(R=R, theta_deg=theta_deg))


def orifice_plate_mask(shape, z_lo, thickness, hole_d) -> np.ndarray:
    nx, ny, nz = shape
    x, y, z = grid(shape)
    s = flat_walls(shape).reshape(nz, ny, nx).copy()
    r2 = (x - (nx - 1) / 2) ** 2 + (y - (ny - 1) / 2) ** 2
    plate = (z >= z_lo) & (z < z_lo + thickness) & (r2 >= (hole_d / 2) ** 2)
    s[plate] = 1
    return s.reshape(-1)


def orifice_192(seed=0) -> Workload:
    """Gravity-driven passage through a sharp-edged orifice: 192x192x768, plate 8 cells
    thick at mid-height with a centred hole of diameter 48, droplet R = 40 whose lowest
    point is 60 cells above the plate, g = 1e-5 downward, angle in [60, 150] from the seed.
    Densities, viscosities, sigma and delta are the paper's orifice values."""
    rng = np.random.default_rng(seed)
    shape = (192, 192, 768)
    nx, ny, nz = shape
    theta = float(rng.uniform(60.0, 150.0))
    R, z_lo, h = 40.0, 380, 8
    solid = orifice_plate_mask(shape, z_lo, h, 48.0)
    zc = (z_lo + h - 0.5) + 60.0 + R
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, zc), R, 6.0)
    prm = default_params(rho_l=1.2, rho_g=0.9, nu_l=0.031, nu_g=0.24, sigma=0.025, delta=6.0,
                         g=(0.0, 0.0, -1e-5))
    return Workload("orifice_192x192x768", shape, solid, uniform_theta(shape, theta),
                    phi0.astype(np.float32), prm, 20000, dict(R=R, theta_deg=theta))


def batch_domains(seed=0, ndom=64, sizes=(32, 48, 64, 96, 128)):
    """64 independent droplet domains: cubic edge L from `sizes`, R = L/4, sessile
    (centre on the wall) or spreading (sphere touching the wall), angle in [30, 150]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(ndom):
        L = int(rng.choice(sizes))
        spreading = bool(rng.integers(2))
        theta = float(rng.uniform(30.0, 150.0))
        R = L / 4.0
        cz = 0.5 + (R if spreading else 0.0)
        w = sessile((L, L, L), R, theta, centre_z=cz)
        w.name = f"domain{k}_{L}"
        w.meta.update(spreading=spreading)
        out.append(w)
    return out


def gaussian_bump_theta(shape, seed, lo=40.0, hi=140.0, nbumps=4) -> np.ndarray:
    """Bottom-wall angle field: sum of 4 Gaussian bumps on the periodic (x, y) plane,
    rescaled to [lo, hi] degrees; top wall 90 degrees."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    x, y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64), indexing="xy")
    B = np.zeros((ny, nx))
    for _ in range(nbumps):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        s = rng.uniform(10.0, 25.0)
        a = rng.uniform(0.5, 1.0)
        dx = np.minimum(np.abs(x - cx), nx - np.abs(x - cx))
        dy = np.minimum(np.abs(y - cy), ny - np.abs(y - cy))
        B += a * np.exp(-(dx ** 2 + dy ** 2) / (2 * s * s))
    B = lo + (hi - lo) * (B - B.min()) / (B.max() - B.min())
    th = np.full((nz, ny, nx), 90.0)
    th[0] = B
    return np.deg2rad(th).astype(np.float32).reshape(-1)


def adjoint_128(seed=0, shape=(128, 128, 64), R=24.0) -> Workload:
    """Contact-angle inversion: flat walls, bottom angle field from Gaussian bumps,
    hemispherical droplet centred on the bottom wall."""
    nx, ny, nz = shape
    solid = flat_walls(shape)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, 0.5), R, 4.0)
    return Workload(f"adjoint_{nx}x{ny}x{nz}", shape, solid, gaussian_bump_theta(shape, seed),
                    phi0.astype(np.float32), default_params(), 1000, dict(R=R))


def random_smooth_field(shape, seed, lo=0.0, hi=1.0) -> np.ndarray:
    """Smooth random periodic field in [lo, hi] (a few low Fourier modes)."""
    rng = np.random.default_rng(seed)
    x, y, z = grid(shape)
    nx, ny, nz = shape
    f = np.zeros_like(x)
    for _ in range(4):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        f += rng.uniform(0.5, 1.0) * np.sin(2 * np.pi * k[0] * x / nx + ph[0]) * \
            np.sin(2 * np.pi * k[1] * y / ny + ph[1]) * np.sin(2 * np.pi * k[2] * z / nz + ph[2])
    f = (f - f.min()) / (f.max() - f.min())
    return (lo + (hi - lo) * f).reshape(-1)


def random_geometry(shape, seed, n_blocks=3) -> np.ndarray:
    """Flat walls plus a few solid boxes at least 2 voxels thick (tiny parity grids)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    s = flat_walls(shape).reshape(nz, ny, nx).copy()
    for _ in range(n_blocks):
        lx, ly, lz = rng.integers(2, 4, size=3)
        x0, y0 = rng.integers(0, nx), rng.integers(0, ny)
        z0 = rng.integers(2, max(3, nz - lz - 2))
        for dz in range(lz):
            for dy in range(ly):
                for dx in range(lx):
                    s[z0 + dz, (y0 + dy) % ny, (x0 + dx) % nx] = 1
    return s.reshape(-1)


# ---------------------------------------------------------------- droplet impact (Sec. III C)

def impact(shape=(64, 64, 48), R=12.0, We=10.0, theta_deg=130.0, delta=4.0, **pkw) -> Workload:
    """Droplet impact on a hydrophobic wall at liquid-to-gas density ratio 1000:
    rho_l = 10, rho_g = 0.01, nu_l = nu_g = 0.05, sigma = 0.02, theta = 130 deg,
    no gravity.  The droplet's lower interface touches the wall (centre at z =
    1/2 + R) and it moves towards the wall with U0 = sqrt(We sigma / (rho_l D0)),
    D0 = 2R; the initial velocity is -U0 phi0 along z (the gas at rest)."""
    nx, ny, nz = shape
    prm = dict(rho_l=10.0, rho_g=0.01, nu_l=0.05, nu_g=0.05, sigma=0.02, delta=delta)
    prm.update(pkw)
    U0 = float(np.sqrt(We * prm["sigma"] / (prm["rho_l"] * 2.0 * R)))
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, 0.5 + R), R, delta).astype(np.float32)
    N = nx * ny * nz
    u0 = np.zeros(3 * N, np.float32)
    u0[2 * N:] = -U0 * phi0
    w = Workload(f"impact_{nx}x{ny}x{nz}", shape, flat_walls(shape), uniform_theta(shape, theta_deg), phi0,
                 default_params(**prm), 0, dict(R=R, We=We, U0=U0, theta_deg=theta_deg))
    w.meta["u0"] = u0
    return w


def impact_256(We=10.0) -> Workload:
    """Throughput case of the impact family: 256^3, R0 = 40."""
    return impact((256, 256, 256), R=40.0, We=We)


# ---------------------------------------------------------------- curved and porous solids
# Voxel geometries beyond planar walls (the paper's outlook, Sec. IV): the wall
# normal and the donor are reconstructed from the mask alone, so these masks
# exercise staircase corners, convex and concave edges and the tie-breaks.

def ball_mask(shape, centre, R, periodic_xy=True) -> np.ndarray:
    """1 on nodes within distance R of centre (x and y distances periodic)."""
    nx, ny, nz = shape
    m = np.zeros((nz, ny, nx), np.uint8)
    r = int(np.ceil(R)) + 1
    zs = np.arange(max(0, int(np.floor(centre[2])) - r), min(nz, int(np.ceil(centre[2])) + r + 1))
    ys = np.arange(int(np.floor(centre[1])) - r, int(np.ceil(centre[1])) + r + 1)
    xs = np.arange(int(np.floor(centre[0])) - r, int(np.ceil(centre[0])) + r + 1)
    if not periodic_xy:
        ys, xs = ys[(ys >= 0) & (ys < ny)], xs[(xs >= 0) & (xs < nx)]
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    inside = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2 <= R * R
    m[Z[inside], Y[inside] % ny, X[inside] % nx] = 1
    return m.reshape(-1)


def sphere_substrate(shape=(64, 64, 48), Rs=14.0, R=10.0, theta_deg=60.0, delta=4.0, **pkw) -> Workload:
    """Sessile droplet on a voxelised solid sphere that rests sunk into the bottom
    wall; the droplet overlaps the sphere's top."""
    nx, ny, nz = shape
    c = ((nx - 1) / 2, (ny - 1) / 2, 0.5 + 0.6 * Rs)
    solid = np.maximum(flat_walls(shape), ball_mask(shape, c, Rs))
    phi0 = tanh_droplet(shape, (c[0], c[1], c[2] + Rs + 0.3 * R), R, delta)
    return Workload(f"sphere_substrate_{nx}x{ny}x{nz}", shape, solid, uniform_theta(shape, theta_deg),
                    phi0.astype(np.float32), default_params(delta=delta, **pkw), 0,
                    dict(Rs=Rs, R=R, theta_deg=theta_deg, centre=c))


def cylinder_substrate(shape=(64, 40, 48), Rc=10.0, R=9.0, theta_deg=90.0, delta=4.0, **pkw) -> Workload:
    """Droplet on a voxelised solid cylinder (axis along y) lying on the bottom wall."""
    nx, ny, nz = shape
    x, y, z = grid(shape)
    cx, cz = (nx - 1) / 2, 0.5 + 0.8 * Rc
    cyl = (((x - cx) ** 2 + (z - cz) ** 2) <= Rc * Rc).astype(np.uint8).reshape(-1)
    solid = np.maximum(flat_walls(shape), cyl)
    phi0 = tanh_droplet(shape, (cx, (ny - 1) / 2, cz + Rc + 0.3 * R), R, delta)
    return Workload(f"cylinder_substrate_{nx}x{ny}x{nz}", shape, solid, uniform_theta(shape, theta_deg),
                    phi0.astype(np.float32), default_params(delta=delta, **pkw), 0,
                    dict(Rc=Rc, R=R, theta_deg=theta_deg))


def rough_wall(shape=(64, 64, 40), seed=0, n_pillars=24, R=12.0, delta=4.0, **pkw) -> Workload:
    """Droplet on a rough bottom wall: random square pillars 2-4 voxels wide and
    1-4 high; contact angle per wall node uniform in [40, 140] degrees."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    s = flat_walls(shape).reshape(nz, ny, nx).copy()
    for _ in range(n_pillars):
        w, h = rng.integers(2, 5), rng.integers(1, 5)
        x0, y0 = rng.integers(0, nx), rng.integers(0, ny)
        for dz in range(1, 1 + h):
            for dy in range(w):
                for dx in range(w):
                    s[dz, (y0 + dy) % ny, (x0 + dx) % nx] = 1
    theta = np.deg2rad(rng.uniform(40.0, 140.0, nx * ny * nz)).astype(np.float32)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, 3.5 + 0.6 * R), R, delta)
    return Workload(f"rough_wall_{nx}x{ny}x{nz}", shape, s.reshape(-1), theta, phi0.astype(np.float32),
                    default_params(delta=delta, **pkw), 0, dict(R=R, seed=seed))


def porous_packing(shape=(64, 64, 64), seed=0, n_spheres=14, r_lo=4.0, r_hi=8.0, R=None, delta=4.0,
                   **pkw) -> Workload:
    """Droplet above a random packing of (overlapping) solid spheres filling the
    lower half of the box (periodic in x and y); contact angle per wall node
    uniform in [40, 140] degrees."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    solid = flat_walls(shape)
    top = 0.0
    for _ in range(n_spheres):
        r = rng.uniform(r_lo, r_hi)
        c = (rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(1.0 + r * 0.5, nz / 2 - r * 0.5))
        top = max(top, c[2] + r)
        solid = np.maximum(solid, ball_mask(shape, c, r))
    R = R if R is not None else min(nx, ny) / 5.0
    theta = np.deg2rad(rng.uniform(40.0, 140.0, nx * ny * nz)).astype(np.float32)
    zc = min(top + 0.6 * R, nz - 2.0 - R)
    phi0 = tanh_droplet(shape, ((nx - 1) / 2, (ny - 1) / 2, zc), R, delta)
    return Workload(f"porous_{nx}x{ny}x{nz}", shape, solid, theta, phi0.astype(np.float32),
                    default_params(delta=delta, **pkw), 0, dict(R=R, seed=seed, n_spheres=n_spheres))


def porous_256(seed=0) -> Workload:
    """Throughput case of the porous family: 256x256x128, 60 spheres of radius
    8-16 in the lower half, droplet R = 32 above."""
    return porous_packing((256, 256, 128), seed=seed, n_spheres=60, r_lo=8.0, r_hi=16.0, R=32.0)


def params_dict(w: Workload) -> dict:
    return dict(w.params)


__all__ = [n for n in dir() if not n.startswith("_")] + ["asdict"]
