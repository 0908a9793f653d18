"""ctypes wrapper around the FP64 C oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Shares nothing with the GPU library: its own C
source, its own build line, its own tables.  Arrays are numpy float64 in the
structure-of-arrays layout ``a[component * N + n]`` with
``n = x + nx * (y + ny * z)``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from contextlib import contextmanager
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cac_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Q = 27


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [("rho_l", C.c_double), ("rho_g", C.c_double), ("nu_l", C.c_double), ("nu_g", C.c_double),
                ("sigma", C.c_double), ("delta", C.c_double), ("D", C.c_double), ("g", C.c_double * 3),
                ("eps_phi", C.c_double), ("eps_n", C.c_double), ("sin_tol", C.c_double),
                ("cot_max", C.c_double), ("volume_correction", C.c_int), ("wall_compression", C.c_int),
                ("collision", C.c_int), ("ghost_localization", C.c_int)]


@dataclass
class Params:
    """Physical and numerical parameters of the step (lattice units)."""
    rho_l: float = 1.0
    rho_g: float = 1.0
    nu_l: float = 0.04
    nu_g: float = 0.04
    sigma: float = 0.02
    delta: float = 4.0
    D: float = 0.1
    g: tuple = (0.0, 0.0, 0.0)
    eps_phi: float = 1e-3
    eps_n: float = 1e-12
    sin_tol: float = 1e-6
    cot_max: float = 1e6
    volume_correction: int = 1
    wall_compression: int = 1
    collision: int = 0          # A2 of Eq. (14): 0 local second moment, 1 gradient form of Eq. (15)
    ghost_localization: int = 1  # lambda_s of Eq. (47) in the ghost (1), or lambda_s = 1 (0, diagnostic)

    def c_struct(self) -> OrcParams:
        p = OrcParams()
        for k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "delta", "D", "eps_phi", "eps_n",
                  "sin_tol", "cot_max"):
            setattr(p, k, float(getattr(self, k)))
        for d in range(3):
            p.g[d] = float(self.g[d])
        p.volume_correction = int(self.volume_correction)
        p.wall_compression = int(self.wall_compression)
        p.collision = int(self.collision)
        p.ghost_localization = int(self.ghost_localization)
        return p


_lib = None


def build_variant(out_path: str, replacements) -> str:
    """Compile a copy of the oracle with textual replacements (old, new) applied
    to its C source into out_path.  For tests that plant a mistake in the oracle
    and check that a pin catches it; every `old` must occur in the source."""
    src = open(_SRC).read()
    for old, new in replacements:
        if old not in src:
            raise ValueError(f"planted change not applicable: {old!r}")
        src = src.replace(old, new)
    csrc = out_path + ".c"
    with open(csrc, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                    "-o", out_path, csrc, "-lm"], check=True)
    return out_path


def build_native(out_path: str) -> str:
    """The same source compiled for the host CPU (-O3 -march=native, still
    without fast-math: ISO C keeps floating-point contraction off, so the
    arithmetic and its order are those of the default build).  For long
    reference runs."""
    subprocess.run(["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                    "-o", out_path, _SRC, "-lm"], check=True)
    return out_path


@contextmanager
def using_library(path: str):
    """Route every call of this module to the oracle library at `path` (a
    variant from build_variant) inside the block."""
    global _lib
    saved = _lib
    _lib = _configure(C.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        _lib = _configure(C.CDLL(build()))
    return _lib


def _configure(L):
    """Argument and result types of the oracle's exported functions."""
    dp = C.POINTER(C.c_double)
    u8p = C.POINTER(C.c_uint8)
    i32p = C.POINTER(C.c_int32)
    pp = C.POINTER(OrcParams)
    L.orc_lattice.argtypes = [C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
    L.orc_feq.argtypes = [C.c_double, dp, dp]
    L.orc_guo.argtypes = [dp, dp, dp]
    L.orc_fneq_reg.argtypes = [dp, dp, dp]
    L.orc_collide_node.argtypes = [pp, C.c_double, dp, C.c_double, dp, dp, dp, dp]
    L.orc_macro_node.argtypes = [pp, C.c_double, dp, C.c_double, dp, dp, dp, dp, dp]
    L.orc_a2_local.argtypes = [C.c_double, dp, dp, dp, dp]
    L.orc_post_node.argtypes = [C.c_double, dp, dp, C.c_double, dp, dp]
    L.orc_a2grad.argtypes = [C.c_int, C.c_int, C.c_int, u8p, dp, dp, dp]
    L.orc_grad_iso.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp]
    L.orc_lap_iso.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp]
    L.orc_wall_nodes.argtypes = [C.c_int, C.c_int, C.c_int, u8p, i32p, i32p, i32p, C.c_int]
    L.orc_wall_nodes.restype = C.c_int
    L.orc_ghost.argtypes = [pp, C.c_int, C.c_int, C.c_int, u8p, dp, dp, dp, dp]
    L.orc_ghost.restype = C.c_int
    L.orc_hydro.argtypes = [pp, C.c_int, C.c_int, C.c_int, u8p, dp, dp, dp, dp, dp, dp]
    L.orc_phase.argtypes = [pp, C.c_int, C.c_int, C.c_int, u8p, dp, dp, dp, dp]
    L.orc_volume.argtypes = [pp, C.c_int, C.c_int, C.c_int, u8p, dp, C.c_double, dp, dp]
    L.orc_mass.argtypes = [C.c_int, C.c_int, C.c_int, u8p, dp]
    L.orc_mass.restype = C.c_double
    L.orc_init.argtypes = [C.c_int, C.c_int, C.c_int, u8p, dp, dp, dp, dp, dp, dp]
    L.orc_step.argtypes = [pp, C.c_int, C.c_int, C.c_int, u8p, dp, dp, dp, dp, dp, C.c_double, C.c_int, dp]
    L.orc_step.restype = C.c_int
    L.orc_num_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    return L


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- node level

def lattice():
    c = (C.c_int * (3 * Q))()
    w = (C.c_double * Q)()
    o = (C.c_int * Q)()
    lib().orc_lattice(c, w, o)
    return np.array(c[:], dtype=np.int64).reshape(Q, 3), np.array(w[:]), np.array(o[:], dtype=np.int64)


def feq(pstar, u):
    u = _f64(u)
    out = np.zeros(Q)
    lib().orc_feq(float(pstar), _d(u), _d(out))
    return out


def guo(u, a):
    u, a = _f64(u), _f64(a)
    out = np.zeros(Q)
    lib().orc_guo(_d(u), _d(a), _d(out))
    return out


def fneq_reg(u, A2):
    u, A2 = _f64(u), _f64(np.asarray(A2).reshape(9))
    out = np.zeros(Q)
    lib().orc_fneq_reg(_d(u), _d(A2), _d(out))
    return out


def collide_node(params: Params, phi, G, L, f):
    G, f = _f64(G), _f64(f)
    fp, u, ps = np.zeros(Q), np.zeros(3), C.c_double()
    p = params.c_struct()
    lib().orc_collide_node(C.byref(p), float(phi), _d(G), float(L), _d(f), _d(fp), _d(u), C.byref(ps))
    return fp, u, ps.value


# ---------------------------------------------------------------- grid level

def grad_iso(psi, shape):
    nx, ny, nz = shape
    psi = _f64(psi).reshape(-1)
    out = np.zeros(3 * psi.size)
    lib().orc_grad_iso(nx, ny, nz, _d(psi), _d(out))
    return out


def lap_iso(psi, shape):
    nx, ny, nz = shape
    psi = _f64(psi).reshape(-1)
    out = np.zeros(psi.size)
    lib().orc_lap_iso(nx, ny, nz, _d(psi), _d(out))
    return out


def wall_nodes(solid, shape):
    """Return (linear index, 6*unnormalised normal (nb,3), donor link or -1)."""
    nx, ny, nz = shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    nb = lib().orc_wall_nodes(nx, ny, nz, _u8(solid), None, None, None, 0)
    idx = np.zeros(max(nb, 1), np.int32)
    n6 = np.zeros(3 * max(nb, 1), np.int32)
    qs = np.zeros(max(nb, 1), np.int32)
    i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
    lib().orc_wall_nodes(nx, ny, nz, _u8(solid), i32(idx), i32(n6), i32(qs), nb)
    return idx[:nb], n6[:3 * nb].reshape(nb, 3), qs[:nb]


def ghost(params, shape, solid, theta, phi_in, with_flux=False):
    """W substep: phi_hat (and, if with_flux, the wall compressive flux, 3N)."""
    nx, ny, nz = shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    theta, phi_in = _f64(theta).reshape(-1), _f64(phi_in).reshape(-1)
    out = np.zeros_like(phi_in)
    aw = np.zeros(3 * phi_in.size)
    p = params.c_struct()
    lib().orc_ghost(C.byref(p), nx, ny, nz, _u8(solid), _d(theta), _d(phi_in), _d(out), _d(aw))
    return (out, aw) if with_flux else out


def hydro(params, shape, solid, phi_hat, f_in):
    nx, ny, nz = shape
    N = nx * ny * nz
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    phi_hat, f_in = _f64(phi_hat).reshape(-1), _f64(f_in).reshape(-1)
    fpost, fout = np.zeros(Q * N), np.zeros(Q * N)
    u, ps = np.zeros(3 * N), np.zeros(N)
    p = params.c_struct()
    lib().orc_hydro(C.byref(p), nx, ny, nz, _u8(solid), _d(phi_hat), _d(f_in), _d(fpost), _d(fout), _d(u), _d(ps))
    return fpost, fout, u, ps


def a2grad(shape, solid, u, omega):
    """Gradient form of the non-equilibrium moment, Eq. (15), at every fluid
    node (a solid neighbour holds the mirror image -u of the node): returns 9
    planes of N, row-major (a, b)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    u, omega = _f64(u).reshape(-1), _f64(omega).reshape(-1)
    out = np.zeros(9 * N)
    lib().orc_a2grad(nx, ny, nz, _u8(solid), _d(u), _d(omega), _d(out))
    return out


def phase(params, shape, solid, phi_hat, u, a_wall=None):
    nx, ny, nz = shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    phi_hat, u = _f64(phi_hat).reshape(-1), _f64(u).reshape(-1)
    aw = None if a_wall is None else _f64(a_wall).reshape(-1)
    out = np.zeros_like(phi_hat)
    p = params.c_struct()
    lib().orc_phase(C.byref(p), nx, ny, nz, _u8(solid), _d(phi_hat), _d(u), _d(aw), _d(out))
    return out


def volume(params, shape, solid, phistar, M_target):
    nx, ny, nz = shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    phistar = _f64(phistar).reshape(-1)
    out = np.zeros_like(phistar)
    lam = C.c_double()
    p = params.c_struct()
    lib().orc_volume(C.byref(p), nx, ny, nz, _u8(solid), _d(phistar), float(M_target), _d(out), C.byref(lam))
    return out, lam.value


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def mass(shape, solid, phi):
    nx, ny, nz = shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    phi = _f64(phi).reshape(-1)
    return lib().orc_mass(nx, ny, nz, _u8(solid), _d(phi))


# ---------------------------------------------------------------- simulation

@dataclass
class OracleSim:
    """Whole-step oracle state on the host (FP64)."""
    shape: tuple
    solid: np.ndarray
    theta: np.ndarray
    params: Params
    f: np.ndarray = field(default=None)
    phi: np.ndarray = field(default=None)
    u: np.ndarray = field(default=None)
    pstar: np.ndarray = field(default=None)
    M_target: float = 0.0
    steps: int = 0

    @classmethod
    def create(cls, shape, solid, theta, params, phi0, pstar0=None, u0=None):
        nx, ny, nz = shape
        N = nx * ny * nz
        s = cls(shape=tuple(shape), solid=np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1),
                theta=_f64(theta).reshape(-1).copy(), params=params)
        s.f = np.zeros(Q * N)
        s.phi = np.zeros(N)
        s.u = np.zeros(3 * N)
        s.pstar = np.zeros(N)
        phi0 = _f64(phi0).reshape(-1)
        ps0 = None if pstar0 is None else _f64(pstar0).reshape(-1)
        u0_ = None if u0 is None else _f64(u0).reshape(-1)
        M = C.c_double()
        lib().orc_init(nx, ny, nz, _u8(s.solid), _d(phi0), _d(ps0), _d(u0_), _d(s.f), _d(s.phi), C.byref(M))
        s.M_target = M.value
        if pstar0 is not None:
            s.pstar[:] = ps0
        if u0 is not None:
            s.u[:] = u0_
        return s

    def step(self, n=1, fpost=None):
        nx, ny, nz = self.shape
        p = self.params.c_struct()
        rc = lib().orc_step(C.byref(p), nx, ny, nz, _u8(self.solid), _d(self.theta), _d(self.f), _d(self.phi),
                            _d(self.u), _d(self.pstar), float(self.M_target), int(n), _d(fpost))
        if rc != 0:
            raise FloatingPointError(f"oracle step returned {rc}")
        self.steps += n
        return self

    def mass(self):
        return mass(self.shape, self.solid, self.phi)
