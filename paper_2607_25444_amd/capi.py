"""ctypes binding of libcac (include/cac.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (the allocation callback returns torch-owned
buffers) and the stream (torch's current stream at construction).  The
library must be built (``python -m paper_2607_25444_amd.build``); loading
fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcac.so")

CAC_OK, CAC_ERR_ARG, CAC_ERR_GEOMETRY, CAC_ERR_HIP, CAC_ERR_NONFINITE, CAC_ERR_STATE, CAC_ERR_ALLOC = range(7)
CAC_DEBUG_POISON, CAC_DEBUG_REVERSE_ORDER = 1, 2


class CacError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class CacParams(C.Structure):
    _fields_ = [("rho_l", C.c_double), ("rho_g", C.c_double), ("nu_l", C.c_double), ("nu_g", C.c_double),
                ("sigma", C.c_double), ("delta", C.c_double), ("D", C.c_double), ("g", C.c_double * 3),
                ("eps_phi", C.c_double), ("eps_n", C.c_double), ("sin_tol", C.c_double), ("cot_max", C.c_double),
                ("volume_correction", C.c_int), ("wall_compression", C.c_int), ("collision", C.c_int),
                ("ghost_localization", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)


class DomainDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("params", CacParams),
                ("solid", C.c_void_p), ("theta_rad", C.c_void_p), ("d_phi0", C.c_void_p)]

# symbol -> (restype, argtypes); every symbol declared in include/cac.h
_vp = C.c_void_p
_hp = C.c_void_p
SIGNATURES = {
    "cac_default_params": (C.c_int, [C.POINTER(CacParams)]),
    "cac_init": (C.c_int, [C.POINTER(_hp), C.c_int, C.c_int, C.c_int, C.POINTER(CacParams), ALLOC_FN, _vp, _vp]),
    "cac_set_geometry": (C.c_int, [_hp, _vp, _vp]),
    "cac_num_wall_nodes": (C.c_int, [_hp, C.POINTER(C.c_int)]),
    "cac_wall_nodes": (C.c_int, [_hp, _vp, _vp, _vp]),
    "cac_wall_tables": (C.c_int, [C.c_int, C.c_int, C.c_int, _vp, C.POINTER(C.c_int), _vp, _vp, _vp, C.c_int]),
    "cac_set_contact_angles": (C.c_int, [_hp, _vp]),
    "cac_set_state": (C.c_int, [_hp, _vp, _vp, _vp]),
    "cac_step": (C.c_int, [_hp, C.c_int]),
    "cac_volume": (C.c_int, [_hp, C.POINTER(C.c_double)]),
    "cac_get_fields": (C.c_int, [_hp, _vp, _vp, _vp]),
    "cac_get_populations": (C.c_int, [_hp, _vp]),
    "cac_sync": (C.c_int, [_hp]),
    "cac_set_launch": (C.c_int, [_hp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "cac_profile_step": (C.c_int, [_hp, C.c_int, C.POINTER(C.c_double)]),
    "cac_pull_copy_probe": (C.c_int, [_hp, C.c_int, C.POINTER(C.c_double)]),
    "cac_set_debug": (C.c_int, [_hp, C.c_int]),
    "cac_destroy": (C.c_int, [_hp]),
    "cac_state_bytes": (C.c_int, [_hp, C.POINTER(C.c_size_t)]),
    "cac_save_state": (C.c_int, [_hp, _vp, C.c_size_t]),
    "cac_load_state": (C.c_int, [_hp, _vp, C.c_size_t]),
    "cac_debug_substep": (C.c_int, [_hp, C.c_int]),
    "cac_debug_buffer": (C.c_int, [_hp, C.c_int, _vp]),
    "cac_tape_forward": (C.c_int, [_hp, C.c_int, C.c_int]),
    "cac_tape_backward": (C.c_int, [_hp, _vp, _vp, _vp]),
    "cac_loss": (C.c_int, [_hp, _vp, _vp, C.POINTER(C.c_double)]),
    "cac_adjoint": (C.c_int, [_hp, C.c_int, C.c_int, _vp, C.POINTER(C.c_double), _vp]),
    "cac_batch_init": (C.c_int, [C.POINTER(_hp), C.c_int, C.POINTER(DomainDesc), ALLOC_FN, _vp, _vp]),
    "cac_batch_set_schedule": (C.c_int, [_hp] + [C.c_int] * 7),
    "cac_batch_get_schedule": (C.c_int, [_hp, C.POINTER(C.c_int)]),
    "cac_batch_autotune": (C.c_int, [_hp, C.c_char_p, C.c_int, C.POINTER(C.c_double)]),
    "cac_batch_step": (C.c_int, [_hp, C.c_int]),
    "cac_batch_sync": (C.c_int, [_hp]),
    "cac_batch_volume": (C.c_int, [_hp, C.POINTER(C.c_double)]),
    "cac_batch_get_fields": (C.c_int, [_hp, C.c_int, _vp, _vp, _vp]),
    "cac_batch_info": (C.c_int, [_hp, C.POINTER(C.c_int), C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    "cac_batch_profile": (C.c_int, [_hp, C.c_int, C.POINTER(C.c_double)]),
    "cac_batch_destroy": (C.c_int, [_hp]),
    "cac_batch_last_error": (C.c_int, [_hp, C.c_char_p, C.c_size_t]),
    "cac_volume_noalloc": (C.c_int, [C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "cac_status_string": (C.c_char_p, [C.c_int]),
    "cac_last_error": (C.c_int, [_hp, C.c_char_p, C.c_size_t]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcac.so (no GPU call is made).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcac.so is not built ({path}); run python -m paper_2607_25444_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_params(d: dict) -> CacParams:
    lib = load_library()
    p = CacParams()
    lib.cac_default_params(C.byref(p))
    for k, v in d.items():
        if k == "g":
            for i in range(3):
                p.g[i] = float(v[i])
        elif hasattr(p, k):
            setattr(p, k, type(getattr(p, k))(v))
    return p


def wall_tables(solid, shape):
    """Host-side wall tables of the library (no GPU use): (index, normal6, donor)."""
    lib = load_library()
    nx, ny, nz = shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    nb = C.c_int()
    st = lib.cac_wall_tables(nx, ny, nz, solid.ctypes.data_as(C.c_void_p), C.byref(nb), None, None, None, 0)
    if st != CAC_OK:
        raise CacError(st, "cac_wall_tables")
    n = nb.value
    idx = np.zeros(max(n, 1), np.int32)
    n6 = np.zeros(3 * max(n, 1), np.int32)
    q = np.zeros(max(n, 1), np.int32)
    st = lib.cac_wall_tables(nx, ny, nz, solid.ctypes.data_as(C.c_void_p), C.byref(nb), idx.ctypes.data_as(C.c_void_p),
                             n6.ctypes.data_as(C.c_void_p), q.ctypes.data_as(C.c_void_p), n)
    if st != CAC_OK:
        raise CacError(st, "cac_wall_tables")
    return idx[:n], n6[:3 * n].reshape(n, 3), q[:n]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def volume_noalloc(shape, d_solid, d_phi, d_out, stream=None):
    """cac_volume_noalloc: FP64 fluid sum of d_phi (torch uint8 mask, float32
    field, float64 output of one element, all on the current device), launched
    on `stream` (a torch stream; None: torch's current stream).  Asynchronous."""
    lib = load_library()
    nx, ny, nz = shape
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    st = lib.cac_volume_noalloc(nx, ny, nz, _ptr(d_solid), _ptr(d_phi), _ptr(d_out), C.c_void_p(stream.cuda_stream))
    if st != CAC_OK:
        buf = C.create_string_buffer(512)
        lib.cac_last_error(None, buf, 512)
        raise CacError(st, buf.value.decode())


class Sim:
    """One lattice on the current CUDA/HIP device, backed by libcac."""

    def __init__(self, shape, params: dict, device=None, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libcac needs a GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.lib = load_library()
        self.shape = tuple(int(v) for v in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.device = torch.device(device or "cuda")
        self._buffers = []
        self.stream = stream or torch.cuda.current_stream(self.device)

        def _alloc(nbytes, user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self._buffers.append(t)
            return t.data_ptr()

        self._alloc_cb = ALLOC_FN(_alloc)
        self.params = make_params(params)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            self._check(self.lib.cac_init(C.byref(h), nx, ny, nz, C.byref(self.params), self._alloc_cb, None,
                                          C.c_void_p(self.stream.cuda_stream)), None)
        self.h = h
        self.nwall = 0

    # -------------------------------------------------------------- plumbing
    def _check(self, st, h="self"):
        if st == CAC_OK:
            return
        msg = self.lib.cac_status_string(st).decode()
        hh = self.h if h == "self" else h
        if hh is not None:
            buf = C.create_string_buffer(512)
            self.lib.cac_last_error(hh, buf, 512)
            if buf.value:
                msg += ": " + buf.value.decode()
        raise CacError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.cac_destroy(self.h)
            self.h = None
            self._buffers.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- API
    def set_geometry(self, solid, theta_rad=None):
        solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        assert solid.size == self.N
        th = None
        if theta_rad is not None:
            th = np.ascontiguousarray(theta_rad, dtype=np.float32).reshape(-1)
            assert th.size == self.N
        self._check(self.lib.cac_set_geometry(self.h, solid.ctypes.data_as(C.c_void_p),
                                              None if th is None else th.ctypes.data_as(C.c_void_p)))
        n = C.c_int()
        self._check(self.lib.cac_num_wall_nodes(self.h, C.byref(n)))
        self.nwall = n.value
        return self

    def wall_nodes(self):
        nb = self.nwall
        idx = np.zeros(max(nb, 1), np.int32)
        n6 = np.zeros(3 * max(nb, 1), np.int32)
        q = np.zeros(max(nb, 1), np.int32)
        self._check(self.lib.cac_wall_nodes(self.h, idx.ctypes.data_as(C.c_void_p), n6.ctypes.data_as(C.c_void_p),
                                            q.ctypes.data_as(C.c_void_p)))
        return idx[:nb], n6[:3 * nb].reshape(nb, 3), q[:nb]

    def set_contact_angles(self, theta_compact):
        t = self.torch.as_tensor(theta_compact, dtype=self.torch.float32, device=self.device).contiguous()
        assert t.numel() == self.nwall
        self._check(self.lib.cac_set_contact_angles(self.h, _ptr(t)))
        self._keep = t  # stream-ordered copy: keep the source alive until the next call
        return self

    def set_state(self, phi, u=None, pstar=None):
        tc = self.torch
        phi_t = tc.as_tensor(phi, dtype=tc.float32, device=self.device).contiguous().reshape(-1)
        u_t = None if u is None else tc.as_tensor(u, dtype=tc.float32, device=self.device).contiguous().reshape(-1)
        p_t = None if pstar is None else tc.as_tensor(pstar, dtype=tc.float32, device=self.device).contiguous().reshape(-1)
        assert phi_t.numel() == self.N
        self._check(self.lib.cac_set_state(self.h, _ptr(phi_t), _ptr(u_t), _ptr(p_t)))
        self._keep_state = (phi_t, u_t, p_t)
        return self

    def step(self, n=1):
        self._check(self.lib.cac_step(self.h, int(n)))
        return self

    def volume(self) -> float:
        out = C.c_double()
        self._check(self.lib.cac_volume(self.h, C.byref(out)))
        return out.value

    def sync(self):
        self._check(self.lib.cac_sync(self.h))
        return self

    def fields(self):
        """(phi[N], u[3N], pstar[N]) as new device tensors (stream-ordered)."""
        tc = self.torch
        phi = tc.empty(self.N, dtype=tc.float32, device=self.device)
        u = tc.empty(3 * self.N, dtype=tc.float32, device=self.device)
        ps = tc.empty(self.N, dtype=tc.float32, device=self.device)
        self._check(self.lib.cac_get_fields(self.h, _ptr(phi), _ptr(u), _ptr(ps)))
        return phi, u, ps

    def populations(self):
        f = self.torch.empty(27 * self.N, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.cac_get_populations(self.h, _ptr(f)))
        return f

    def profile_step(self, n):
        """Run n steps with per-kernel HIP events; returns ms per kernel (W, H, P, V), summed."""
        ms = (C.c_double * 4)()
        self._check(self.lib.cac_profile_step(self.h, int(n), ms))
        return list(ms)

    def set_debug(self, poison=False, reverse_order=False):
        """NaN poisoning of never-read data (at the next set_state/load_state) and
        reverse workgroup order (from the next step); results must not change."""
        self._check(self.lib.cac_set_debug(self.h, (CAC_DEBUG_POISON if poison else 0) |
                                           (CAC_DEBUG_REVERSE_ORDER if reverse_order else 0)))
        return self

    def pull_copy_probe(self, reps=20):
        """Milliseconds per launch of the 27-plane pull copy (the collide-stream's
        access pattern without its arithmetic).  Leaves the handle without a state."""
        ms = C.c_double()
        self._check(self.lib.cac_pull_copy_probe(self.h, int(reps), C.byref(ms)))
        return ms.value

    def set_launch(self, bx, by, bz, use_graph=False, phase_tile=0):
        self._check(self.lib.cac_set_launch(self.h, int(bx), int(by), int(bz), int(phase_tile),
                                            int(bool(use_graph))))
        return self

    # -------------------------------------------------------------- checkpoints, test hooks
    def save_state(self):
        """Saved state as a new device byte tensor."""
        nb = C.c_size_t()
        self._check(self.lib.cac_state_bytes(self.h, C.byref(nb)))
        buf = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.cac_save_state(self.h, _ptr(buf), nb.value))
        return buf

    def load_state(self, buf):
        self._check(self.lib.cac_load_state(self.h, _ptr(buf), buf.numel()))
        self._keep_loaded = buf
        return self

    def debug_substep(self, which):
        self._check(self.lib.cac_debug_substep(self.h, int(which)))
        return self

    def debug_buffer(self, which):
        n = {0: 1, 1: 1, 2: 3, 3: 27, 4: 27, 5: 3}[which] * self.N
        out = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.cac_debug_buffer(self.h, int(which), _ptr(out)))
        return out

    # -------------------------------------------------------------- adjoint
    def tape_forward(self, nsteps, K):
        """Advance nsteps steps and record them (checkpoints every K) for tape_backward.
        The last segment is recorded into the reverse sweep's rings; K >= nsteps keeps
        the whole rollout in device memory (about 128 B per node and step), and then
        tape_backward replays nothing."""
        self._check(self.lib.cac_tape_forward(self.h, int(nsteps), int(K)))
        return self

    def tape_backward(self, phibar, want_phi0=True):
        """Reverse sweep seeded with dL/dphi after the recorded steps (device, N).
        Returns (dL/dtheta per wall node as float64, dL/dphi0 as float32 or None)."""
        tc = self.torch
        pb = tc.as_tensor(phibar, dtype=tc.float32, device=self.device).contiguous().reshape(-1)
        assert pb.numel() == self.N
        dth = tc.zeros(max(self.nwall, 1), dtype=tc.float64, device=self.device)
        dphi0 = tc.empty(self.N, dtype=tc.float32, device=self.device) if want_phi0 else None
        self._check(self.lib.cac_tape_backward(self.h, _ptr(pb), _ptr(dth), _ptr(dphi0)))
        self._keep_seed = pb
        return dth[:self.nwall], dphi0

    def loss(self, phi_target):
        """(L, dL/dphi) for L = 1/2 sum_fluid (phi - phi_target)^2 of the current state."""
        tc = self.torch
        tgt = tc.as_tensor(phi_target, dtype=tc.float32, device=self.device).contiguous().reshape(-1)
        seed = tc.empty(self.N, dtype=tc.float32, device=self.device)
        out = C.c_double()
        self._check(self.lib.cac_loss(self.h, _ptr(tgt), _ptr(seed), C.byref(out)))
        return out.value, seed

    def adjoint(self, nsteps, K, phi_target):
        """Forward nsteps from the current state, loss against phi_target, reverse sweep:
        returns (L, dL/dtheta per wall node, float64 device tensor)."""
        tc = self.torch
        tgt = tc.as_tensor(phi_target, dtype=tc.float32, device=self.device).contiguous().reshape(-1)
        dth = tc.zeros(max(self.nwall, 1), dtype=tc.float64, device=self.device)
        out = C.c_double()
        self._check(self.lib.cac_adjoint(self.h, int(nsteps), int(K), _ptr(tgt), C.byref(out), _ptr(dth)))
        return out.value, dth[:self.nwall]


def _autograd_function():
    import torch

    class CACStep(torch.autograd.Function):
        """phi^N = CACStep.apply(theta, phi0, sim, nsteps, K): nsteps coupled steps of `sim`
        from the initial phase field phi0 (N) with contact angles theta (one per wall node).
        The backward pass is the library's reverse sweep (checkpoints every K steps) and
        returns dL/dtheta and dL/dphi0."""

        @staticmethod
        def forward(ctx, theta, phi0, sim, nsteps, K):
            sim.set_contact_angles(theta.detach())
            sim.set_state(phi0.detach())
            sim.tape_forward(nsteps, K)
            ctx.sim = sim
            phi = sim.fields()[0]
            return phi

        @staticmethod
        def backward(ctx, gphi):
            dth, dphi0 = ctx.sim.tape_backward(gphi.detach(), want_phi0=True)
            return dth.to(torch.float32), dphi0, None, None, None

    return CACStep


_CACStep = None


def cac_step_function():
    """The torch.autograd.Function wrapping a recorded rollout (built on first use)."""
    global _CACStep
    if _CACStep is None:
        _CACStep = _autograd_function()
    return _CACStep


def from_workload(w, device=None) -> Sim:
    """Sim with the geometry, angles and initial phase field of a workload."""
    s = Sim(w.shape, w.params, device=device)
    s.set_geometry(w.solid, w.theta)
    s.set_state(w.phi0)
    return s


def pi_half() -> float:
    return math.pi / 2


class Batch:
    """Many independent domains advanced together by the persistent batched kernels."""

    def __init__(self, workloads, device=None, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libcac needs a GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._buffers = []

        def _alloc(nbytes, user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self._buffers.append(t)
            return t.data_ptr()

        self._alloc_cb = ALLOC_FN(_alloc)
        self.shapes = [tuple(w.shape) for w in workloads]
        n = len(workloads)
        descs = (DomainDesc * n)()
        keep = []
        for k, w in enumerate(workloads):
            solid = np.ascontiguousarray(w.solid, dtype=np.uint8).reshape(-1)
            th = np.ascontiguousarray(w.theta, dtype=np.float32).reshape(-1)
            phi = torch.as_tensor(w.phi0, dtype=torch.float32, device=self.device).contiguous().reshape(-1)
            keep += [solid, th, phi]
            descs[k].nx, descs[k].ny, descs[k].nz = w.shape
            descs[k].params = make_params(w.params)
            descs[k].solid = solid.ctypes.data_as(C.c_void_p)
            descs[k].theta_rad = th.ctypes.data_as(C.c_void_p)
            descs[k].d_phi0 = C.c_void_p(phi.data_ptr())
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.cac_batch_init(C.byref(h), n, descs, self._alloc_cb, None, C.c_void_p(self.stream.cuda_stream))
        if st != CAC_OK:
            raise CacError(st, "cac_batch_init: " + self.lib.cac_status_string(st).decode())
        self.h = h
        self.ndom = n
        self.sync()
        del keep

    def _check(self, st):
        if st == CAC_OK:
            return
        buf = C.create_string_buffer(512)
        self.lib.cac_batch_last_error(self.h, buf, 512)
        raise CacError(st, self.lib.cac_status_string(st).decode() + ": " + buf.value.decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.cac_batch_destroy(self.h)
            self.h = None
            self._buffers.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, bx, by, bz, phase_tile, grid_mult, order, use_graph=True):
        self._check(self.lib.cac_batch_set_schedule(self.h, bx, by, bz, phase_tile, grid_mult, order, int(use_graph)))
        return self

    def schedule(self):
        out = (C.c_int * 7)()
        self._check(self.lib.cac_batch_get_schedule(self.h, out))
        return tuple(out)

    def autotune(self, cache_path=None, trial_steps=5):
        ms = C.c_double()
        self._check(self.lib.cac_batch_autotune(self.h, None if cache_path is None else cache_path.encode(),
                                                int(trial_steps), C.byref(ms)))
        return ms.value

    def step(self, n=1):
        self._check(self.lib.cac_batch_step(self.h, int(n)))
        return self

    def sync(self):
        self._check(self.lib.cac_batch_sync(self.h))
        return self

    def volumes(self):
        out = (C.c_double * self.ndom)()
        self._check(self.lib.cac_batch_volume(self.h, out))
        return list(out)

    def fields(self, k):
        tc = self.torch
        nx, ny, nz = self.shapes[k]
        N = nx * ny * nz
        phi = tc.empty(N, dtype=tc.float32, device=self.device)
        u = tc.empty(3 * N, dtype=tc.float32, device=self.device)
        ps = tc.empty(N, dtype=tc.float32, device=self.device)
        self._check(self.lib.cac_batch_get_fields(self.h, int(k), _ptr(phi), _ptr(u), _ptr(ps)))
        return phi, u, ps

    def info(self):
        n, tot, fl = C.c_int(), C.c_longlong(), C.c_longlong()
        self._check(self.lib.cac_batch_info(self.h, C.byref(n), C.byref(tot), C.byref(fl)))
        return n.value, tot.value, fl.value

    def profile_step(self, n):
        ms = (C.c_double * 4)()
        self._check(self.lib.cac_batch_profile(self.h, int(n), ms))
        return list(ms)
