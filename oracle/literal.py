"""Literal full-tensor FP64 implementation of the coupled CAC step in PyTorch
(CPU), for brute-force cross-checks on tiny grids and, through autograd, the
exact discrete adjoint of the step.

TEST INFRASTRUCTURE ONLY.  Written independently of ``cac_oracle.c`` (its own
lattice tables and wall geometry) in whole-array form: periodic shifts with
``torch.roll``, Hermite tensors H2 (27x3x3) and H3 (27x3x3x3) contracted with
``einsum``.  Same readings as the C oracle (order W -> H -> P -> V, Jacobi
ghosts, A2 as the moment of f - f^eq + S/2, forces as accelerations,
bounce-back, zero advective flux at wall faces, the wall compressive-flux
switch, and the switch ``collision`` = 1 that takes A2 in the gradient form
of Eq. (15) from the new velocity field, a solid neighbour holding the mirror
image -u of the node).  Non-smooth points (minmod, upwind, the chi band, the normal guard,
lambda_s at 0, the cot regularisation) follow the branch the forward pass
takes; ``torch.where`` selections and guarded square roots keep gradients
finite.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np
import torch

DT = torch.float64


def _velocities():
    # all of {-1,0,1}^3, rest first, then opposite pairs by |c|^2 (not the C oracle's order)
    vs = [c for c in itertools.product((-1, 0, 1), repeat=3) if c != (0, 0, 0)]
    vs.sort(key=lambda c: (sum(abs(v) for v in c), c))
    out = [(0, 0, 0)]
    seen = set()
    for c in vs:
        if c in seen:
            continue
        m = tuple(-v for v in c)
        out += [c, m]
        seen |= {c, m}
    return out


C_LIST = _velocities()
CV = torch.tensor(C_LIST, dtype=DT)                            # (27, 3)
W1D = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
WV = torch.tensor([W1D[a] * W1D[b] * W1D[c] for a, b, c in C_LIST], dtype=DT)
OPP = [C_LIST.index(tuple(-v for v in c)) for c in C_LIST]
CS2 = 1.0 / 3.0
I3 = torch.eye(3, dtype=DT)
H2 = torch.einsum("ia,ib->iab", CV, CV) - CS2 * I3              # Eq. (12)
H3 = (torch.einsum("ia,ib,ig->iabg", CV, CV, CV)
      - CS2 * (torch.einsum("ia,bg->iabg", CV, I3) + torch.einsum("ib,ag->iabg", CV, I3)
               + torch.einsum("ig,ab->iabg", CV, I3)))          # Eq. (13)


def shift(a, c):
    """Field value at x + c (periodic), for arrays indexed [..., z, y, x]."""
    return torch.roll(a, shifts=(-int(c[2]), -int(c[1]), -int(c[0])), dims=(-3, -2, -1))


def grad_iso(psi):
    """Eq. (22)."""
    g = torch.zeros((3,) + psi.shape, dtype=DT)
    for i, c in enumerate(C_LIST):
        if i == 0:
            continue
        v = shift(psi, c) * (WV[i] / CS2)
        for d in range(3):
            if c[d]:
                g[d] = g[d] + c[d] * v
    return g


def lap_iso(psi):
    """Eq. (23)."""
    s = torch.zeros_like(psi)
    for i, c in enumerate(C_LIST):
        if i:
            s = s + WV[i] * shift(psi, c)
    return (2.0 / CS2) * (s - (1.0 - WV[0]) * psi)


def _safe_sqrt(x, ok):
    return torch.sqrt(torch.where(ok, x, torch.ones_like(x)))


class Geometry:
    """Wall nodes of a mask, computed here from the definitions (Sec. II B)."""

    def __init__(self, solid3):
        self.solid = torch.as_tensor(solid3, dtype=torch.bool)
        nz, ny, nx = self.solid.shape
        s = self.solid.numpy()
        walls, donors, normals = [], [], []
        for z, y, x in zip(*np.nonzero(s)):
            fl = []
            for q, c in enumerate(C_LIST):
                if q == 0:
                    continue
                if not s[(z + c[2]) % nz, (y + c[1]) % ny, (x + c[0]) % nx]:
                    fl.append(q)
            if not fl:
                continue
            nt = [0.0, 0.0, 0.0]
            for q in fl:
                k = sum(abs(v) for v in C_LIST[q])
                for d in range(3):
                    nt[d] -= C_LIST[q][d] / k   # weights 1, 1/2, 1/3, Eq. (37)
            nn = math.sqrt(sum(v * v for v in nt))
            walls.append((z, y, x))
            if nn < 1e-12:
                donors.append(-1)
                normals.append((0.0, 0.0, 0.0))
                continue
            n = [v / nn for v in nt]
            # alignment score Eq. (39); exact ties resolved towards the first velocity in the
            # order (0,0,0),(1,0,0),(-1,0,0),... that the C oracle and the library also use
            best, bq = None, None
            for q in sorted(fl, key=lambda q: _canon_index(C_LIST[q])):
                c = C_LIST[q]
                num = -sum(c[d] * nt[d] for d in range(3)) * 6.0
                sc = round(num) / math.sqrt(sum(abs(v) for v in c))
                if best is None or sc > best + 1e-9:
                    best, bq = sc, q
            donors.append(bq)
            normals.append(tuple(n))
        self.walls = walls
        self.donor = donors
        self.normal = torch.tensor(normals, dtype=DT).reshape(-1, 3)


_CANON = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
          (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1), (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
          (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]


def _canon_index(c):
    return _CANON.index(tuple(c))


def ghost_update(p, geo, theta_w, phi_in):
    """W (Sec. II B): new ghosts from the donors (Jacobi: phi_in holds the previous
    ghosts).  Returns phi_hat and the wall compressive flux (3, nz, ny, nx)."""
    nz, ny, nx = phi_in.shape
    G = grad_iso(phi_in)
    phi_hat = phi_in.clone()
    aw = torch.zeros((3,) + phi_in.shape, dtype=DT)
    ks = [k for k, q in enumerate(geo.donor) if q >= 0]
    if not ks:
        return phi_hat, aw
    zs = torch.tensor([geo.walls[k][0] for k in ks])
    ys = torch.tensor([geo.walls[k][1] for k in ks])
    xs = torch.tensor([geo.walls[k][2] for k in ks])
    cq = torch.tensor([C_LIST[geo.donor[k]] for k in ks], dtype=torch.long)
    fz, fy, fx = (zs + cq[:, 2]) % nz, (ys + cq[:, 1]) % ny, (xs + cq[:, 0]) % nx
    nw = geo.normal[ks]
    phif = phi_in[fz, fy, fx]
    Gf = G[:, fz, fy, fx].T                                          # (nb, 3)
    Gpar = Gf - (Gf * nw).sum(1, keepdim=True) * nw                  # Eq. (42)
    t2 = (Gpar * Gpar).sum(1)
    t = torch.where(t2 > 0, _safe_sqrt(t2, t2 > 0), torch.zeros_like(t2))
    th = theta_w[ks]
    thc = math.pi - th                                               # Eq. (43)
    sn, cs = torch.sin(thc), torch.cos(thc)
    reg = sn.abs() < p["sin_tol"]
    cot = torch.where(reg, torch.sign(cs) * p["cot_max"], cs / torch.where(reg, torch.ones_like(sn), sn))
    dn = -t * cot                                                    # Eq. (44)
    Gc = Gpar + dn[:, None] * nw                                     # Eq. (45)
    l2 = 4.0 * phif * (1.0 - phif)
    lam = torch.where(l2 > 0, _safe_sqrt(l2, l2 > 0), torch.zeros_like(l2))  # Eq. (47)
    g = phif + lam * (Gc * (-cq.to(DT))).sum(1)                      # Eq. (46)
    phi_hat = phi_hat.index_put((zs, ys, xs), g)
    if p.get("wall_compression", 1):
        c2 = (Gc * Gc).sum(1)
        ok = c2 > p["eps_n"] ** 2
        inv = torch.where(ok, 1.0 / _safe_sqrt(c2, ok), torch.zeros_like(c2))
        av = (g * (1.0 - g) * inv)[:, None] * Gc
        for d in range(3):
            aw[d] = aw[d].index_put((zs, ys, xs), av[:, d])
    return phi_hat, aw


def feq(ps, u):
    """Eq. (11) with the full Hermite tensors; u has shape (3, ...)."""
    uu = torch.einsum("a...,b...->ab...", u, u)
    uuu = torch.einsum("a...,b...,g...->abg...", u, u, u)
    cu = torch.einsum("ia,a...->i...", CV, u)
    return WV.view(-1, *([1] * ps.dim())) * (ps + cu / CS2 + torch.einsum("iab,ab...->i...", H2, uu) / (2 * CS2 ** 2)
                                             + torch.einsum("iabg,abg...->i...", H3, uuu) / (6 * CS2 ** 3))


def guo(u, a):
    """Eq. (17) with the forcing as an acceleration."""
    cu = torch.einsum("ia,a...->i...", CV, u)
    ca = torch.einsum("ia,a...->i...", CV, a)
    ua = (u * a).sum(0)
    return WV.view(-1, *([1] * ua.dim())) * ((ca - ua) / CS2 + cu * ca / CS2 ** 2)


def fneq_reg(u, A2):
    """Eqs. (14), (16)."""
    A3 = (torch.einsum("a...,bg...->abg...", u, A2) + torch.einsum("b...,ag...->abg...", u, A2)
          + torch.einsum("g...,ab...->abg...", u, A2))
    return WV.view(-1, *([1] * (A2.dim() - 2))) * (torch.einsum("iab,ab...->i...", H2, A2) / (2 * CS2 ** 2)
                                                   + torch.einsum("iabg,abg...->i...", H3, A3) / (6 * CS2 ** 3))


def hydro(p, solid, phi_hat, f):
    """H (Sec. II A): collision at the fluid nodes, then pull streaming with
    halfway bounce-back.  f has shape (27, nz, ny, nx) and is read on fluid
    nodes only; the outputs are zero on solid nodes."""
    shp = phi_hat.shape
    N = phi_hat.numel()
    G = grad_iso(phi_hat).reshape(3, N)
    L = lap_iso(phi_hat).reshape(N)
    fl3 = ~solid
    idx = torch.nonzero(fl3.reshape(N)).squeeze(1)
    ph = phi_hat.reshape(N)[idx]
    Gf = G[:, idx]
    Lf = L[idx]
    ff = f.reshape(27, N)[:, idx]
    beta, kphi = 12.0 * p["sigma"] / p["delta"], 1.5 * p["sigma"] * p["delta"]
    mu_phi = 4.0 * beta * (ph - 1.0) * ph * (ph - 0.5) - kphi * Lf    # Eq. (19)
    Fs = mu_phi * Gf
    rho = p["rho_g"] + (p["rho_l"] - p["rho_g"]) * ph                  # Eqs. (8)-(10)
    mu = p["rho_g"] * p["nu_g"] + (p["rho_l"] * p["nu_l"] - p["rho_g"] * p["nu_g"]) * ph
    nu = mu / rho
    omega = 1.0 / (0.5 + nu / CS2)
    grho = (p["rho_l"] - p["rho_g"]) * Gf
    ps = ff.sum(0)
    j = CV.T @ ff
    Fp = -ps * CS2 * grho                                              # Eq. (20)
    gv = torch.tensor(p["g"], dtype=DT).view(3, 1)
    Fext = (rho - p["rho_g"]) * gv
    a1 = (Fs + Fp + Fext) / rho
    u1 = j + 0.5 * a1
    Pi = torch.einsum("ia,ib,in->abn", CV, CV, ff - feq(ps, u1))       # Eq. (21)
    Fnu = -(nu * omega / CS2) * torch.einsum("abn,bn->an", Pi, grho)
    a = a1 + Fnu / rho
    u = j + 0.5 * a                                                    # Eq. (7)
    fe = feq(ps, u)
    S = guo(u, a)
    u_all = torch.zeros((3, N), dtype=DT).index_copy(1, idx, u).reshape((3,) + tuple(shp))
    if p.get("collision", 0) == 1:
        # gradient form, Eq. (15): A2_ab = -(c_s^2/omega)(d_a u_b + d_b u_a), the
        # derivatives by Eq. (22) on the new velocity field; a solid neighbour holds
        # the mirror image -u of the node, i.e. the stencil of the field that is zero
        # on solids minus u(x) times the stencil of the solid indicator
        gs = grad_iso(solid.to(DT)).reshape(3, N)[:, idx]
        D = torch.stack([grad_iso(u_all[c]).reshape(3, N)[:, idx] - u[c] * gs for c in range(3)], 1)  # D[b, a] = d_b u_a
        A2 = -(CS2 / omega) * (D + D.transpose(0, 1))
    else:
        A2 = torch.einsum("ia,ib,in->abn", CV, CV, ff - fe + 0.5 * S)
    fp = fe + 0.5 * S + (1.0 - omega) * fneq_reg(u, A2)                # Eq. (3)
    fpost = torch.zeros((27, N), dtype=DT).index_copy(1, idx, fp).reshape((27,) + tuple(shp))
    ps_all = torch.zeros(N, dtype=DT).index_copy(0, idx, ps).reshape(shp)
    fnew = []
    for i, c in enumerate(C_LIST):
        mc = tuple(-v for v in c)
        src_solid = shift(solid, mc)
        fnew.append(torch.where(src_solid, fpost[OPP[i]], shift(fpost[i], mc)))
    fnew = torch.stack(fnew)
    fnew = torch.where(fl3, fnew, torch.zeros_like(fnew))
    return fpost, fnew, u_all, ps_all


def _minmod(a, b):
    """Eq. (32); ties |a| = |b| pick a."""
    pick = torch.where(a.abs() <= b.abs(), a, b)
    return torch.where(a * b > 0, pick, torch.zeros_like(a))


def phase(p, solid, phi_hat, u, aw):
    """P (Sec. II A 1), Eq. (28)."""
    kappa = 4.0 * p["D"] / p["delta"]
    fl = ~solid
    div_a = torch.zeros_like(phi_hat)
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        em = [-v for v in e]
        e2 = [2 * v for v in e]
        phn, php, phpp = shift(phi_hat, em), shift(phi_hat, e), shift(phi_hat, e2)
        s_here = _minmod(phi_hat - phn, php - phi_hat)
        s_next = _minmod(php - phi_hat, phpp - php)
        uf = 0.5 * (u[d] + shift(u[d], e))
        up = torch.where(uf >= 0, phi_hat + 0.5 * s_here, php - 0.5 * s_next)
        open_face = fl & shift(fl, e)
        F = torch.where(open_face, uf * up, torch.zeros_like(uf))     # flux through x + e_d/2
        div_a = div_a + F - shift(F, em)
    L = lap_iso(phi_hat)
    G = grad_iso(phi_hat)
    g2 = (G * G).sum(0)
    ok = g2 > p["eps_n"] ** 2
    inv = torch.where(ok, 1.0 / _safe_sqrt(g2, ok), torch.zeros_like(g2))
    a = phi_hat * (1.0 - phi_hat) * inv * G
    a = torch.where(fl, a, aw)
    div_c = torch.zeros_like(phi_hat)
    for i, c in enumerate(C_LIST):
        if i:
            div_c = div_c + (WV[i] / CS2) * sum(c[d] * shift(a[d], c) for d in range(3) if c[d])
    ps = phi_hat - div_a + p["D"] * L - kappa * div_c
    return torch.where(fl, ps, phi_hat)


def volume(p, solid, phistar, M_target):
    """V (Sec. II C)."""
    fl = ~solid
    eps = p["eps_phi"]
    Ms = torch.where(fl, phistar, torch.zeros_like(phistar)).sum()
    band = fl & (phistar > eps) & (phistar < 1.0 - eps)
    chi = torch.where(band, phistar * (1.0 - phistar), torch.zeros_like(phistar))
    W = chi.sum()
    if not p.get("volume_correction", 1) or float(W.detach()) <= 0.0:
        return phistar
    lam = (M_target - Ms) / W
    return phistar + lam * chi


def _pdict(params):
    if isinstance(params, dict):
        return dict(params)
    return dataclasses.asdict(params)


class LiteralSim:
    """Whole-array FP64 state: f (27, nz, ny, nx) post-streaming, phi (nz, ny, nx)
    with the previous ghosts on wall nodes, and the target mass of Eq. (50)."""

    def __init__(self, shape, solid, params, phi0, pstar0=None, u0=None):
        nx, ny, nz = shape
        self.shape = tuple(shape)
        self.p = _pdict(params)
        self.solid = torch.as_tensor(np.asarray(solid).reshape(nz, ny, nx).astype(bool))
        self.geo = Geometry(self.solid.numpy())
        fl = ~self.solid
        self.phi = torch.as_tensor(np.asarray(phi0, dtype=np.float64).reshape(nz, ny, nx)).clone()
        ps = torch.zeros((nz, ny, nx), dtype=DT) if pstar0 is None else \
            torch.as_tensor(np.asarray(pstar0, dtype=np.float64).reshape(nz, ny, nx))
        u = torch.zeros((3, nz, ny, nx), dtype=DT) if u0 is None else \
            torch.as_tensor(np.asarray(u0, dtype=np.float64).reshape(3, nz, ny, nx))
        self.f = torch.where(fl, feq(ps, u), torch.zeros((27, nz, ny, nx), dtype=DT))
        self.M_target = torch.where(fl, self.phi, torch.zeros_like(self.phi)).sum().detach()
        self.u = torch.zeros((3, nz, ny, nx), dtype=DT)
        self.pstar = torch.zeros((nz, ny, nx), dtype=DT)

    def wall_theta_from_field(self, theta_field):
        """Per-wall-node angles (geometry order, ascending node index) from an
        N-array with x fastest."""
        nx, ny, nz = self.shape
        t3 = np.asarray(theta_field, dtype=np.float64).reshape(nz, ny, nx)
        return torch.tensor([t3[z, y, x] for (z, y, x) in self.geo.walls], dtype=DT)

    def wall_linear_index(self):
        nx, ny, nz = self.shape
        return np.array([x + nx * (y + ny * z) for (z, y, x) in self.geo.walls], dtype=np.int64)

    def step(self, theta_w, n=1):
        """n steps W -> H -> P -> V with per-wall-node angles theta_w (radians)."""
        for _ in range(n):
            phi_hat, aw = ghost_update(self.p, self.geo, theta_w, self.phi)
            fpost, fnew, u, ps = hydro(self.p, self.solid, phi_hat, self.f)
            phistar = phase(self.p, self.solid, phi_hat, u, aw)
            self.phi = volume(self.p, self.solid, phistar, self.M_target)
            self.f = fnew
            self.u = u
            self.pstar = ps
        return self


def rollout_grad(shape, solid, params, phi0, theta_w, nsteps, phi_target):
    """Loss L = 1/2 sum_fluid (phi^N - phi_target)^2 after nsteps steps from phi0
    (populations at rest, p* = 0) and its exact discrete gradients by autograd:
    returns (L, dL/dtheta per wall node, dL/dphi0 on all nodes).  The target
    volume of the correction is the fluid sum of phi0, so dL/dphi0 includes its
    path through M_target."""
    sim = LiteralSim(shape, solid, params, phi0)
    th = torch.as_tensor(np.asarray(theta_w, dtype=np.float64)).clone().requires_grad_(True)
    p0 = sim.phi.detach().clone().requires_grad_(True)
    fl = ~sim.solid
    sim.phi = p0
    sim.M_target = torch.where(fl, p0, torch.zeros_like(p0)).sum()
    sim.step(th, nsteps)
    nx, ny, nz = shape
    tgt = torch.as_tensor(np.asarray(phi_target, dtype=np.float64).reshape(nz, ny, nx))
    L = 0.5 * (torch.where(fl, sim.phi - tgt, torch.zeros_like(tgt)) ** 2).sum()
    gth, gphi = torch.autograd.grad(L, [th, p0])
    return float(L.detach()), gth.numpy(), gphi.numpy().reshape(-1)
