// step_device.hpp -- device bodies of the coupled step, shared by the
// single-lattice kernels (kernels.hip) and the batched persistent kernels
// (batch.hip).  Included only by HIP sources of libcac.
#pragma once

#include "cac_internal.hpp"

namespace cac {

// ------------------------------------------------------------------ helpers

// Hardware dispatch sends workgroup b to XCD b % 8.  Re-number so that XCD k
// owns a contiguous block of logical tiles (halo rows stay in its L2).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n)
{
    const uint32_t k = b & 7u, j = b >> 3, q = n >> 3, r = n & 7u;
    return k * q + (k < r ? k : r) + j;
}

struct Node {
    int x, y, z;
    bool in;
};

__device__ __forceinline__ Node tile_node(const Grid &g, const Tiling &t, uint32_t tile)
{
    const uint32_t txy = (uint32_t)t.tx * (uint32_t)t.ty;
    const uint32_t tz = tile / txy;
    const uint32_t r = tile - tz * txy;
    const uint32_t ty = r / (uint32_t)t.tx;
    const uint32_t tx = r - ty * (uint32_t)t.tx;
    const int tid = threadIdx.x;
    const int lx = tid % t.bx;
    const int ly = (tid / t.bx) % t.by;
    const int lz = tid / (t.bx * t.by);
    Node nd;
    nd.x = (int)tx * t.bx + lx;
    nd.y = (int)ty * t.by + ly;
    nd.z = (int)tz * t.bz + lz;
    nd.in = nd.x < g.nx && nd.y < g.ny && nd.z < g.nz;
    return nd;
}

// Periodic neighbour offsets along each axis: o[0] = coordinate - 1,
// o[1] = coordinate, o[2] = coordinate + 1 (wrapped), already scaled by the
// axis stride.
struct Offs {
    uint32_t x[3], y[3], z[3];
};

__host__ __device__ __forceinline__ Offs node_offsets(const Grid &g, int x, int y, int z)
{
    Offs o;
    o.x[0] = (uint32_t)(x ? x - 1 : g.nx - 1);
    o.x[1] = (uint32_t)x;
    o.x[2] = (uint32_t)(x + 1 < g.nx ? x + 1 : 0);
    o.y[0] = (uint32_t)(y ? y - 1 : g.ny - 1) * (uint32_t)g.nx;
    o.y[1] = (uint32_t)y * (uint32_t)g.nx;
    o.y[2] = (uint32_t)(y + 1 < g.ny ? y + 1 : 0) * (uint32_t)g.nx;
    o.z[0] = (uint32_t)(z ? z - 1 : g.nz - 1) * g.nxny;
    o.z[1] = (uint32_t)z * g.nxny;
    o.z[2] = (uint32_t)(z + 1 < g.nz ? z + 1 : 0) * g.nxny;
    return o;
}

template <int DX, int DY, int DZ>
__host__ __device__ __forceinline__ uint32_t at(const Offs &o)
{
    return o.x[DX + 1] + o.y[DY + 1] + o.z[DZ + 1];
}

// 1-D smoothing weights of the D3Q27 tensor-product weights: w_i = t(cx)t(cy)t(cz)/216,
// t(0) = 4, t(+-1) = 1.
__host__ __device__ constexpr float tw(int d) { return d == 0 ? 4.0f : 1.0f; }

// Isotropic gradient (Eq. (22)) and Laplacian (Eq. (23)) from a 3x3x3 stencil
// s[k], k = (dz+1)*9 + (dy+1)*3 + (dx+1), in tensor-product form on the
// differences d = s - s(0,0,0) (exact in FP32 for neighbouring values, so the
// Laplacian does not lose digits to cancellation):
//   grad_x = sum_{dy,dz} t(dy) t(dz) [d(+1,dy,dz) - d(-1,dy,dz)] / 72
//   lap    = sum t(dx) t(dy) t(dz) d / 36
__host__ __device__ __forceinline__ void stencil_grad_lap(const float (&s)[27], float &gx, float &gy, float &gz, float &lap)
{
    const float c0 = s[13];
    float S[9];  // x-smoothed differences at (dy, dz)
    gx = 0.f;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const float m = s[3 * j] - c0, c = s[3 * j + 1] - c0, p = s[3 * j + 2] - c0;
        S[j] = m + 4.0f * c + p;
        const int dy = j % 3 - 1, dz = j / 3 - 1;
        gx += tw(dy) * tw(dz) * (p - m);
    }
    gx *= (1.0f / 72.0f);
    gy = 0.f;
    gz = 0.f;
    float l = 0.f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) gy += tw(dz - 1) * (S[dz * 3 + 2] - S[dz * 3 + 0]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) gz += tw(dy - 1) * (S[6 + dy] - S[0 + dy]);
#pragma unroll
    for (int j = 0; j < 9; ++j) l += tw(j % 3 - 1) * tw(j / 3 - 1) * S[j];
    gy *= (1.0f / 72.0f);
    gz *= (1.0f / 72.0f);
    lap = l * (1.0f / 36.0f);
}

// Hermite coefficients of a population set f_i = w_i [ps + 3 c.b + 4.5 H2:C2 + 4.5 H3:C3]
// (c_s^2 = 1/3).  C3 is symmetric; only the 7 components that D3Q27 carries
// (H3_aaa = 0 on the lattice) are stored.
struct Herm {
    float ps, bx, by, bz;
    float xx, yy, zz, xy, xz, yz, tr3;  // C2 and trace(C2)/3
    float xxy, xxz, yyx, yyz, zzx, zzy, xyz;
};

// Even and odd parts of f_i for the pair (i, opp(i)): f_i = E + O, f_opp = E - O.
template <int I>
__device__ __forceinline__ void herm_pair(const Herm &h, float &E, float &O)
{
    constexpr float cx = (float)Lat::cx[I], cy = (float)Lat::cy[I], cz = (float)Lat::cz[I];
    constexpr float w = Lat::w(I);
    const float ccc = cx * cx * h.xx + cy * cy * h.yy + cz * cz * h.zz +
                      2.0f * (cx * cy * h.xy + cx * cz * h.xz + cy * cz * h.yz);
    E = w * (h.ps + 4.5f * (ccc - h.tr3));
    const float cb = cx * h.bx + cy * h.by + cz * h.bz;
    constexpr float hx = cx * cx - 1.0f / 3.0f, hy = cy * cy - 1.0f / 3.0f, hz = cz * cz - 1.0f / 3.0f;
    const float h3 = 3.0f * (hx * (cy * h.xxy + cz * h.xxz) + hy * (cx * h.yyx + cz * h.yyz) +
                             hz * (cx * h.zzx + cy * h.zzy)) +
                     6.0f * cx * cy * cz * h.xyz;
    O = w * (3.0f * cb + 4.5f * h3);
}

// Single equilibrium population, Eq. (11): w [ps + 3 cu + 4.5 ((cu)^2 - u^2/3) + 4.5 ((cu)^3 - cu u^2)]
template <int I>
__device__ __forceinline__ float feq_one(float ps, float ux, float uy, float uz)
{
    constexpr float cx = (float)Lat::cx[I], cy = (float)Lat::cy[I], cz = (float)Lat::cz[I];
    const float cu = cx * ux + cy * uy + cz * uz;
    const float uu = ux * ux + uy * uy + uz * uz;
    return Lat::w(I) * (ps + 3.0f * cu + 4.5f * (cu * cu - uu * (1.0f / 3.0f)) + 4.5f * (cu * cu * cu - cu * uu));
}

// ------------------------------------------------------------------ W: ghosts

// Ghost value of wall node b (Sec. II B, Eqs. (36)-(47)), one thread per
// wall node.  Donor x_f = b + c_q (Eq. (41)); phi_f and the isotropic
// gradient G at x_f (Eq. (22)) from fluid values of the current buffer and,
// at wall points of the stencil, the previous ghosts in the other buffer
// (Jacobi).  With the unit wall normal n_w (Eq. (38)), the tangential gradient
// G_par = G - (G.n_w) n_w (Eq. (42)) and theta_c = pi - theta (Eq. (43)), the
// corrected gradient of Eqs. (44)-(45) is G_c = G_par - |G_par| cot(theta_c) n_w
// and the extrapolation of Eq. (46) along r_fs = -c_q reads
//   phi_g = phi_f - lambda_s [ c_q.G_par - |G_par| cot(theta_c) (c_q.n_w) ],
// lambda_s of Eq. (47).  Reads only fluid data and old ghosts, writes only b.
__device__ __forceinline__ void ghost_node(const Grid &g, const DevParams &p, int k, const int32_t *__restrict__ widx,
                                           const uint8_t *__restrict__ wq, const float *__restrict__ wn,
                                           const float *__restrict__ theta, float *phi_cur,
                                           const float *__restrict__ phi_old, const uint32_t *__restrict__ nbr,
                                           float *__restrict__ a)
{
    const int q = wq[k];
    if (q >= 27) return;  // skipped node: ghost keeps its value
    const uint32_t b = (uint32_t)widx[k];
    const int bx = (int)(b % (uint32_t)g.nx);
    const int by = (int)((b / (uint32_t)g.nx) % (uint32_t)g.ny);
    const int bz = (int)(b / g.nxny);
    int cxq = 0, cyq = 0, czq = 0;
    static_for<27>([&](auto I) {
        if (q == I) {
            cxq = Lat::cx[I];
            cyq = Lat::cy[I];
            czq = Lat::cz[I];
        }
    });
    int fx = bx + cxq, fy = by + cyq, fz = bz + czq;
    fx = fx < 0 ? fx + g.nx : (fx >= g.nx ? fx - g.nx : fx);
    fy = fy < 0 ? fy + g.ny : (fy >= g.ny ? fy - g.ny : fy);
    fz = fz < 0 ? fz + g.nz : (fz >= g.nz ? fz - g.nz : fz);
    const Offs o = node_offsets(g, fx, fy, fz);
    const uint32_t m = nbr[at<0, 0, 0>(o)];
    float s[27];
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        constexpr int dx = kk % 3 - 1, dy = (kk / 3) % 3 - 1, dz = kk / 9 - 1;
        constexpr int li = Lat::idx(dx, dy, dz);
        const uint32_t id = at<dx, dy, dz>(o);
        s[kk] = ((m >> li) & 1u) ? phi_old[id] : phi_cur[id];
    });
    float gx, gy, gz, lap;
    stencil_grad_lap(s, gx, gy, gz, lap);
    const float phif = s[13];
    const float nx = wn[3 * k], ny = wn[3 * k + 1], nz = wn[3 * k + 2];
    const float gn = gx * nx + gy * ny + gz * nz;
    const float px = gx - gn * nx, py = gy - gn * ny, pz = gz - gn * nz;  // G_par
    const float t = sqrtf(px * px + py * py + pz * pz);
    const float thc = 3.14159265358979f - theta[k];
    float sn, cs;
    sincosf(thc, &sn, &cs);
    // cot(theta_c), replaced by +-cot_max where |sin(theta_c)| < sin_tol
    const float cot = (fabsf(sn) < p.sin_tol) ? copysignf(p.cot_max, cs) : cs / sn;
    const float tc = t * cot;
    const float cq_par = (float)cxq * px + (float)cyq * py + (float)czq * pz;
    const float cq_n = (float)cxq * nx + (float)cyq * ny + (float)czq * nz;
    const float l2 = 4.0f * phif * (1.0f - phif);
    const float lam = p.ghost_lambda ? sqrtf(l2 > 0.0f ? l2 : 0.0f) : 1.0f;
    const float gv = phif - lam * (cq_par - tc * cq_n);
    phi_cur[b] = gv;
    if (p.wall_compression) {
        const float cgx = px - tc * nx, cgy = py - tc * ny, cgz = pz - tc * nz;  // G_c
        const float c2 = cgx * cgx + cgy * cgy + cgz * cgz;
        float ax = 0.f, ay = 0.f, az = 0.f;
        if (c2 > p.eps_n2) {
            const float sc = gv * (1.0f - gv) * rsqrtf(c2);
            ax = sc * cgx;
            ay = sc * cgy;
            az = sc * cgz;
        }
        a[b] = ax;
        a[g.N + b] = ay;
        a[2u * g.N + b] = az;
    }
}

// 1/x: the hardware reciprocal (1 ulp) on the device, a division on the host.
__host__ __device__ __forceinline__ float fast_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// Pull of the populations that stream into node n (Sec. II A): f_i(x) =
// f*_i(x - c_i), or f*_opp(i)(x) when x - c_i is solid (halfway bounce-back),
// taken pair by pair (i, opp(i) = i + 1).  NTL: non-temporal loads (each
// population is read once per step).
template <bool NTL>
__device__ __forceinline__ void pull_populations(const Grid &g, const Offs &o, uint32_t n, uint32_t m,
                                                 const float *__restrict__ fin, float (&f)[27])
{
    const uint32_t N = g.N;
    auto ld = [&](uint32_t k) {
        if constexpr (NTL)
            return __builtin_nontemporal_load(&fin[k]);
        else
            return fin[k];
    };
    f[0] = ld(n);
    static_for<13>([&](auto P) {
        constexpr int i = 2 * P + 1;
        const uint32_t src_i = at<Lat::cx[i + 1], Lat::cy[i + 1], Lat::cz[i + 1]>(o);
        f[i] = ld(((m >> (i + 1)) & 1u) ? (uint32_t)(i + 1) * N + n : (uint32_t)i * N + src_i);
        const uint32_t src_o = at<Lat::cx[i], Lat::cy[i], Lat::cz[i]>(o);
        f[i + 1] = ld(((m >> i) & 1u) ? (uint32_t)i * N + n : (uint32_t)(i + 1) * N + src_o);
    });
}

// Moments p* = sum f, j = sum f c, P = sum f c c (Eqs. (6)-(7)) over the opposite
// pairs: with s = f_i + f_opp and d = f_i - f_opp, j takes +-d and P takes s.
// mom = (p*, j_x, j_y, j_z, P_xx, P_yy, P_zz, P_xy, P_xz, P_yz), started at
// (f_0, 0, ...) and updated pair by pair in the order i = 1, 3, ..., 25.
template <int I>
__host__ __device__ __forceinline__ void pair_moment_add(float fi, float fo, float (&mom)[10])
{
    constexpr int cx = Lat::cx[I], cy = Lat::cy[I], cz = Lat::cz[I];
    const float sm = fi + fo, df = fi - fo;
    mom[0] += sm;
    if constexpr (cx != 0) { mom[1] += (float)cx * df; mom[4] += sm; }
    if constexpr (cy != 0) { mom[2] += (float)cy * df; mom[5] += sm; }
    if constexpr (cz != 0) { mom[3] += (float)cz * df; mom[6] += sm; }
    if constexpr (cx * cy != 0) mom[7] += (float)(cx * cy) * sm;
    if constexpr (cx * cz != 0) mom[8] += (float)(cx * cz) * sm;
    if constexpr (cy * cz != 0) mom[9] += (float)(cy * cz) * sm;
}

__host__ __device__ __forceinline__ void pair_moments(const float (&f)[27], float (&mom)[10])
{
    mom[0] = f[0];
#pragma unroll
    for (int k = 1; k < 10; ++k) mom[k] = 0.f;
    static_for<13>([&](auto P) {
        constexpr int i = 2 * P + 1;
        pair_moment_add<i>(f[i], f[i + 1], mom);
    });
}

// ------------------------------------------------------------------ H: hydro

// Macroscopic part of the collision at a fluid node (Sec. II A) from the
// kinetic moments mom = (p*, j, P) of the pulled populations and the phi
// stencil (value ph, gradient g, Laplacian lap): mu_phi and F_sigma
// (Eq. (19)), mixture laws (Eqs. (8)-(10)), F_p (Eq. (20)), F_ext and F_nu
// (Eq. (21), with the equilibrium at u' = j + a'/2 built without F_nu), the
// acceleration a = F/rho and u = j + a/2 (Eq. (7)).
struct Macro {
    float ps, ux, uy, uz, ax, ay, az, omega;
};

__device__ __forceinline__ Macro macro_node(const DevParams &p, float ph, float gx, float gy, float gz, float lap,
                                            const float (&mom)[10])
{
    const float ps = mom[0], jx = mom[1], jy = mom[2], jz = mom[3];
    const float Pxx = mom[4], Pyy = mom[5], Pzz = mom[6], Pxy = mom[7], Pxz = mom[8], Pyz = mom[9];
    const float mu_phi = p.beta4 * ph * (ph - 1.0f) * (ph - 0.5f) - p.kappa_phi * lap;
    float Fx = mu_phi * gx, Fy = mu_phi * gy, Fz = mu_phi * gz;
    const float rho = p.rho_g + p.drho * ph;
    const float irho = fast_rcp(rho);
    const float nu = (p.mu_g + p.dmu * ph) * irho;
    const float omega = fast_rcp(0.5f + 3.0f * nu);
    float ax, ay, az;
    if (p.variable_density) {
        const float grx = p.drho * gx, gry = p.drho * gy, grz = p.drho * gz;
        const float cp = -ps * (1.0f / 3.0f);
        const float fe = p.drho * ph;
        Fx += cp * grx + fe * p.gx;
        Fy += cp * gry + fe * p.gy;
        Fz += cp * grz + fe * p.gz;
        const float a1x = Fx * irho, a1y = Fy * irho, a1z = Fz * irho;
        const float ux1 = jx + 0.5f * a1x, uy1 = jy + 0.5f * a1y, uz1 = jz + 0.5f * a1z;
        const float p3 = ps * (1.0f / 3.0f);
        const float Qxx = Pxx - p3 - ux1 * ux1, Qyy = Pyy - p3 - uy1 * uy1, Qzz = Pzz - p3 - uz1 * uz1;
        const float Qxy = Pxy - ux1 * uy1, Qxz = Pxz - ux1 * uz1, Qyz = Pyz - uy1 * uz1;
        const float cnu = -3.0f * nu * omega * irho;
        ax = a1x + cnu * (Qxx * grx + Qxy * gry + Qxz * grz);
        ay = a1y + cnu * (Qxy * grx + Qyy * gry + Qyz * grz);
        az = a1z + cnu * (Qxz * grx + Qyz * gry + Qzz * grz);
    } else {
        ax = Fx * irho;
        ay = Fy * irho;
        az = Fz * irho;
    }
    Macro M;
    M.ps = ps;
    M.ux = jx + 0.5f * ax;
    M.uy = jy + 0.5f * ay;
    M.uz = jz + 0.5f * az;
    M.ax = ax;
    M.ay = ay;
    M.az = az;
    M.omega = omega;
    return M;
}

// Hermite coefficients of the post-collision populations (Eqs. (3), (11),
// (14), (16), (17) with the trapezoidal shift):
//   f*_i = w_i [p* + 3 c.(u + a/2) + 4.5 H2:C2 + 4.5 H3:C3],
//   C2 = uu + (ua + au)/2 + (1 - omega) A2,  C3 = uuu + (1 - omega) S(u A2),
// A2 = (xx, yy, zz, xy, xz, yz) the non-equilibrium moment.
__device__ __forceinline__ Herm herm_post(const Macro &M, const float (&A2)[6])
{
    const float ux = M.ux, uy = M.uy, uz = M.uz, ax = M.ax, ay = M.ay, az = M.az;
    const float A2xx = A2[0], A2yy = A2[1], A2zz = A2[2], A2xy = A2[3], A2xz = A2[4], A2yz = A2[5];
    const float om1 = 1.0f - M.omega;
    Herm h;
    h.ps = M.ps;
    h.bx = ux + 0.5f * ax;
    h.by = uy + 0.5f * ay;
    h.bz = uz + 0.5f * az;
    h.xx = ux * ux + ux * ax + om1 * A2xx;
    h.yy = uy * uy + uy * ay + om1 * A2yy;
    h.zz = uz * uz + uz * az + om1 * A2zz;
    h.xy = ux * uy + 0.5f * (ux * ay + ax * uy) + om1 * A2xy;
    h.xz = ux * uz + 0.5f * (ux * az + ax * uz) + om1 * A2xz;
    h.yz = uy * uz + 0.5f * (uy * az + ay * uz) + om1 * A2yz;
    h.tr3 = (h.xx + h.yy + h.zz) * (1.0f / 3.0f);
    // C3 = uuu + (1 - omega)(u_a A2_bg + u_b A2_ag + u_g A2_ab)
    h.xxy = ux * ux * uy + om1 * (2.0f * ux * A2xy + uy * A2xx);
    h.xxz = ux * ux * uz + om1 * (2.0f * ux * A2xz + uz * A2xx);
    h.yyx = uy * uy * ux + om1 * (2.0f * uy * A2xy + ux * A2yy);
    h.yyz = uy * uy * uz + om1 * (2.0f * uy * A2yz + uz * A2yy);
    h.zzx = uz * uz * ux + om1 * (2.0f * uz * A2xz + ux * A2zz);
    h.zzy = uz * uz * uy + om1 * (2.0f * uz * A2yz + uy * A2zz);
    h.xyz = ux * uy * uz + om1 * (ux * A2yz + uy * A2xz + uz * A2xy);
    return h;
}

// Fused pull collide-stream at fluid node x (Sec. II A):
//   pull f_i(x) = f*_i(x - c_i), or f*_opp(i)(x) when x - c_i is solid
//   (halfway bounce-back); phi stencil -> grad, lap (Eqs. (22)-(23));
//   mu_phi and F_sigma (Eq. (19)); mixture laws (Eqs. (8)-(10)); moments
//   (Eqs. (6)-(7)); F_p (Eq. (20)), F_ext, F_nu (Eq. (21)); third-order
//   equilibrium (Eq. (11)), Guo forcing (Eq. (17)) with the trapezoidal shift,
//   recursive regularisation (Eqs. (14), (16)):
//     f*_i = w_i [p* + 3 c.(u + a/2) + 4.5 H2:C2 + 4.5 H3:C3],
//     C2 = uu + (ua + au)/2 + (1 - omega) A2,  C3 = uuu + (1 - omega) S(u A2),
//     A2 = P - p*/3 I - uu + (ua + au)/2  (second moment of f - f^eq + S/2).
//   Writes f* and u.
//   Populations are written with non-temporal hints: each is touched once per
//   step and the 27-plane sets are far larger than the caches, so they should
//   not evict phi, u and the masks, which the stencils re-read.  NTL = true
//   reads them with the same hint; that pays when a workgroup covers whole
//   rows (bx = nx), whose y and z neighbour rows are pulled by workgroups
//   running at the same time.  Narrower tiles re-read neighbour rows later,
//   from L2, and run faster with ordinary loads (NTL = false; about 10% on
//   the 64-domain batch, 12% on 256 x 256 x 128).
template <bool NTL>
__device__ __forceinline__ void hydro_node(const Grid &g, const DevParams &p, const Node &nd,
                                           const float *__restrict__ fin, float *__restrict__ fout,
                                           const float *__restrict__ phi, const uint32_t *__restrict__ nbr,
                                           float *__restrict__ u, uint32_t *__restrict__ flag, bool walls = true)
{
    if (!nd.in) return;
    const Offs o = node_offsets(g, nd.x, nd.y, nd.z);
    const uint32_t n = at<0, 0, 0>(o);
    // walls == false: the caller knows that no node of its tile is solid or next to a solid node
    const uint32_t m = walls ? nbr[n] : 0u;
    if (m & 1u) return;
    const uint32_t N = g.N;

    float s[27];
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        s[kk] = phi[at<kk % 3 - 1, (kk / 3) % 3 - 1, kk / 9 - 1>(o)];
    });
    float f[27];
    pull_populations<NTL>(g, o, n, m, fin, f);

    float gx, gy, gz, lap;
    stencil_grad_lap(s, gx, gy, gz, lap);
    const float ph = s[13];

    // kinetic moments
    float mom[10];
    pair_moments(f, mom);
    const float ps = mom[0];
    const float Pxx = mom[4], Pyy = mom[5], Pzz = mom[6], Pxy = mom[7], Pxz = mom[8], Pyz = mom[9];

    const Macro M = macro_node(p, ph, gx, gy, gz, lap, mom);
    const float ux = M.ux, uy = M.uy, uz = M.uz, ax = M.ax, ay = M.ay, az = M.az;

    // A2 (R2 reading: local second moment of f - f^eq + S/2)
    const float p3 = ps * (1.0f / 3.0f);
    float A2[6];
    A2[0] = Pxx - p3 - ux * ux + ux * ax;
    A2[1] = Pyy - p3 - uy * uy + uy * ay;
    A2[2] = Pzz - p3 - uz * uz + uz * az;
    A2[3] = Pxy - ux * uy + 0.5f * (ux * ay + ax * uy);
    A2[4] = Pxz - ux * uz + 0.5f * (ux * az + ax * uz);
    A2[5] = Pyz - uy * uz + 0.5f * (uy * az + ay * uz);
    const Herm h = herm_post(M, A2);

    const uint32_t n4 = 4u * n, N4 = 4u * N;
    __builtin_nontemporal_store(Lat::w(0) * (h.ps - 4.5f * h.tr3), &fout[n]);
    static_for<13>([&](auto P) {
        constexpr int i = 2 * P + 1;
        float E, O;
        herm_pair<i>(h, E, O);
        __builtin_nontemporal_store(E + O, &fout[(uint32_t)i * N + n]);
        __builtin_nontemporal_store(E - O, &fout[(uint32_t)(i + 1) * N + n]);
    });

    u[n] = ux;
    u[N + n] = uy;
    u[2u * N + n] = uz;
    if (!(isfinite(ux) && isfinite(uy) && isfinite(uz) && isfinite(ps))) flag[0] = 1u;
}

// ------------------------------------------------------------------ P: CAC

template <int NT>
__device__ __forceinline__ void block_sum2(double &x, double &y)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
    }
    __shared__ double sx[NT / 64], sy[NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sx[wid] = x;
        sy[wid] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) {
            tx += sx[k];
            ty += sy[k];
        }
        x = tx;
        y = ty;
    }
}

// CAC update (Eq. (28)) as a 2.5-D stencil: a workgroup owns a BX x BY
// column tile and marches up a chunk of ZC planes.  LDS holds a ring of five
// phi planes (z-2..z+2, halo 2 in x and y), a ring of three planes of the
// compressive flux a = phi(1-phi) grad/|grad| (z-1..z+1, halo 1) and a ring
// of four planes of solid flags (z-1..z+2).  At each plane: store phi(z+2)
// and the flags of z+1, build a(z+1) from the isotropic gradient (Eq. (22),
// normal of Eq. (25)), then update the nodes of plane z:
//   phi* = phi - div(F_a) + D lap(phi) - kappa div_iso(a)
// with MUSCL-minmod face fluxes (Eqs. (29)-(34)), zero on faces touching a
// solid node, and div_iso with the weights w_i/c_s^2.  On solid nodes a is
// the value the ghost update assigned (zero unless wall_compression is on).
// Each thread also accumulates sum(phi*) and sum(chi) (Eqs. (49), (51)) in
// FP64; the workgroup writes one partial per tile.
__host__ __device__ __forceinline__ int wrapc(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Element at a byte offset from a base pointer.  In the phase kernel the base
// is a plane (uniform across the workgroup) and the offset a 32-bit per-thread
// constant: the per-thread part is computed once, not per plane.  (The
// compiler still forms a 64-bit address for each access, one VALU instruction
// per load; buffer loads without it were measured no faster here.)
template <class T>
__device__ __forceinline__ T &at_byte(T *base, uint32_t off)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}
template <class T>
__device__ __forceinline__ const T &at_byte(const T *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// Per-plane partial sums of the tensor-product stencils on a 3x3 plane patch
// v[3*(dy+1) + (dx+1)] around a column:
//   sx = sum_dy t(dy) [v(+1,dy) - v(-1,dy)]   (x differences smoothed in y)
//   sy = sum_dx t(dx) [v(dx,+1) - v(dx,-1)]
//   tq = sum t(dx) t(dy) [v - v(0,0)]          (smoothed, relative to the centre)
// A column's gradient and Laplacian over planes -1, 0, +1 follow as
//   grad_x = (sx_- + 4 sx_0 + sx_+)/72, grad_y likewise with sy,
//   grad_z = (tq_+ - tq_- + 36 (c_+ - c_-))/72,
//   lap    = (tq_- + 4 tq_0 + tq_+ + 36 (c_- + c_+ - 2 c_0))/36,
// the same sums as Eqs. (22)-(23), regrouped plane by plane.
struct PlaneSums {
    float sx, sy, tq, c;
};

__device__ __forceinline__ PlaneSums plane_sums(const float (&v)[9])
{
    PlaneSums r;
    r.c = v[4];
    r.sx = (v[2] - v[0]) + 4.0f * (v[5] - v[3]) + (v[8] - v[6]);
    r.sy = (v[6] - v[0]) + 4.0f * (v[7] - v[1]) + (v[8] - v[2]);
    r.tq = (v[0] - r.c) + (v[2] - r.c) + (v[6] - r.c) + (v[8] - r.c) +
           4.0f * ((v[1] - r.c) + (v[3] - r.c) + (v[5] - r.c) + (v[7] - r.c));
    return r;
}

// minmod of Eq. (32) in branch-free form: equal to 0 when ab <= 0, else the
// argument of smaller magnitude -- which is the median of a, b and 0 (one
// v_med3_f32 on the device).
__host__ __device__ __forceinline__ float minmod2(float a, float b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
#else
    return fmaxf(fminf(a, b), 0.0f) + fminf(fmaxf(a, b), 0.0f);
#endif
}

// The two face fluxes of a node along one axis from phi at offsets -2..+2 and
// the axial velocity at -1, 0, +1 (Eqs. (30)-(34)); the slope at the node is
// shared by both faces.  open_m/open_p: the face does not touch a solid node.
__device__ __forceinline__ float muscl_axis(float q0, float q1, float q2, float q3, float q4, float um, float uc,
                                            float up, bool open_m, bool open_p)
{
    const float d0 = q1 - q0, d1 = q2 - q1, d2 = q3 - q2, d3 = q4 - q3;
    const float sm = minmod2(d0, d1), sc = minmod2(d1, d2), sp = minmod2(d2, d3);
    const float ufp = 0.5f * (uc + up), ufm = 0.5f * (um + uc);
    const float fp = ufp * (ufp >= 0.0f ? q2 + 0.5f * sc : q3 - 0.5f * sp);
    const float fm = ufm * (ufm >= 0.0f ? q1 + 0.5f * sm : q2 - 0.5f * sc);
    return (open_p ? fp : 0.0f) - (open_m ? fm : 0.0f);
}

// One (column tile, z-chunk) of the phase update; the workgroup's FP64 sums
// go to *partial_out (written by thread 0).  With `chunk` given, every node
// that enters the interface sum also sets the byte of its 1024-node chunk
// there, counted from node offset `coff` (the volume correction touches no
// other chunk).  Must be entered by the whole workgroup; reuses its LDS on
// every call.
template <int BX, int BY, int U = 2>
__device__ __forceinline__ void phase_tile(const Grid &g, const PhaseTiling &pt, const DevParams &p, uint32_t tile,
                                           const float *__restrict__ phi, float *__restrict__ phi_out,
                                           const float *__restrict__ u, const float *__restrict__ aw,
                                           const uint8_t *__restrict__ solid, double2 *partial_out,
                                           uint32_t *__restrict__ flag, uint8_t *__restrict__ chunk,
                                           uint32_t coff = 0u)
{
    constexpr int NT = BX * BY;
    constexpr int HX = BX + 4, HY = BY + 4;  // phi plane, halo 2
    constexpr int AX = BX + 2, AY = BY + 2;  // flux / flag plane, halo 1
    constexpr int PF = (HX * HY + NT - 1) / NT;  // phi values per thread per plane
    constexpr int NRING = 2 * (AX + AY) - 4;    // halo-1 points outside the tile
    constexpr int PA = 1 + (NRING + NT - 1) / NT;  // flux points per thread per plane
    __shared__ float sphi[5][HY][HX];
    __shared__ float sa[3][3][AY][AX];
    __shared__ uint8_t ssol[4][AY][AX];

    const int tcx = (int)(tile % (uint32_t)pt.ntx);
    const int tcy = (int)((tile / (uint32_t)pt.ntx) % (uint32_t)pt.nty);
    const int tcz = (int)(tile / ((uint32_t)pt.ntx * (uint32_t)pt.nty));
    const int x0 = tcx * BX, y0 = tcy * BY, z0 = tcz * pt.zc;
    const int z1 = min(z0 + pt.zc, g.nz);
    const int tid = threadIdx.x;
    const int lx = tid % BX, ly = tid / BX;
    const int x = x0 + lx, y = y0 + ly;
    const bool col_in = x < g.nx && y < g.ny;
    const uint32_t N = g.N;

    auto pslot = [&](int zz) { return (zz - z0 + 10) % 5; };
    auto aslot = [&](int zz) { return (zz - z0 + 3) % 3; };
    auto sslot = [&](int zz) { return (zz - z0 + 4) & 3; };
    // plane offset with periodic wrap; the planes visited lie within a few of [0, nz),
    // so the modulo (a long integer division) is taken only off that range
    auto zoff = [&](int zz) {
        const int w = (zz >= 0 && zz < g.nz) ? zz : wrapc(zz, g.nz);
        return (uint32_t)w * g.nxny;
    };

    // this thread's share of the halo planes: in-plane offset (bytes for phi,
    // nodes for the flags) and LDS position
    uint32_t pxy[PF], axy[PA];
    int apos[PA];
#pragma unroll
    for (int r = 0; r < PF; ++r) {
        const int k = tid + r * NT;
        const int hx = k % HX, hy = k / HX;
        pxy[r] = k < HX * HY ? 4u * ((uint32_t)wrapc(x0 - 2 + hx, g.nx) + (uint32_t)wrapc(y0 - 2 + hy, g.ny) * (uint32_t)g.nx) : 0u;
    }
    // flux points (and solid flags) of this thread in the halo-1 plane: r = 0 is
    // its own column, so the plane sums build_a forms there serve the column's
    // update too; r >= 1 walk the ring around the tile (rows 0 and AY-1, then
    // columns 0 and AX-1)
#pragma unroll
    for (int r = 0; r < PA; ++r) {
        int ax = lx + 1, ay = ly + 1;
        bool ok = true;
        if (r > 0) {
            const int j = tid + (r - 1) * NT;
            ok = j < NRING;
            if (j < 2 * AX) {
                ax = j % AX;
                ay = j < AX ? 0 : AY - 1;
            } else {
                const int k = j - 2 * AX;
                ax = k < AY - 2 ? 0 : AX - 1;
                ay = 1 + k % (AY - 2);
            }
        }
        axy[r] = ok ? (uint32_t)wrapc(x0 - 1 + ax, g.nx) + (uint32_t)wrapc(y0 - 1 + ay, g.ny) * (uint32_t)g.nx : 0u;
        apos[r] = ok ? ay * AX + ax : -1;
    }
    auto aval = [&](int r) { return r == 0 || apos[r] >= 0; };
    auto fetch_phi = [&](int zz, float (&v)[PF]) {
        const uint32_t zo = zoff(zz);
#pragma unroll
        for (int r = 0; r < PF; ++r)
            if (tid + r * NT < HX * HY) v[r] = at_byte(phi + zo, pxy[r]);
    };
    auto store_phi = [&](int zz, const float (&v)[PF]) {
        float *dst = &sphi[pslot(zz)][0][0];
#pragma unroll
        for (int r = 0; r < PF; ++r)
            if (tid + r * NT < HX * HY) dst[tid + r * NT] = v[r];
    };
    auto fetch_sol = [&](int zz, uint8_t (&v)[PA]) {
        const uint32_t zo = zoff(zz);
#pragma unroll
        for (int r = 0; r < PA; ++r)
            if (aval(r)) v[r] = at_byte(solid + zo, axy[r]);
    };
    auto store_sol = [&](int zz, const uint8_t (&v)[PA]) {
        uint8_t *dst = &ssol[sslot(zz)][0][0];
#pragma unroll
        for (int r = 0; r < PA; ++r)
            if (aval(r)) dst[apos[r]] = v[r];
    };
    // 3x3 patch of phi plane zz centred on halo-1 position (ax, ay) (= halo-2 position + 1)
    auto patch = [&](int zz, int ax, int ay, float (&v)[9]) {
        const float *pl = &sphi[pslot(zz)][0][0];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = pl[(ay + j / 3) * HX + ax + j % 3];
    };

    // rolling plane sums of every flux point this thread builds (planes zz-1, zz)
    PlaneSums bprev[PA], bcur[PA];
    auto flux_points_sums = [&](int zz, PlaneSums (&out)[PA]) {
#pragma unroll
        for (int r = 0; r < PA; ++r) {
            if (!aval(r)) continue;
            float v[9];
            patch(zz, apos[r] % AX, apos[r] / AX, v);
            out[r] = plane_sums(v);
        }
    };
    // compressive flux plane zz: needs phi planes zz-1..zz+1 (sums of zz-1, zz rolled in)
    auto build_a = [&](int zz) {
        const int sl = aslot(zz);
        const uint32_t zo = zoff(zz);
        PlaneSums nxt[PA];
        flux_points_sums(zz + 1, nxt);
#pragma unroll
        for (int r = 0; r < PA; ++r) {
            if (!aval(r)) continue;
            const int pos = apos[r];
            float cx = 0.f, cy = 0.f, cz = 0.f;
            if ((&ssol[sslot(zz)][0][0])[pos]) {
                if (p.wall_compression) {
                    const uint32_t id = axy[r] + zo;
                    cx = aw[id];
                    cy = aw[N + id];
                    cz = aw[2u * N + id];
                }
            } else {
                const PlaneSums &m = bprev[r], &c = bcur[r], &q = nxt[r];
                const float gx = (m.sx + 4.0f * c.sx + q.sx) * (1.0f / 72.0f);
                const float gy = (m.sy + 4.0f * c.sy + q.sy) * (1.0f / 72.0f);
                const float gz = (q.tq - m.tq + 36.0f * (q.c - m.c)) * (1.0f / 72.0f);
                const float g2 = gx * gx + gy * gy + gz * gz;
                if (g2 > p.eps_n2) {
                    const float sc = c.c * (1.0f - c.c) * rsqrtf(g2);
                    cx = sc * gx;
                    cy = sc * gy;
                    cz = sc * gz;
                }
            }
            (&sa[sl][0][0][0])[pos] = cx;
            (&sa[sl][1][0][0])[pos] = cy;
            (&sa[sl][2][0][0])[pos] = cz;
            bprev[r] = bcur[r];
            bcur[r] = nxt[r];
        }
    };

    // velocities this node's fluxes need on plane zz (in-plane byte offsets)
    const uint32_t cxy = col_in ? 4u * ((uint32_t)x + (uint32_t)y * (uint32_t)g.nx) : 0u;
    const uint32_t xm = col_in ? 4u * ((uint32_t)wrapc(x - 1, g.nx) + (uint32_t)y * (uint32_t)g.nx) : 0u;
    const uint32_t xp = col_in ? 4u * ((uint32_t)wrapc(x + 1, g.nx) + (uint32_t)y * (uint32_t)g.nx) : 0u;
    const uint32_t ym = col_in ? 4u * ((uint32_t)x + (uint32_t)wrapc(y - 1, g.ny) * (uint32_t)g.nx) : 0u;
    const uint32_t yp = col_in ? 4u * ((uint32_t)x + (uint32_t)wrapc(y + 1, g.ny) * (uint32_t)g.nx) : 0u;
    struct UPlane {
        float xm, xc, xp, ym, yc, yp, zn;  // zn: u_z one plane up
    };
    auto fetch_u = [&](int zz, UPlane &v) {
        if (!col_in) return;
        const uint32_t zo = zoff(zz);
        const float *ux = u + zo, *uy = u + N + zo, *uz = u + 2u * N + zoff(zz + 1);
        v.xm = at_byte(ux, xm);
        v.xc = at_byte(ux, cxy);
        v.xp = at_byte(ux, xp);
        v.ym = at_byte(uy, ym);
        v.yc = at_byte(uy, cxy);
        v.yp = at_byte(uy, yp);
        v.zn = at_byte(uz, cxy);
    };

    const int hx = lx + 2, hy = ly + 2, ax = lx + 1, ay = ly + 1;
    // column-rolling sums of the output node: Laplacian sums (tq, c) of planes, the
    // in-plane cross of plane z, and the flux-divergence plane sums
    auto col_patch = [&](int zz, float (&v)[9]) { patch(zz, lx + 1, ly + 1, v); };
    auto flux_sums = [&](int zz, float &X, float &Y, float &Z) {
        const int sl = aslot(zz);
        const float *fx = &sa[sl][0][0][0], *fy = &sa[sl][1][0][0], *fz = &sa[sl][2][0][0];
        const int c0 = ay * AX + ax;
        X = (fx[c0 - AX + 1] - fx[c0 - AX - 1]) + 4.0f * (fx[c0 + 1] - fx[c0 - 1]) + (fx[c0 + AX + 1] - fx[c0 + AX - 1]);
        Y = (fy[c0 + AX - 1] - fy[c0 - AX - 1]) + 4.0f * (fy[c0 + AX] - fy[c0 - AX]) + (fy[c0 + AX + 1] - fy[c0 - AX + 1]);
        Z = fz[c0 - AX - 1] + fz[c0 - AX + 1] + fz[c0 + AX - 1] + fz[c0 + AX + 1] +
            4.0f * (fz[c0 - AX] + fz[c0 - 1] + fz[c0 + 1] + fz[c0 + AX]) + 16.0f * fz[c0];
    };

    // prologue: phi planes z0-2..z0+1, flags z0-1, z0, flux planes z0-1, z0
    {
        float v[PF];
        uint8_t f8[PA];
        for (int zz = z0 - 2; zz <= z0 + 1; ++zz) {
            fetch_phi(zz, v);
            store_phi(zz, v);
        }
        for (int zz = z0 - 1; zz <= z0; ++zz) {
            fetch_sol(zz, f8);
            store_sol(zz, f8);
        }
    }
    __syncthreads();
    flux_points_sums(z0 - 2, bprev);
    flux_points_sums(z0 - 1, bcur);
    build_a(z0 - 1);
    build_a(z0);
    __syncthreads();
    // output column state for plane z0
    float tq_m, tq_c, c_m2, c_m, c_c, cr_xm, cr_xp, cr_ym, cr_yp, X_m, X_c, Y_m, Y_c, Z_m, Z_c;
    {
        float v[9];
        col_patch(z0 - 1, v);
        const PlaneSums sm = plane_sums(v);
        col_patch(z0, v);
        const PlaneSums sc = plane_sums(v);
        tq_m = sm.tq;
        c_m = sm.c;
        tq_c = sc.tq;
        c_c = sc.c;
        cr_xm = v[3];
        cr_xp = v[5];
        cr_ym = v[1];
        cr_yp = v[7];
        c_m2 = sphi[pslot(z0 - 2)][hy][hx];
        flux_sums(z0 - 1, X_m, Y_m, Z_m);
        flux_sums(z0, X_c, Y_c, Z_c);
    }
    float nphi[PF];
    uint8_t nsol[PA];
    UPlane uc{}, un{};
    float uzm = 0.f, uzc = 0.f, uzp = 0.f;
    fetch_phi(z0 + 2, nphi);
    fetch_sol(z0 + 1, nsol);
    fetch_u(z0, uc);
    if (col_in) {
        uzm = at_byte(u + 2u * N + zoff(z0 - 1), cxy);
        uzc = at_byte(u + 2u * N + zoff(z0), cxy);
    }
    uzp = uc.zn;
    // z axis of the advective flux, rolled along the column: the slope at the
    // node (zsc), phi(z+1) - phi(z) (zd2) and the face flux at z-1/2 before the
    // solid test (zfm) carry over from plane z-1, where they were the upper
    // slope, the upper difference and the flux at its z+1/2 face
    float zsc, zd2, zfm;
    {
        const float q3 = sphi[pslot(z0 + 1)][hy][hx];
        const float d0 = c_m - c_m2, d1 = c_c - c_m, d2 = q3 - c_c;
        const float sm = minmod2(d0, d1);
        zsc = minmod2(d1, d2);
        zd2 = d2;
        const float uf = 0.5f * (uzm + uzc);
        zfm = uf * (uf >= 0.0f ? c_m + 0.5f * sm : c_c - 0.5f * zsc);
    }

    double sphis = 0.0, schi = 0.0;
    // one plane of the march; called twice per loop trip (the unrolled form
    // keeps the rolled column state in place instead of copying it)
    auto plane = [&](const int z) __attribute__((always_inline)) {
        // Two barriers per plane.  The stores below may run while slower waves
        // still update plane z-1, which reads phi planes z-1..z+1, flux plane z
        // and flag planes z-2..z: the slots written here (phi z+2, flags z+1)
        // are none of those, with rings of five and four.
        store_phi(z + 2, nphi);
        store_sol(z + 1, nsol);
        if (z + 1 < z1) {  // prefetch for the next plane; lands while this one computes
            fetch_phi(z + 3, nphi);
            fetch_sol(z + 2, nsol);
            fetch_u(z + 1, un);
        }
        __syncthreads();
        build_a(z + 1);
        __syncthreads();
        // new column sums of plane z+1 (phi: this thread's own flux point,
        // just rolled into bprev[0]) and flux plane z+1
        const PlaneSums sp = bprev[0];
        const float *p1 = &sphi[pslot(z + 1)][0][0];
        const int h0 = hy * HX + hx;
        const float nx_m = p1[h0 - 1], nx_p = p1[h0 + 1], ny_m = p1[h0 - HX], ny_p = p1[h0 + HX];
        float X_p, Y_p, Z_p;
        flux_sums(z + 1, X_p, Y_p, Z_p);
        // z flux at z+1/2 (Eqs. (30)-(34)), for every column so that it rolls
        const float c_p2 = sphi[pslot(z + 2)][hy][hx];
        const float zd3 = c_p2 - sp.c;
        const float zsp = minmod2(zd2, zd3);
        const float ufp = 0.5f * (uzc + uzp);
        const float zfp = ufp * (ufp >= 0.0f ? c_c + 0.5f * zsc : sp.c - 0.5f * zsp);
        const uint8_t *fl = &ssol[sslot(z)][0][0];
        const int c0 = ay * AX + ax;
        if (col_in && !fl[c0]) {
            const float ph = c_c;
            const float lap = (tq_m + 4.0f * tq_c + sp.tq + 36.0f * ((c_m - ph) + (sp.c - ph))) * (1.0f / 36.0f);
            const float *p0 = &sphi[pslot(z)][0][0];
            float div_a = muscl_axis(p0[h0 - 2], cr_xm, ph, cr_xp, p0[h0 + 2], uc.xm, uc.xc, uc.xp, !fl[c0 - 1], !fl[c0 + 1]);
            div_a += muscl_axis(p0[h0 - 2 * HX], cr_ym, ph, cr_yp, p0[h0 + 2 * HX], uc.ym, uc.yc, uc.yp, !fl[c0 - AX],
                                !fl[c0 + AX]);
            div_a += (!ssol[sslot(z + 1)][ay][ax] ? zfp : 0.0f) - (!ssol[sslot(z - 1)][ay][ax] ? zfm : 0.0f);
            const float div_c = (X_m + 4.0f * X_c + X_p + Y_m + 4.0f * Y_c + Y_p + Z_p - Z_m) * (1.0f / 72.0f);
            const float ps = ph - div_a + p.D * lap - p.kappa * div_c;
            at_byte(phi_out + (uint32_t)z * g.nxny, cxy) = ps;
            if (!isfinite(ps)) flag[0] = 1u;
            sphis += (double)ps;
            if (ps > p.eps_phi && ps < 1.0f - p.eps_phi) {
                schi += (double)ps * (1.0 - (double)ps);
                if (chunk) chunk[(coff + (uint32_t)z * g.nxny + (cxy >> 2)) >> 10] = 1;
            }
        }
        // roll the column state to plane z+1
        tq_m = tq_c;
        tq_c = sp.tq;
        c_m = c_c;
        c_c = sp.c;
        cr_xm = nx_m;
        cr_xp = nx_p;
        cr_ym = ny_m;
        cr_yp = ny_p;
        zsc = zsp;
        zd2 = zd3;
        zfm = zfp;
        X_m = X_c;
        X_c = X_p;
        Y_m = Y_c;
        Y_c = Y_p;
        Z_m = Z_c;
        Z_c = Z_p;
        uc = un;
        uzc = uzp;
        uzp = un.zn;
    };
    // the plane loop unrolled U times (the rolled column state then stays in
    // place; U = 4 in the single-lattice kernel, 2 where the batched kernels'
    // extra registers would cost a wave per SIMD)
    static_assert(U == 2 || U == 4, "plane loop unrolled 2 or 4 times");
    int z = z0;
    if constexpr (U == 4) {
        for (; z + 3 < z1; z += 4) {
            plane(z);
            plane(z + 1);
            plane(z + 2);
            plane(z + 3);
        }
        for (; z < z1; ++z) plane(z);
    } else {
        for (; z + 1 < z1; z += 2) {
            plane(z);
            plane(z + 1);
        }
        if (z < z1) plane(z);
    }
    block_sum2<NT>(sphis, schi);
    if (tid == 0) *partial_out = make_double2(sphis, schi);
}

}  // namespace cac
