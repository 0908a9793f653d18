// adjoint_device.hpp -- per-node bodies of the reverse (adjoint) step of the
// coupled CAC lattice Boltzmann update.  Each body is the transpose of the
// Jacobian of the forward step at the recorded state, node by node, written
// by hand from the forward bodies in step_device.hpp:
//
//   forward step n:  phi-hat = W(phi^n, theta)            ghosts (Sec. II B)
//                    f*^n, u = H(pull(f*^{n-1}), phi-hat)  collision (Sec. II A)
//                    phi*    = P(phi-hat, u, a_wall)       CAC update (Sec. II A 1)
//                    phi^{n+1} = V(phi*)                   volume correction (Sec. II C)
//
//   reverse:  (pb^{n+1}, mb^{n+1}) -> (pb^n, mb^n),  dL/dtheta += ...
//
// pb is the cotangent of the phase field (all nodes), mb the cotangents of
// the ten moments (p*, j, P) that the collision reads (see AdjStep).  At the
// non-smooth points the forward branch is differentiated: the selected
// argument of minmod (the left one on ties), the upwind side, zero outside
// the correction band, zero normal under its guard, and zero derivative of
// lambda_s = sqrt(4 phi (1 - phi)) for 4 phi (1 - phi) <= 1e-12, of
// |grad_par| for |grad_par| <= 1e-12 and of the regularised cotangent.
//
// The bodies are __host__ __device__: the HIP kernels call them per thread,
// and a host build can run them node by node.
#pragma once

#include <math.h>

#include "step_device.hpp"

namespace cac {

#define CAC_HD __host__ __device__ __forceinline__

// Scheduling fence for the device pass: keeps the compiler from hoisting every
// load of the node body to its start (which would need more than 128 VGPRs).
// CAC_PIN(v) makes the value v exist at that point of the program (an empty
// asm statement reads and writes it), so that the arithmetic feeding it is
// not sunk below later loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define CAC_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#define CAC_PIN(v) asm volatile("" : "+v"(v))
#else
#define CAC_SCHED_FENCE() ((void)0)
#define CAC_PIN(v) ((void)0)
#endif

// Transpose of phi^{n+1} = phi* + lambda chi(phi*) on fluid nodes, with
// lambda = (M - sum phi*) / sum chi (Eqs. (49)-(55)):
//   psi = (1 + lambda chi'(phi*)) (pb - cbar),   cbar = sum(pb chi) / sum chi.
CAC_HD float psi_of(float pb, float ps, float lam, float cb, float eps)
{
    const float chip = (ps > eps && ps < 1.0f - eps) ? 1.0f - 2.0f * ps : 0.0f;
    return (1.0f + lam * chip) * (pb - cb);
}

// psi field of one reverse step: the cotangent of phi* on fluid nodes, 0 on solid nodes.
CAC_HD void adj_psi_node(const DevParams &p, const AdjStep &S, uint32_t n)
{
    S.psi[n] = S.solid[n] ? 0.0f : psi_of(S.pb_in[n], S.phistar[n], (float)S.rs[0], (float)S.rs[1], p.eps_phi);
}

// Isotropic gradient (Eq. (22)) of a 3x3x3 patch v[k], k = (dz+1)*9 + (dy+1)*3 + (dx+1),
// without the centre-difference form (for cotangent fields, which are not smooth).
CAC_HD void patch_grad(const float (&v)[27], float &gx, float &gy, float &gz)
{
    gx = gy = gz = 0.f;
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        constexpr int dx = kk % 3 - 1, dy = (kk / 3) % 3 - 1, dz = kk / 9 - 1;
        constexpr float w = tw(dx) * tw(dy) * tw(dz) * (1.0f / 72.0f);
        if constexpr (dx != 0) gx += ((float)dx * w) * v[kk];
        if constexpr (dy != 0) gy += ((float)dy * w) * v[kk];
        if constexpr (dz != 0) gz += ((float)dz * w) * v[kk];
    });
}

// Transpose of the two MUSCL face fluxes of a node along one axis (the node is
// point 2 of five; the forward is muscl_axis).  q: phi-hat, uu: axial
// velocity, pp: psi, fl: fluid flags at the five points.  Returns the
// cotangent of phi-hat at the node; ub gets the cotangent of its velocity.
// A face carries flux only between two fluid nodes.
CAC_HD float muscl_axis_adj(const float (&q)[5], const float (&uu)[5], const float (&pp)[5], const bool (&fl)[5],
                            float &ub)
{
    float uf[4], Fb[4];
    bool open[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        open[k] = fl[k] && fl[k + 1];
        uf[k] = 0.5f * (uu[k] + uu[k + 1]);
        Fb[k] = open[k] ? pp[k + 1] - pp[k] : 0.0f;  // F enters phi* with -1 at its left node, +1 at its right
    }
    // minmod slopes at points 1..3 and the argument they take: +1 left difference, -1 right, 0 none
    float sl[4];
    int sel[4];
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        const float a = q[k] - q[k - 1], b = q[k + 1] - q[k];
        sl[k] = minmod2(a, b);
        const bool same = (a > 0.0f && b > 0.0f) || (a < 0.0f && b < 0.0f);
        sel[k] = same ? (fabsf(a) <= fabsf(b) ? 1 : -1) : 0;
    }
    sl[0] = 0.f;
    sel[0] = 0;
    // upwind states of the faces (1,2) and (2,3)
    const float up1 = uf[1] >= 0.0f ? q[1] + 0.5f * sl[1] : q[2] - 0.5f * sl[2];
    const float up2 = uf[2] >= 0.0f ? q[2] + 0.5f * sl[2] : q[3] - 0.5f * sl[3];
    ub = 0.5f * ((open[1] ? Fb[1] * up1 : 0.0f) + (open[2] ? Fb[2] * up2 : 0.0f));
    // cotangents of the slopes: s_k enters face (k, k+1) from the left when u_f >= 0
    // and face (k-1, k) from the right when u_f < 0
    float sb[4];
#pragma unroll
    for (int k = 1; k <= 3; ++k)
        sb[k] = (uf[k] >= 0.0f ? 0.5f * Fb[k] * uf[k] : 0.0f) - (uf[k - 1] < 0.0f ? 0.5f * Fb[k - 1] * uf[k - 1] : 0.0f);
    float r = (uf[2] >= 0.0f ? Fb[2] * uf[2] : 0.0f) + (uf[1] < 0.0f ? Fb[1] * uf[1] : 0.0f);
    r += sel[1] == -1 ? sb[1] : 0.0f;                              // s_1 = minmod(q1 - q0, q2 - q1)
    r += sel[2] == 1 ? sb[2] : (sel[2] == -1 ? -sb[2] : 0.0f);     // s_2 = minmod(q2 - q1, q3 - q2)
    r += sel[3] == 1 ? -sb[3] : 0.0f;                              // s_3 = minmod(q3 - q2, q4 - q3)
    return r;
}

// Cotangent of a pulled population f_i from the ten moment cotangents, held as
// a = (p*, j_x, j_y, j_z), b = (P_xx, P_yy, P_zz, P_xy), c = (P_xz, P_yz):
// mb_0 + c_i . j-bar + c_i c_i : P-bar.  With rev, the same for the opposite
// link (c_i -> -c_i flips the odd part only): the population that bounced
// back from a solid x + c_i.
template <int I>
CAC_HD float pop_bar(float4 a, float4 b, float2 c, bool rev = false)
{
    constexpr int cx = Lat::cx[I], cy = Lat::cy[I], cz = Lat::cz[I];
    float e = a.x, l = 0.f;
    if constexpr (cx != 0) {
        e += b.x;
        l += (float)cx * a.y;
    }
    if constexpr (cy != 0) {
        e += b.y;
        l += (float)cy * a.z;
    }
    if constexpr (cz != 0) {
        e += b.z;
        l += (float)cz * a.w;
    }
    if constexpr (cx * cy != 0) e += (float)(cx * cy) * b.w;
    if constexpr (cx * cz != 0) e += (float)(cx * cz) * c.x;
    if constexpr (cy * cz != 0) e += (float)(cy * cz) * c.y;
    return rev ? e - l : e + l;
}

// Cotangents of the Hermite coefficients of the post-collision populations
// (the C2 trace is folded into xx, yy, zz).
struct HermBar {
    float ps = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
    float xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
    float xxy = 0.f, xxz = 0.f, yyx = 0.f, yyz = 0.f, zzx = 0.f, zzy = 0.f, xyz = 0.f;
};

// Transpose of the Hermite projection of the post-collision populations
// f*_i = w_i [ps + 3 c.b + 4.5 (cc : C2 - tr C2 / 3) + 4.5 H3 : C3] (herm_pair):
// h = sum_i fb_i d f*_i / d (coefficients), summed over the 27 links by
// moments.  The D3Q27 weights factorise, w_i = w1(cx) w1(cy) w1(cz) with
// w1(0) = 2/3 and w1(+-1) = 1/6, so h is a linear map of the 17 moments
// M_abc = sum_i w_i cx^a cy^b cz^c fb_i that it needs, and each x-line of
// links (cy, cz fixed) enters them through three partial sums over cx.
// Moment order in M: 000 100 010 001 200 020 002 110 101 011 210 201 120 021
// 102 012 111.
struct HermMoments {
    float M[17] = {};
    static constexpr int A[17] = {0, 1, 0, 0, 2, 0, 0, 1, 1, 0, 2, 2, 1, 0, 1, 0, 1};
    static constexpr int B[17] = {0, 0, 1, 0, 0, 2, 0, 1, 0, 1, 1, 0, 2, 2, 0, 1, 1};
    static constexpr int C[17] = {0, 0, 0, 1, 0, 0, 2, 0, 1, 1, 0, 1, 0, 1, 2, 2, 1};
    static constexpr float pw(int v, int e) { return e == 0 ? 1.0f : e == 1 ? (float)v : (float)(v * v); }
    static constexpr float w1(int v) { return v == 0 ? 2.0f / 3.0f : 1.0f / 6.0f; }
    // one x-line: fb at cx = -1, 0, +1
    template <int CY, int CZ>
    CAC_HD void add_line(float gm, float g0, float gp)
    {
        const float S = gp + gm, D = gp - gm;
        const float A0 = 4.0f * g0 + S;  // 6 sum_cx w1(cx) fb; D and S likewise for cx^1, cx^2
        static_for<17>([&](auto K) {
            constexpr int k = K;
            constexpr float cf = w1(CY) * w1(CZ) * (1.0f / 6.0f) * pw(CY, B[k]) * pw(CZ, C[k]);
            if constexpr (cf != 0.0f) M[k] += cf * (A[k] == 0 ? A0 : A[k] == 1 ? D : S);
        });
    }
    CAC_HD void pin()
    {
#pragma unroll
        for (int k = 0; k < 17; ++k) CAC_PIN(M[k]);
    }
    CAC_HD HermBar herm() const
    {
        HermBar h;
        const float t = 1.0f / 3.0f;
        h.ps = M[0];
        h.bx = 3.0f * M[1];
        h.by = 3.0f * M[2];
        h.bz = 3.0f * M[3];
        h.xx = 4.5f * (M[4] - t * M[0]);
        h.yy = 4.5f * (M[5] - t * M[0]);
        h.zz = 4.5f * (M[6] - t * M[0]);
        h.xy = 9.0f * M[7];
        h.xz = 9.0f * M[8];
        h.yz = 9.0f * M[9];
        h.xxy = 13.5f * (M[10] - t * M[2]);
        h.xxz = 13.5f * (M[11] - t * M[3]);
        h.yyx = 13.5f * (M[12] - t * M[1]);
        h.yyz = 13.5f * (M[13] - t * M[3]);
        h.zzx = 13.5f * (M[14] - t * M[1]);
        h.zzy = 13.5f * (M[15] - t * M[2]);
        h.xyz = 27.0f * M[16];
        return h;
    }
};

// Transpose of the collision of hydro_node at one fluid node.
// mom: moments (p*, j, P) of the pulled populations; (gx, gy, gz, lap, ph):
// phi-hat gradient, Laplacian and value; hb: cotangents of the Hermite
// coefficients of the post-collision populations (HermMoments); (ubx, uby, ubz):
// cotangent of the velocity output.  Writes the moment cotangents mb and adds
// the cotangents of ph, of the gradient and of the Laplacian.
CAC_HD void collide_adj(const DevParams &p, const float (&mom)[10], float gx, float gy, float gz, float lap, float ph,
                        const HermBar &hb, float ubx, float uby, float ubz, float (&mb)[10], float &phb,
                        float &Gbx, float &Gby, float &Gbz, float &lapb)
{
    // ---------------- forward recompute, in the order of hydro_node
    const float ps = mom[0], jx = mom[1], jy = mom[2], jz = mom[3];
    const float Pxx = mom[4], Pyy = mom[5], Pzz = mom[6], Pxy = mom[7], Pxz = mom[8], Pyz = mom[9];
    const float mu_phi = p.beta4 * ph * (ph - 1.0f) * (ph - 0.5f) - p.kappa_phi * lap;
    const float F0x = mu_phi * gx, F0y = mu_phi * gy, F0z = mu_phi * gz;
    const float rho = p.rho_g + p.drho * ph;
    const float irho = fast_rcp(rho);
    const float nu = (p.mu_g + p.dmu * ph) * irho;
    const float omega = fast_rcp(0.5f + 3.0f * nu);
    const bool vd = p.variable_density != 0;
    float grx = 0.f, gry = 0.f, grz = 0.f, cp = 0.f, Fx = F0x, Fy = F0y, Fz = F0z;
    float u1x = 0.f, u1y = 0.f, u1z = 0.f, Qxx = 0.f, Qyy = 0.f, Qzz = 0.f, Qxy = 0.f, Qxz = 0.f, Qyz = 0.f, cnu = 0.f;
    float ax, ay, az;
    if (vd) {
        grx = p.drho * gx;
        gry = p.drho * gy;
        grz = p.drho * gz;
        cp = -ps * (1.0f / 3.0f);
        const float fe = p.drho * ph;
        Fx += cp * grx + fe * p.gx;
        Fy += cp * gry + fe * p.gy;
        Fz += cp * grz + fe * p.gz;
        const float a1x = Fx * irho, a1y = Fy * irho, a1z = Fz * irho;
        u1x = jx + 0.5f * a1x;
        u1y = jy + 0.5f * a1y;
        u1z = jz + 0.5f * a1z;
        const float p3 = ps * (1.0f / 3.0f);
        Qxx = Pxx - p3 - u1x * u1x;
        Qyy = Pyy - p3 - u1y * u1y;
        Qzz = Pzz - p3 - u1z * u1z;
        Qxy = Pxy - u1x * u1y;
        Qxz = Pxz - u1x * u1z;
        Qyz = Pyz - u1y * u1z;
        cnu = -3.0f * nu * omega * irho;
        ax = a1x + cnu * (Qxx * grx + Qxy * gry + Qxz * grz);
        ay = a1y + cnu * (Qxy * grx + Qyy * gry + Qyz * grz);
        az = a1z + cnu * (Qxz * grx + Qyz * gry + Qzz * grz);
    } else {
        ax = F0x * irho;
        ay = F0y * irho;
        az = F0z * irho;
    }
    const float ux = jx + 0.5f * ax, uy = jy + 0.5f * ay, uz = jz + 0.5f * az;
    const float p3 = ps * (1.0f / 3.0f);
    const float A2xx = Pxx - p3 - ux * ux + ux * ax;
    const float A2yy = Pyy - p3 - uy * uy + uy * ay;
    const float A2zz = Pzz - p3 - uz * uz + uz * az;
    const float A2xy = Pxy - ux * uy + 0.5f * (ux * ay + ax * uy);
    const float A2xz = Pxz - ux * uz + 0.5f * (ux * az + ax * uz);
    const float A2yz = Pyz - uy * uz + 0.5f * (uy * az + ay * uz);
    const float om1 = 1.0f - omega;

    const float hps = hb.ps, hbx = hb.bx, hby = hb.by, hbz = hb.bz;
    const float hxx = hb.xx, hyy = hb.yy, hzz = hb.zz, hxy = hb.xy, hxz = hb.xz, hyz = hb.yz;
    const float hxxy = hb.xxy, hxxz = hb.xxz, hyyx = hb.yyx, hyyz = hb.yyz, hzzx = hb.zzx, hzzy = hb.zzy,
                hxyz = hb.xyz;

    // ---------------- back through C2, C3 and b = u + a/2
    float Ubx = ubx + hbx, Uby = uby + hby, Ubz = ubz + hbz;
    float Abx = 0.5f * hbx, Aby = 0.5f * hby, Abz = 0.5f * hbz;
    float om1b = 0.f;
    float Bxx = 0.f, Byy = 0.f, Bzz = 0.f, Bxy = 0.f, Bxz = 0.f, Byz = 0.f;  // cotangents of A2
    // C2_aa = u_a^2 + u_a a_a + om1 A2_aa
    Ubx += hxx * (2.0f * ux + ax); Abx += hxx * ux; om1b += hxx * A2xx; Bxx += hxx * om1;
    Uby += hyy * (2.0f * uy + ay); Aby += hyy * uy; om1b += hyy * A2yy; Byy += hyy * om1;
    Ubz += hzz * (2.0f * uz + az); Abz += hzz * uz; om1b += hzz * A2zz; Bzz += hzz * om1;
    // C2_ab = u_a u_b + (u_a a_b + a_a u_b)/2 + om1 A2_ab
    Ubx += hxy * (uy + 0.5f * ay); Uby += hxy * (ux + 0.5f * ax); Abx += 0.5f * hxy * uy; Aby += 0.5f * hxy * ux;
    om1b += hxy * A2xy; Bxy += hxy * om1;
    Ubx += hxz * (uz + 0.5f * az); Ubz += hxz * (ux + 0.5f * ax); Abx += 0.5f * hxz * uz; Abz += 0.5f * hxz * ux;
    om1b += hxz * A2xz; Bxz += hxz * om1;
    Uby += hyz * (uz + 0.5f * az); Ubz += hyz * (uy + 0.5f * ay); Aby += 0.5f * hyz * uz; Abz += 0.5f * hyz * uy;
    om1b += hyz * A2yz; Byz += hyz * om1;
    // C3_aab = u_a^2 u_b + om1 (2 u_a A2_ab + u_b A2_aa)
    auto c3aab = [&](float h, float ua, float ub_, float A2ab, float A2aa, float &Ua, float &Ub, float &Bab, float &Baa) {
        Ua += h * (2.0f * ua * ub_ + 2.0f * om1 * A2ab);
        Ub += h * (ua * ua + om1 * A2aa);
        om1b += h * (2.0f * ua * A2ab + ub_ * A2aa);
        Bab += h * (2.0f * om1 * ua);
        Baa += h * (om1 * ub_);
    };
    c3aab(hxxy, ux, uy, A2xy, A2xx, Ubx, Uby, Bxy, Bxx);
    c3aab(hxxz, ux, uz, A2xz, A2xx, Ubx, Ubz, Bxz, Bxx);
    c3aab(hyyx, uy, ux, A2xy, A2yy, Uby, Ubx, Bxy, Byy);
    c3aab(hyyz, uy, uz, A2yz, A2yy, Uby, Ubz, Byz, Byy);
    c3aab(hzzx, uz, ux, A2xz, A2zz, Ubz, Ubx, Bxz, Bzz);
    c3aab(hzzy, uz, uy, A2yz, A2zz, Ubz, Uby, Byz, Bzz);
    // C3_xyz = ux uy uz + om1 (ux A2yz + uy A2xz + uz A2xy)
    Ubx += hxyz * (uy * uz + om1 * A2yz);
    Uby += hxyz * (ux * uz + om1 * A2xz);
    Ubz += hxyz * (ux * uy + om1 * A2xy);
    om1b += hxyz * (ux * A2yz + uy * A2xz + uz * A2xy);
    Byz += hxyz * om1 * ux;
    Bxz += hxyz * om1 * uy;
    Bxy += hxyz * om1 * uz;

    // ---------------- back through A2 = P - p*/3 I - uu + (ua + au)/2
    float psb = hps, Pbxx = Bxx, Pbyy = Byy, Pbzz = Bzz, Pbxy = Bxy, Pbxz = Bxz, Pbyz = Byz;
    psb -= (Bxx + Byy + Bzz) * (1.0f / 3.0f);
    Ubx += Bxx * (ax - 2.0f * ux); Abx += Bxx * ux;
    Uby += Byy * (ay - 2.0f * uy); Aby += Byy * uy;
    Ubz += Bzz * (az - 2.0f * uz); Abz += Bzz * uz;
    Ubx += Bxy * (0.5f * ay - uy); Uby += Bxy * (0.5f * ax - ux); Aby += 0.5f * Bxy * ux; Abx += 0.5f * Bxy * uy;
    Ubx += Bxz * (0.5f * az - uz); Ubz += Bxz * (0.5f * ax - ux); Abz += 0.5f * Bxz * ux; Abx += 0.5f * Bxz * uz;
    Uby += Byz * (0.5f * az - uz); Ubz += Byz * (0.5f * ay - uy); Abz += 0.5f * Byz * uy; Aby += 0.5f * Byz * uz;
    float omb = -om1b;

    // ---------------- u = j + a/2
    float jbx = Ubx, jby = Uby, jbz = Ubz;
    Abx += 0.5f * Ubx;
    Aby += 0.5f * Uby;
    Abz += 0.5f * Ubz;

    // ---------------- back through the forces to a
    float irhob = 0.f, nub = 0.f, F0bx, F0by, F0bz;
    float grbx = 0.f, grby = 0.f, grbz = 0.f;
    if (vd) {
        // a = a1 + cnu (Q gr)
        const float Qgx = Qxx * grx + Qxy * gry + Qxz * grz;
        const float Qgy = Qxy * grx + Qyy * gry + Qyz * grz;
        const float Qgz = Qxz * grx + Qyz * gry + Qzz * grz;
        float a1bx = Abx, a1by = Aby, a1bz = Abz;
        const float cnub = Abx * Qgx + Aby * Qgy + Abz * Qgz;
        const float Qbxx = cnu * Abx * grx, Qbyy = cnu * Aby * gry, Qbzz = cnu * Abz * grz;
        const float Qbxy = cnu * (Abx * gry + Aby * grx);
        const float Qbxz = cnu * (Abx * grz + Abz * grx);
        const float Qbyz = cnu * (Aby * grz + Abz * gry);
        grbx += cnu * (Abx * Qxx + Aby * Qxy + Abz * Qxz);
        grby += cnu * (Abx * Qxy + Aby * Qyy + Abz * Qyz);
        grbz += cnu * (Abx * Qxz + Aby * Qyz + Abz * Qzz);
        // cnu = -3 nu omega / rho
        nub += cnub * (-3.0f * omega * irho);
        omb += cnub * (-3.0f * nu * irho);
        irhob += cnub * (-3.0f * nu * omega);
        // Q = P - p*/3 I - u1 u1
        Pbxx += Qbxx; Pbyy += Qbyy; Pbzz += Qbzz; Pbxy += Qbxy; Pbxz += Qbxz; Pbyz += Qbyz;
        psb -= (Qbxx + Qbyy + Qbzz) * (1.0f / 3.0f);
        const float u1bx = -2.0f * Qbxx * u1x - Qbxy * u1y - Qbxz * u1z;
        const float u1by = -2.0f * Qbyy * u1y - Qbxy * u1x - Qbyz * u1z;
        const float u1bz = -2.0f * Qbzz * u1z - Qbxz * u1x - Qbyz * u1y;
        // u1 = j + a1/2
        jbx += u1bx; jby += u1by; jbz += u1bz;
        a1bx += 0.5f * u1bx; a1by += 0.5f * u1by; a1bz += 0.5f * u1bz;
        // a1 = F / rho
        const float Fbx = a1bx * irho, Fby = a1by * irho, Fbz = a1bz * irho;
        irhob += a1bx * Fx + a1by * Fy + a1bz * Fz;
        // F = F0 + cp gr + fe g_body, cp = -p*/3, fe = drho phi
        F0bx = Fbx; F0by = Fby; F0bz = Fbz;
        const float cpb = Fbx * grx + Fby * gry + Fbz * grz;
        grbx += cp * Fbx; grby += cp * Fby; grbz += cp * Fbz;
        const float feb = Fbx * p.gx + Fby * p.gy + Fbz * p.gz;
        phb += p.drho * feb;
        psb -= cpb * (1.0f / 3.0f);
    } else {
        F0bx = Abx * irho;
        F0by = Aby * irho;
        F0bz = Abz * irho;
        irhob += Abx * F0x + Aby * F0y + Abz * F0z;
    }
    // gr = drho grad phi
    Gbx += p.drho * grbx;
    Gby += p.drho * grby;
    Gbz += p.drho * grbz;
    // F0 = mu_phi grad phi
    const float mub = F0bx * gx + F0by * gy + F0bz * gz;
    Gbx += mu_phi * F0bx;
    Gby += mu_phi * F0by;
    Gbz += mu_phi * F0bz;
    // omega = 1 / (1/2 + 3 nu)
    nub += omb * (-3.0f * omega * omega);
    // nu = (mu_g + dmu phi) / rho
    phb += nub * p.dmu * irho;
    irhob += nub * (p.mu_g + p.dmu * ph);
    // 1/rho, rho = rho_g + drho phi
    phb += p.drho * (-irhob * irho * irho);
    // mu_phi = beta4 phi (phi - 1)(phi - 1/2) - kappa_phi lap
    phb += mub * p.beta4 * (3.0f * ph * ph - 3.0f * ph + 0.5f);
    lapb += -p.kappa_phi * mub;

    mb[0] = psb;
    mb[1] = jbx;
    mb[2] = jby;
    mb[3] = jbz;
    mb[4] = Pbxx;
    mb[5] = Pbyy;
    mb[6] = Pbzz;
    mb[7] = Pbxy;
    mb[8] = Pbxz;
    mb[9] = Pbyz;
}

// Reverse of P, V-transpose and H at node (x, y, z): every node writes its
// stencil record rec (cotangents of grad phi-hat, lap phi-hat, and the local
// cotangent of phi-hat); fluid nodes also write their moment cotangents and
// wall nodes the cotangent of their compressive flux.
CAC_HD void adj_main_node(const Grid &g, const DevParams &p, const AdjStep &S, int x, int y, int z)
{
    const Offs o = node_offsets(g, x, y, z);
    const uint32_t n = at<0, 0, 0>(o);
    const uint32_t m = S.nbr[n];
    const uint32_t N = g.N;
    const bool sol = (m & 1u) != 0;
    float4 *rec4 = reinterpret_cast<float4 *>(S.rec);  // (grad x, y, z; Laplacian) cotangents
    float *recl = S.rec + 4u * N;                       // local cotangent of phi-hat
    if (sol && !((~m) & 0x07FFFFFEu)) {  // solid node without fluid neighbours: pass-through only
        rec4[n] = make_float4(0.f, 0.f, 0.f, 0.f);
        recl[n] = S.pb_in[n];
        return;
    }
    // psi on the 3x3x3 patch (zero on solid nodes)
    float pf[27];
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        pf[kk] = S.psi[at<kk % 3 - 1, (kk / 3) % 3 - 1, kk / 9 - 1>(o)];
    });
    // cotangent of the compressive flux a here: the transpose of -kappa div_iso(a) is kappa grad_iso(psi_f)
    float agx, agy, agz;
    patch_grad(pf, agx, agy, agz);
    agx *= p.kappa;
    agy *= p.kappa;
    agz *= p.kappa;
    CAC_PIN(agx);
    CAC_PIN(agy);
    CAC_PIN(agz);
    CAC_SCHED_FENCE();

    // phi-hat patch, its gradient and Laplacian (used on fluid nodes)
    float s[27];
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        s[kk] = S.phihat[at<kk % 3 - 1, (kk / 3) % 3 - 1, kk / 9 - 1>(o)];
    });
    float gx, gy, gz, lap;
    stencil_grad_lap(s, gx, gy, gz, lap);
    CAC_PIN(gx);
    CAC_PIN(gy);
    CAC_PIN(gz);
    CAC_PIN(lap);
    CAC_SCHED_FENCE();

    // identity part of P and V (solid nodes keep phi-hat: pass-through)
    float phb = sol ? S.pb_in[n] : pf[13];

    // MUSCL advection along the three axes
    float ub[3];
    {
        const int xs[5] = {wrapc(x - 2, g.nx), (int)o.x[0], x, (int)o.x[2], wrapc(x + 2, g.nx)};
        const uint32_t ys[5] = {(uint32_t)wrapc(y - 2, g.ny) * (uint32_t)g.nx, o.y[0], o.y[1], o.y[2],
                                (uint32_t)wrapc(y + 2, g.ny) * (uint32_t)g.nx};
        const uint32_t zs[5] = {(uint32_t)wrapc(z - 2, g.nz) * g.nxny, o.z[0], o.z[1], o.z[2],
                                (uint32_t)wrapc(z + 2, g.nz) * g.nxny};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float q[5], uu[5], pp[5];
            bool fl[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const uint32_t id = d == 0 ? (uint32_t)xs[k] + o.y[1] + o.z[1]
                                  : d == 1 ? o.x[1] + ys[k] + o.z[1]
                                           : o.x[1] + o.y[1] + zs[k];
                if (k == 2) {
                    q[k] = s[13];
                    fl[k] = !sol;
                    pp[k] = pf[13];
                } else if (k == 1 || k == 3) {
                    const int kk = 13 + (k - 2) * (d == 0 ? 1 : d == 1 ? 3 : 9);
                    q[k] = s[kk];
                    const int li = d == 0 ? (k == 1 ? 2 : 1) : d == 1 ? (k == 1 ? 4 : 3) : (k == 1 ? 6 : 5);
                    fl[k] = !((m >> li) & 1u);
                    pp[k] = pf[kk];
                } else {
                    q[k] = S.phihat[id];
                    fl[k] = S.solid[id] == 0;
                    pp[k] = S.psi[id];
                }
                uu[k] = S.u[(uint32_t)d * N + id];
            }
            phb += muscl_axis_adj(q, uu, pp, fl, ub[d]);
            CAC_PIN(phb);
            CAC_PIN(ub[d]);
            CAC_SCHED_FENCE();
        }
    }
    if (sol) {
        if (p.wall_compression) {
            S.awb[n] = agx;
            S.awb[N + n] = agy;
            S.awb[2u * N + n] = agz;
        }
        rec4[n] = make_float4(0.f, 0.f, 0.f, 0.f);
        recl[n] = phb;
        return;
    }

    const float ph = s[13];
    float Gbx = 0.f, Gby = 0.f, Gbz = 0.f;
    // compressive flux a = phi (1 - phi) grad / |grad| (Eq. (25)), zero under the guard
    {
        const float g2 = gx * gx + gy * gy + gz * gz;
        if (g2 > p.eps_n2) {
            const float inv = 1.0f / sqrtf(g2);
            const float nx = gx * inv, ny = gy * inv, nz = gz * inv;
            const float an = agx * nx + agy * ny + agz * nz;
            const float h = ph * (1.0f - ph);
            phb += (1.0f - 2.0f * ph) * an;
            const float c = h * inv;
            Gbx += c * (agx - an * nx);
            Gby += c * (agy - an * ny);
            Gbz += c * (agz - an * nz);
        }
    }
    // diffusion D lap(phi): the Laplacian stencil is symmetric
    float lapb = p.D * pf[13];

    CAC_SCHED_FENCE();
    // moments of the pulled populations of the step, in the pair order of hydro_node
    float mom[10] = {__builtin_nontemporal_load(&S.fprev[n]), 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    static_for<13>([&](auto P) {
        constexpr int i = 2 * P + 1;
        const uint32_t src_i = at<Lat::cx[i + 1], Lat::cy[i + 1], Lat::cz[i + 1]>(o);
        const float fi = __builtin_nontemporal_load(
            &S.fprev[((m >> (i + 1)) & 1u) ? (uint32_t)(i + 1) * N + n : (uint32_t)i * N + src_i]);
        const uint32_t src_o = at<Lat::cx[i], Lat::cy[i], Lat::cz[i]>(o);
        const float fo = __builtin_nontemporal_load(
            &S.fprev[((m >> i) & 1u) ? (uint32_t)i * N + n : (uint32_t)(i + 1) * N + src_o]);
        pair_moment_add<i>(fi, fo, mom);
    });
#pragma unroll
    for (int k = 0; k < 10; ++k) CAC_PIN(mom[k]);
    CAC_SCHED_FENCE();
    const float4 *mA = reinterpret_cast<const float4 *>(S.mb_in);
    const float4 *mB = mA + N;
    const float2 *mC = reinterpret_cast<const float2 *>(S.mb_in + 8u * N);
    const float4 a0 = mA[n], b0 = mB[n];
    const float2 c0 = mC[n];
    // cotangent of each pulled population from the node it came from: x + c_i,
    // or x itself with the link reversed when x + c_i is solid (bounce-back)
    auto fbar = [&](auto Ic) -> float {
        constexpr int i = Ic;
        constexpr bool needc = Lat::cz[i] != 0 && (Lat::cx[i] != 0 || Lat::cy[i] != 0);
        const bool rev = ((m >> i) & 1u) != 0;
        const uint32_t id = rev ? n : at<Lat::cx[i], Lat::cy[i], Lat::cz[i]>(o);
        const float2 ci = needc ? mC[id] : make_float2(0.f, 0.f);
        return pop_bar<i>(mA[id], mB[id], ci, rev);
    };
    HermMoments hm;
    static_for<9>([&](auto Lc) {
        constexpr int cy = (int)Lc % 3 - 1, cz = (int)Lc / 3 - 1;
        constexpr int im = Lat::idx(-1, cy, cz), i0 = Lat::idx(0, cy, cz), ip = Lat::idx(1, cy, cz);
        const float gm = fbar(std::integral_constant<int, im>{});
        const float gp = fbar(std::integral_constant<int, ip>{});
        float g0;
        if constexpr (i0 == 0)
            g0 = a0.x;  // the rest population stays at the node
        else
            g0 = fbar(std::integral_constant<int, i0>{});
        hm.add_line<cy, cz>(gm, g0, gp);
        if constexpr ((int)Lc % 2 == 1) {
            hm.pin();
            CAC_SCHED_FENCE();
        }
    });
    const HermBar hb = hm.herm();
    CAC_SCHED_FENCE();
    float mbo[10];
    collide_adj(p, mom, gx, gy, gz, lap, ph, hb, ub[0], ub[1], ub[2], mbo, phb, Gbx, Gby, Gbz, lapb);
    float4 *oA = reinterpret_cast<float4 *>(S.mb_out);
    oA[n] = make_float4(mbo[0], mbo[1], mbo[2], mbo[3]);
    oA[N + n] = make_float4(mbo[4], mbo[5], mbo[6], mbo[7]);
    reinterpret_cast<float2 *>(S.mb_out + 8u * N)[n] = make_float2(mbo[8], mbo[9]);
    rec4[n] = make_float4(Gbx, Gby, Gbz, lapb);
    recl[n] = phb;
}

// Transpose of the gradient and Laplacian stencils: cotangent of phi-hat at
// node (x, y, z) = local part - div_iso(grad cotangents) + lap(Laplacian cotangents).
CAC_HD void adj_assemble_node(const Grid &g, const AdjStep &S, int x, int y, int z)
{
    const Offs o = node_offsets(g, x, y, z);
    const uint32_t n = at<0, 0, 0>(o);
    const uint32_t N = g.N;
    const float4 *rec4 = reinterpret_cast<const float4 *>(S.rec);
    const float L0 = rec4[n].w;
    float dv = 0.f, lp = 0.f;
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        constexpr int dx = kk % 3 - 1, dy = (kk / 3) % 3 - 1, dz = kk / 9 - 1;
        if constexpr (kk != 13) {
            constexpr float w = tw(dx) * tw(dy) * tw(dz);
            const float4 q = rec4[at<dx, dy, dz>(o)];
            if constexpr (dx != 0) dv += ((float)dx * w * (1.0f / 72.0f)) * q.x;
            if constexpr (dy != 0) dv += ((float)dy * w * (1.0f / 72.0f)) * q.y;
            if constexpr (dz != 0) dv += ((float)dz * w * (1.0f / 72.0f)) * q.z;
            lp += (w * (1.0f / 36.0f)) * (q.w - L0);
        }
    });
    S.pb_out[n] = S.rec[4u * N + n] + lp - dv;
}

// Transpose of the ghost update (ghost_node) for every wall node served by
// donor slot d: adds dL/dtheta of each wall node and writes the donor's
// cotangents (of phi_f, and of the gradient at the donor).
CAC_HD void adj_wall_donor(const Grid &g, const DevParams &p, const AdjStep &S, int d)
{
    const uint32_t dn = (uint32_t)S.don_node[d];
    const int fx = (int)(dn % (uint32_t)g.nx);
    const int fy = (int)((dn / (uint32_t)g.nx) % (uint32_t)g.ny);
    const int fz = (int)(dn / g.nxny);
    const Offs o = node_offsets(g, fx, fy, fz);
    const uint32_t m = S.nbr[dn];
    float s[27];
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        constexpr int dx = kk % 3 - 1, dy = (kk / 3) % 3 - 1, dz = kk / 9 - 1;
        constexpr int li = Lat::idx(dx, dy, dz);
        const uint32_t id = at<dx, dy, dz>(o);
        s[kk] = ((m >> li) & 1u) ? S.phiold[id] : S.phihat[id];
    });
    float gx, gy, gz, lap;
    stencil_grad_lap(s, gx, gy, gz, lap);
    const float phif = s[13];
    const float l2 = 4.0f * phif * (1.0f - phif);
    const float lam = sqrtf(l2 > 0.0f ? l2 : 0.0f);
    const float lamp = l2 > 1e-12f ? (2.0f - 4.0f * phif) / lam : 0.0f;  // d lambda_s / d phi_f
    float pfb = 0.f, Gsx = 0.f, Gsy = 0.f, Gsz = 0.f;
    for (int e = S.don_start[d]; e < S.don_start[d + 1]; ++e) {
        const int k = S.don_wall[e];
        const int q = S.wq[k];
        const uint32_t b = (uint32_t)S.widx[k];
        float cq[3] = {0.f, 0.f, 0.f};
        static_for<27>([&](auto I) {
            if (q == I) {
                cq[0] = (float)Lat::cx[I];
                cq[1] = (float)Lat::cy[I];
                cq[2] = (float)Lat::cz[I];
            }
        });
        const float nx = S.wn[3 * k], ny = S.wn[3 * k + 1], nz = S.wn[3 * k + 2];
        // forward of ghost_node
        const float gn = gx * nx + gy * ny + gz * nz;
        const float px = gx - gn * nx, py = gy - gn * ny, pz = gz - gn * nz;
        const float t = sqrtf(px * px + py * py + pz * pz);
        const float thc = 3.14159265358979f - S.theta[k];
        float sn, cs;
        sincosf(thc, &sn, &cs);
        const bool reg = fabsf(sn) < p.sin_tol;
        const float cot = reg ? copysignf(p.cot_max, cs) : cs / sn;
        const float dnv = -t * cot;
        const float cgx = px + dnv * nx, cgy = py + dnv * ny, cgz = pz + dnv * nz;
        const float gcq = cgx * cq[0] + cgy * cq[1] + cgz * cq[2];
        const float gv = phif - lam * gcq;
        // reverse
        float gb = S.pb_out[b];
        float Cbx = 0.f, Cby = 0.f, Cbz = 0.f;
        if (p.wall_compression) {
            const float c2 = cgx * cgx + cgy * cgy + cgz * cgz;
            if (c2 > p.eps_n2) {
                const float ic = 1.0f / sqrtf(c2);
                const float hx = cgx * ic, hy = cgy * ic, hz = cgz * ic;
                const float abx = S.awb[b], aby = S.awb[g.N + b], abz = S.awb[2u * g.N + b];
                const float an = abx * hx + aby * hy + abz * hz;
                gb += (1.0f - 2.0f * gv) * an;
                const float c = gv * (1.0f - gv) * ic;
                Cbx += c * (abx - an * hx);
                Cby += c * (aby - an * hy);
                Cbz += c * (abz - an * hz);
            }
        }
        // g = phi_f - lambda_s (grad_c . c_q)   (Eq. (46) with r_fs = -c_q)
        pfb += gb * (1.0f - lamp * gcq);
        Cbx -= gb * lam * cq[0];
        Cby -= gb * lam * cq[1];
        Cbz -= gb * lam * cq[2];
        // grad_c = grad_par + dn n, dn = -t cot (Eqs. (44)-(45))
        const float dnb = Cbx * nx + Cby * ny + Cbz * nz;
        float Pbx = Cbx, Pby = Cby, Pbz = Cbz;
        const float tb = -dnb * cot;
        if (!reg) S.thb[k] += (double)(-dnb * t / (sn * sn));  // d cot(pi - theta)/d theta = 1/sin^2
        if (t > 1e-12f) {
            const float it = tb / t;
            Pbx += it * px;
            Pby += it * py;
            Pbz += it * pz;
        }
        // grad_par = (I - n n) grad (Eq. (42))
        const float pn = Pbx * nx + Pby * ny + Pbz * nz;
        Gsx += Pbx - pn * nx;
        Gsy += Pby - pn * ny;
        Gsz += Pbz - pn * nz;
    }
    S.dg[d] = make_float4(pfb, Gsx, Gsy, Gsz);
}

// Cotangent of phi^n on a node next to a donor: phi-hat's cotangent (not on
// active wall nodes, whose phi-hat is the new ghost) plus the transpose of the
// donor values and donor gradients (Eq. (22)) that read it.
CAC_HD void adj_fix_node(const Grid &g, const AdjStep &S, uint32_t e)
{
    const uint32_t ent = S.near[e];
    const uint32_t zn = ent & 0x7FFFFFFFu;
    const bool wall = (ent >> 31) != 0;
    const int x = (int)(zn % (uint32_t)g.nx);
    const int y = (int)((zn / (uint32_t)g.nx) % (uint32_t)g.ny);
    const int z = (int)(zn / g.nxny);
    const Offs o = node_offsets(g, x, y, z);
    float v = wall ? 0.0f : S.pb_out[zn];
    const int d0 = S.don_map[zn];
    if (d0 >= 0) v += S.dg[d0].x;
    static_for<27>([&](auto K) {
        constexpr int kk = K;
        constexpr int dx = kk % 3 - 1, dy = (kk / 3) % 3 - 1, dz = kk / 9 - 1;
        if constexpr (kk != 13) {
            constexpr float w = tw(dx) * tw(dy) * tw(dz) * (1.0f / 72.0f);
            const int dj = S.don_map[at<-dx, -dy, -dz>(o)];  // donor at z - c reads this node through +c
            if (dj >= 0) {
                const float4 q = S.dg[dj];
                v += w * ((float)dx * q.y + (float)dy * q.z + (float)dz * q.w);
            }
        }
    });
    S.pb_out[zn] = v;
}

}  // namespace cac
