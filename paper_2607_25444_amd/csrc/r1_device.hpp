// r1_device.hpp -- device bodies of the gradient-form hydrodynamic substep
// (collision = 1; the thread-safe formulation of Sec. II A with the
// non-equilibrium moment of Eq. (15)), shared by the single-lattice kernels
// (r1.hip) and the batched ones (batch.hip).  Not part of the public ABI.
#pragma once

#include "step_device.hpp"

namespace cac {

// Gradient form of the non-equilibrium moment at fluid node n (solid-neighbour
// mask m) from its velocity stencil s*[k], k = (dz+1)*9 + (dy+1)*3 + (dx+1),
// in which solid neighbours already hold the mirror image -u of the node;
// then its post-collision populations
// (non-temporal stores: read once, by the pull).
__device__ __forceinline__ void r1_rebuild(uint32_t N, uint32_t n, const float (&sx)[27], const float (&sy)[27],
                                           const float (&sz)[27], const float *__restrict__ rec,
                                           float *__restrict__ fout)
{
    // d_b u_a by the isotropic gradient of each component
    float xx_, xy_, xz_, yx_, yy_, yz_, zx_, zy_, zz_, l_;
    stencil_grad_lap(sx, xx_, yx_, zx_, l_);  // d_x u_x, d_y u_x, d_z u_x
    stencil_grad_lap(sy, xy_, yy_, zy_, l_);  // d_x u_y, d_y u_y, d_z u_y
    stencil_grad_lap(sz, xz_, yz_, zz_, l_);  // d_x u_z, d_y u_z, d_z u_z

    Macro M;
    M.ps = rec[n];
    M.ax = rec[N + n];
    M.ay = rec[2u * N + n];
    M.az = rec[3u * N + n];
    M.omega = rec[4u * N + n];
    M.ux = sx[13];
    M.uy = sy[13];
    M.uz = sz[13];
    const float c = -(1.0f / 3.0f) * fast_rcp(M.omega);
    float A2[6];
    A2[0] = c * (2.0f * xx_);
    A2[1] = c * (2.0f * yy_);
    A2[2] = c * (2.0f * zz_);
    A2[3] = c * (xy_ + yx_);
    A2[4] = c * (xz_ + zx_);
    A2[5] = c * (yz_ + zy_);
    const Herm h = herm_post(M, A2);

    __builtin_nontemporal_store(Lat::w(0) * (h.ps - 4.5f * h.tr3), &fout[n]);
    static_for<13>([&](auto P) {
        constexpr int i = 2 * P + 1;
        float E, O;
        herm_pair<i>(h, E, O);
        __builtin_nontemporal_store(E + O, &fout[(uint32_t)i * N + n]);
        __builtin_nontemporal_store(E - O, &fout[(uint32_t)(i + 1) * N + n]);
    });
}

// Stream and collide at fluid node x: pull of the rebuilt populations, then
// the macroscopic part of the collision; writes the record and u.  NTL:
// non-temporal population loads (row-wide tiles, as in the local-moment
// kernel).
template <bool SELF, bool NTL>
__device__ __forceinline__ void r1_stream_node(const Grid &g, const DevParams &p, const Node &nd,
                                               const float *__restrict__ fin, const float *__restrict__ phi,
                                               const uint32_t *__restrict__ nbr, const float *__restrict__ pstar0,
                                               float *__restrict__ u, float *__restrict__ rec,
                                               uint32_t *__restrict__ flag, bool walls = true)
{
    if (!nd.in) return;
    const Offs o = node_offsets(g, nd.x, nd.y, nd.z);
    const uint32_t n = at<0, 0, 0>(o);
    // walls == false: no node of the caller's tile is solid or next to a solid node
    const uint32_t m = walls ? nbr[n] : 0u;
    if (m & 1u) return;
    const uint32_t N = g.N;

    float s[27];
    static_for<27>([&](auto J) {
        constexpr int kk = J;
        s[kk] = phi[at<kk % 3 - 1, (kk / 3) % 3 - 1, kk / 9 - 1>(o)];
    });
    float f[27];
    if constexpr (SELF) {
        const float ps0 = pstar0[n], ux0 = u[n], uy0 = u[N + n], uz0 = u[2u * N + n];
        static_for<27>([&](auto J) {
            constexpr int i = J;
            f[i] = feq_one<i>(ps0, ux0, uy0, uz0);
        });
    } else {
        pull_populations<NTL>(g, o, n, m, fin, f);
    }

    float gx, gy, gz, lap;
    stencil_grad_lap(s, gx, gy, gz, lap);
    float mom[10];
    pair_moments(f, mom);
    const Macro M = macro_node(p, s[13], gx, gy, gz, lap, mom);

    rec[n] = M.ps;
    rec[N + n] = M.ax;
    rec[2u * N + n] = M.ay;
    rec[3u * N + n] = M.az;
    rec[4u * N + n] = M.omega;
    u[n] = M.ux;
    u[N + n] = M.uy;
    u[2u * N + n] = M.uz;
    if (!(isfinite(M.ux) && isfinite(M.uy) && isfinite(M.uz) && isfinite(M.ps))) flag[0] = 1u;
}

// Rebuild pass over column tile `tile` of CX x CY nodes marching through a z-chunk:
// the velocity planes z-1, z, z+1 (with a one-node halo in x and y) sit in a
// ring of four LDS slots, so each velocity value is loaded from memory about
// (CX+2)(CY+2)/(CX CY) times per chunk instead of 27 times.  Plane z+2 is
// fetched into registers while plane z is rebuilt and is written into the ring
// at the start of plane z+1, into the slot of plane z-2.  The last reads of
// that slot belong to the rebuild of plane z-1, which every wave finishes
// before it arrives at the barrier of plane z; a wave starting plane z+1 has
// passed that barrier, so one barrier per plane suffices.  Every thread takes
// part in the loads and the barriers; threads outside the grid skip only the
// node update.
template <int CX, int CY>
__device__ __forceinline__ void r1_rebuild_tile(const Grid &g, const PhaseTiling &pt, uint32_t tile,
                                                const float *__restrict__ rec, const float *__restrict__ u,
                                                const uint32_t *__restrict__ nbr, float *__restrict__ fout)
{
    constexpr int NT = CX * CY, LX = CX + 2, LP = (CX + 2) * (CY + 2);
    constexpr int PQ = (LP + NT - 1) / NT;  // halo-plane points per thread
    __shared__ float su[4][3][LP];          // [slot][component][position]
    const uint32_t txy = (uint32_t)pt.ntx * (uint32_t)pt.nty;
    const uint32_t zci = tile / txy, rxy = tile - zci * txy;
    const uint32_t tyi = rxy / (uint32_t)pt.ntx, txi = rxy - tyi * (uint32_t)pt.ntx;
    const int x0 = (int)txi * CX, y0 = (int)tyi * CY;
    const int z0 = (int)zci * pt.zc, z1 = min(z0 + pt.zc, g.nz);
    const int tid = (int)threadIdx.x, lx = tid % CX, ly = tid / CX;
    const int x = x0 + lx, y = y0 + ly;
    const bool inxy = x < g.nx && y < g.ny;
    const uint32_t N = g.N;

    // in-plane node offsets of this thread's halo-plane points (periodic wrap)
    uint32_t qoff[PQ];
#pragma unroll
    for (int r = 0; r < PQ; ++r) {
        const int q = tid + r * NT, qx = q % LX, qy = q / LX;
        qoff[r] = q < LP ? (uint32_t)wrapc(x0 - 1 + qx, g.nx) + (uint32_t)wrapc(y0 - 1 + qy, g.ny) * (uint32_t)g.nx
                         : 0u;
    }
    float pre[PQ][3];
    auto fetch = [&](int zg) {
        const uint32_t zo = (uint32_t)wrapc(zg, g.nz) * g.nxny;
#pragma unroll
        for (int r = 0; r < PQ; ++r)
            if (tid + r * NT < LP) {
                const uint32_t gi = qoff[r] + zo;
                pre[r][0] = u[gi];
                pre[r][1] = u[N + gi];
                pre[r][2] = u[2u * N + gi];
            }
    };
    auto slot = [&](int zg) { return (zg - z0 + 4) & 3; };  // zg >= z0 - 1
    auto store = [&](int zg) {
        const int s = slot(zg);
#pragma unroll
        for (int r = 0; r < PQ; ++r)
            if (tid + r * NT < LP) {
                su[s][0][tid + r * NT] = pre[r][0];
                su[s][1][tid + r * NT] = pre[r][1];
                su[s][2][tid + r * NT] = pre[r][2];
            }
    };
    fetch(z0 - 1);
    store(z0 - 1);
    fetch(z0);
    store(z0);
    fetch(z0 + 1);
    for (int z = z0; z < z1; ++z) {
        store(z + 1);
        if (z + 1 < z1) fetch(z + 2);
        __syncthreads();
        if (inxy) {
            const uint32_t n = (uint32_t)x + (uint32_t)y * (uint32_t)g.nx + (uint32_t)z * g.nxny;
            const uint32_t m = nbr[n];
            if (!(m & 1u)) {
                const int sl[3] = {slot(z - 1), slot(z), slot(z + 1)};
                const int qc = (lx + 1) + LX * (ly + 1);
                const float cx0 = su[sl[1]][0][qc], cy0 = su[sl[1]][1][qc], cz0 = su[sl[1]][2][qc];
                float sx[27], sy[27], sz[27];
                static_for<27>([&](auto J) {
                    constexpr int kk = J;
                    constexpr int dx = kk % 3 - 1, dy = (kk / 3) % 3 - 1, dz = kk / 9 - 1;
                    constexpr int li = Lat::idx(dx, dy, dz);
                    const int q = (lx + 1 + dx) + LX * (ly + 1 + dy);
                    const int sv = sl[dz + 1];
                    // a solid neighbour holds the mirror image -u of the node: the
                    // velocity vanishes at the half-link, where bounce-back puts the wall
                    const bool sol = ((m >> li) & 1u) != 0u;
                    const float vx = su[sv][0][q], vy = su[sv][1][q], vz = su[sv][2][q];
                    sx[kk] = sol ? -cx0 : vx;
                    sy[kk] = sol ? -cy0 : vy;
                    sz[kk] = sol ? -cz0 : vz;
                });
                r1_rebuild(N, n, sx, sy, sz, rec, fout);
            }
        }
    }
}

}  // namespace cac
