// adj_emu.cpp -- test harness: the reverse-step node bodies of libcac
// (adjoint_device.hpp) compiled for the host and run node by node over a tiny
// grid, one reverse step per call.  Lets the CPU test suite check the
// hand-written transposes against the oracle adjoint without a GPU.
// emu_reverse_step: prm = (rho_l, rho_g, nu_l, nu_g, sigma, delta, D, g[3],
// eps_phi, eps_n, sin_tol, cot_max, volume_correction, wall_compression);
// the forward state of the step and the cotangents use the library layouts.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "adjoint_device.hpp"
#include "adjoint_tables.hpp"

using namespace cac;

extern "C" int emu_reverse_step(int nx, int ny, int nz, const double *prm, const uint8_t *solid, int nwall,
                                const int32_t *widx, const int32_t *n6, const int32_t *wdonor, const float *theta,
                                double M_target, const float *fprev, const float *phihat, const float *phiold,
                                const float *u, const float *phistar, const float *pb_in, const float *mb_in,
                                float *pb_out, float *mb_out, double *thb)
{
    Grid g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.N = (uint32_t)nx * ny * nz;
    g.nxny = (uint32_t)nx * ny;
    const uint32_t N = g.N;
    // prm: rho_l rho_g nu_l nu_g sigma delta D g0 g1 g2 eps_phi eps_n sin_tol cot_max vc wc
    DevParams p{};
    p.rho_g = (float)prm[1];
    p.drho = (float)(prm[0] - prm[1]);
    p.mu_g = (float)(prm[1] * prm[3]);
    p.dmu = (float)(prm[0] * prm[2] - prm[1] * prm[3]);
    p.beta4 = (float)(4.0 * 12.0 * prm[4] / prm[5]);
    p.kappa_phi = (float)(1.5 * prm[4] * prm[5]);
    p.D = (float)prm[6];
    p.kappa = (float)(4.0 * prm[6] / prm[5]);
    p.gx = (float)prm[7]; p.gy = (float)prm[8]; p.gz = (float)prm[9];
    p.eps_phi = (float)prm[10];
    p.eps_n2 = (float)(prm[11] * prm[11]);
    p.sin_tol = (float)prm[12];
    p.cot_max = (float)prm[13];
    p.volume_correction = prm[14] != 0;
    p.wall_compression = prm[15] != 0;
    p.ghost_lambda = 1;
    p.variable_density = prm[0] != prm[1];
    std::vector<uint32_t> nbr(N);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                uint32_t n = x + nx * (y + ny * z), m = solid[n] ? 1u : 0u;
                for (int i = 1; i < 27; ++i) {
                    int xx = (x + Lat::cx[i] + nx) % nx, yy = (y + Lat::cy[i] + ny) % ny, zz = (z + Lat::cz[i] + nz) % nz;
                    if (solid[xx + nx * (yy + ny * zz)]) m |= 1u << i;
                }
                nbr[n] = m;
            }
    std::vector<uint8_t> wq(nwall);
    std::vector<float> wn(3 * nwall);
    for (int k = 0; k < nwall; ++k) {
        wq[k] = wdonor[k] < 0 ? 255 : (uint8_t)wdonor[k];
        double a = n6[3 * k], b = n6[3 * k + 1], c = n6[3 * k + 2], nn = std::sqrt(a * a + b * b + c * c);
        wn[3 * k] = nn > 0 ? (float)(a / nn) : 0.f;
        wn[3 * k + 1] = nn > 0 ? (float)(b / nn) : 0.f;
        wn[3 * k + 2] = nn > 0 ? (float)(c / nn) : 0.f;
    }
    DonorTables D;
    build_donor_tables(g, widx, wdonor, nwall, D);
    std::vector<float> rec(5 * (size_t)N, 0.f), awb(3 * (size_t)N, 0.f), psi(N, 0.f);
    std::vector<float4> dg(D.don_node.size() + 1);
    double rs[4] = {0, 0, 0, 0}, scal[8] = {M_target, 0, 0, 0, 0, 0, 0, 0};
    // V transpose sums
    double a = 0, b = 0, c = 0;
    for (uint32_t n = 0; n < N; ++n) {
        if (solid[n]) continue;
        float v = phistar[n];
        b += v;
        if (v > p.eps_phi && v < 1.0f - p.eps_phi) {
            double ch = (double)v * (1.0 - (double)v);
            c += ch;
            a += (double)pb_in[n] * ch;
        }
    }
    bool on = p.volume_correction && c > 0.0;
    rs[0] = on ? (M_target - b) / c : 0.0;
    rs[1] = on ? a / c : 0.0;
    AdjStep S{};
    S.fprev = fprev; S.phihat = phihat; S.phiold = phiold; S.u = u; S.phistar = phistar;
    S.pb_in = pb_in; S.mb_in = mb_in; S.pb_out = pb_out; S.mb_out = mb_out;
    S.rec = rec.data(); S.awb = awb.data(); S.psi = psi.data(); S.nbr = nbr.data(); S.solid = solid;
    S.widx = widx; S.wq = wq.data(); S.wn = wn.data(); S.theta = theta;
    S.don_start = D.don_start.data(); S.don_wall = D.don_wall.data(); S.don_node = D.don_node.data();
    S.ndon = (int)D.don_node.size(); S.don_map = D.don_map.data(); S.dg = dg.data();
    S.near = D.near.data(); S.nnear = (uint32_t)D.near.size(); S.thb = thb; S.rs = rs; S.scal = scal;
    for (uint32_t n = 0; n < N; ++n) adj_psi_node(p, S, n);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) adj_main_node(g, p, S, x, y, z);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) adj_assemble_node(g, S, x, y, z);
    for (int d = 0; d < S.ndon; ++d) adj_wall_donor(g, p, S, d);
    for (uint32_t e = 0; e < S.nnear; ++e) adj_fix_node(g, S, e);
    return 0;
}
