// runtime.cpp -- host side of libcac: handle, geometry preprocessing, buffer
// management, step sequencing and the C ABI declared in include/cac.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cac.h"
#include "handle.hpp"
#include "probe.hpp"

using namespace cac;

namespace cac {
DevParams make_dev_params(const cac_params &p);
Tiling make_tiling(const Grid &g, int bx, int by, int bz);
void build_geometry(const Grid &g, const uint8_t *solid, std::vector<uint32_t> &nbr, std::vector<int32_t> &widx,
                    std::vector<int32_t> &wn6, std::vector<int32_t> &wdonor, int &nskip);
bool valid_params(const cac_params &p);
const char *free_call_error();  // last failed handle-free call of this thread (noalloc.hip)
}  // namespace cac

namespace cac {

cac_status fail(cac_handle *h, cac_status s, const char *fmt, ...)
{
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return s;
}

void *dev_alloc(cac_handle *h, size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    if (h->alloc) return h->alloc(bytes, h->alloc_user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    h->owned.push_back(p);
    return p;
}

}  // namespace cac

namespace cac {

bool valid_params(const cac_params &p)
{
    return p.rho_l > 0 && p.rho_g > 0 && p.nu_l > 0 && p.nu_g > 0 && p.delta > 0 && p.D >= 0 && p.sigma >= 0 &&
           p.eps_phi >= 0 && p.eps_phi < 0.5 && (p.collision == 0 || p.collision == 1) &&
           (p.ghost_localization == 0 || p.ghost_localization == 1);
}

DevParams make_dev_params(const cac_params &p)
{
    DevParams d{};
    d.rho_g = (float)p.rho_g;
    d.drho = (float)(p.rho_l - p.rho_g);
    d.mu_g = (float)(p.rho_g * p.nu_g);
    d.dmu = (float)(p.rho_l * p.nu_l - p.rho_g * p.nu_g);
    d.beta4 = (float)(4.0 * 12.0 * p.sigma / p.delta);
    d.kappa_phi = (float)(1.5 * p.sigma * p.delta);
    d.D = (float)p.D;
    d.kappa = (float)(4.0 * p.D / p.delta);
    d.gx = (float)p.g[0];
    d.gy = (float)p.g[1];
    d.gz = (float)p.g[2];
    d.eps_phi = (float)p.eps_phi;
    d.eps_n2 = (float)(p.eps_n * p.eps_n);
    d.sin_tol = (float)p.sin_tol;
    d.cot_max = (float)p.cot_max;
    d.volume_correction = p.volume_correction ? 1 : 0;
    d.wall_compression = p.wall_compression ? 1 : 0;
    d.ghost_lambda = p.ghost_localization ? 1 : 0;
    d.variable_density = (p.rho_l != p.rho_g) ? 1 : 0;
    return d;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// LDS to reserve per collide-stream workgroup of nt threads so that at most
// 4 waves per SIMD (16 per CU) are resident: the workgroups that fit a CU's
// LDS then number 16 / (nt / 64).  The collide-stream uses no LDS; with fewer
// workgroups in flight fewer 27-plane streams compete for HBM, and it runs
// 5-6% faster than at its register-limited 6-7 waves per SIMD.  0 when the
// device does not report its LDS size.
uint32_t hydro_lds_reserve(int dev, int nt)
{
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || lds <= 0)
        return 0u;
    const int wgs = std::max(1, 16 / (nt / 64));
    const uint32_t r = (uint32_t)(lds / (wgs + 1) + 64);
    return r <= 65536u ? r : 0u;
}

Tiling make_tiling(const Grid &g, int bx, int by, int bz)
{
    Tiling t{};
    t.bx = bx;
    t.by = by;
    t.bz = bz;
    t.tx = (g.nx + bx - 1) / bx;
    t.ty = (g.ny + by - 1) / by;
    t.tz = (g.nz + bz - 1) / bz;
    t.ntiles = (uint32_t)t.tx * (uint32_t)t.ty * (uint32_t)t.tz;
    return t;
}

// Default tile: 64 nodes along x when the row is long enough, else the row.
void default_tile(const Grid &g, int &bx, int &by, int &bz)
{
    bx = g.nx >= 64 ? 64 : (g.nx >= 32 ? 32 : 16);
    by = 256 / bx >= 4 ? 4 : 256 / bx;
    bz = 256 / (bx * by);
}

// Integer comparison of donor scores m/sqrt(k) (k = |c|^2 in {1,2,3}):
// true when m1/sqrt(k1) > m2/sqrt(k2), evaluated exactly.
bool score_greater(long m1, long k1, long m2, long k2)
{
    const int s1 = (m1 > 0) - (m1 < 0), s2 = (m2 > 0) - (m2 < 0);
    if (s1 != s2) return s1 > s2;
    if (s1 == 0) return false;
    const long l = m1 * m1 * k2, r = m2 * m2 * k1;
    return s1 > 0 ? l > r : l < r;
}

// nbr bitmask and the wall-node tables of Sec. II B.
void build_geometry(const Grid &g, const uint8_t *solid, std::vector<uint32_t> &nbr, std::vector<int32_t> &widx,
                    std::vector<int32_t> &wn6, std::vector<int32_t> &wdonor, int &nskip)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    nbr.assign(g.N, 0u);
    widx.clear();
    wn6.clear();
    wdonor.clear();
    nskip = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint32_t n = (uint32_t)x + (uint32_t)nx * ((uint32_t)y + (uint32_t)ny * (uint32_t)z);
                uint32_t m = solid[n] ? 1u : 0u;
                for (int i = 1; i < 27; ++i) {
                    const int xx = (x + Lat::cx[i] + nx) % nx, yy = (y + Lat::cy[i] + ny) % ny,
                              zz = (z + Lat::cz[i] + nz) % nz;
                    const uint32_t nn = (uint32_t)xx + (uint32_t)nx * ((uint32_t)yy + (uint32_t)ny * (uint32_t)zz);
                    if (solid[nn]) m |= 1u << i;
                }
                nbr[n] = m;
                if (!(m & 1u)) continue;
                // wall node: at least one fluid link
                const uint32_t fluid_links = (~m) & 0x07FFFFFEu;
                if (!fluid_links) continue;
                // six times the unnormalised normal: sum over fluid links of (6/|c|^2)(-c)
                long n6[3] = {0, 0, 0};
                for (int i = 1; i < 27; ++i)
                    if ((fluid_links >> i) & 1u) {
                        const long w6 = 6 / Lat::norm2(i);
                        n6[0] -= w6 * Lat::cx[i];
                        n6[1] -= w6 * Lat::cy[i];
                        n6[2] -= w6 * Lat::cz[i];
                    }
                int best = -1;
                if (n6[0] || n6[1] || n6[2]) {
                    long bm = 0, bk = 1;
                    for (int i = 1; i < 27; ++i) {
                        if (!((fluid_links >> i) & 1u)) continue;
                        const long mm = -(Lat::cx[i] * n6[0] + Lat::cy[i] * n6[1] + Lat::cz[i] * n6[2]);
                        const long kk = Lat::norm2(i);
                        if (best < 0 || score_greater(mm, kk, bm, bk)) {
                            best = i;
                            bm = mm;
                            bk = kk;
                        }
                    }
                } else {
                    ++nskip;
                }
                widx.push_back((int32_t)n);
                wn6.push_back((int32_t)n6[0]);
                wn6.push_back((int32_t)n6[1]);
                wn6.push_back((int32_t)n6[2]);
                wdonor.push_back(best);
            }
}

}  // namespace cac

namespace cac {

hipError_t launch_h(cac_handle *h, int c)
{
    if (h->prm.collision == 0) return launch_hydro(h->g, h->t, h->dp, h->F, c, c, h->stream);
    // gradient form: the first step after the state is set pulls each node's own equilibrium
    if (h->steps > 0) {
        const hipError_t e = launch_r1_rebuild(h->g, h->t, h->dp, h->F, h->stream);
        if (e != hipSuccess) return e;
    }
    return launch_r1_stream(h->g, h->t, h->dp, h->F, c, h->steps == 0, h->stream);
}

cac_status run_step(cac_handle *h)
{
    const int c = h->cur;
    HIPCHK(h, launch_ghost(h->g, h->dp, h->F, c, h->stream));
    HIPCHK(h, launch_h(h, c));
    HIPCHK(h, launch_phase(h->g, h->t, h->dp, h->F, c, h->stream));
    HIPCHK(h, launch_volume(h->g, h->t, h->dp, h->F, c ^ 1, h->stream));
    h->cur ^= 1;
    h->steps++;
    return CAC_OK;
}

}  // namespace cac

namespace {

void drop_graphs(cac_handle *h)
{
    for (auto &e : h->gexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

// Capture one step starting from parity `par` into gexec[par].
cac_status capture_step(cac_handle *h, int par)
{
    hipGraph_t graph = nullptr;
    const int save_cur = h->cur;
    const long long save_steps = h->steps;
    if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    h->cur = par;
    hipStream_t user = h->stream;
    h->stream = h->cap_stream;
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        h->stream = user;
        h->cur = save_cur;
        return fail(h, CAC_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
    }
    cac_status st = run_step(h);
    e = hipStreamEndCapture(h->stream, &graph);
    h->stream = user;
    h->cur = save_cur;
    h->steps = save_steps;
    if (st != CAC_OK) return st;
    if (e != hipSuccess) return fail(h, CAC_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h->gexec[par], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(h, CAC_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    return CAC_OK;
}

}  // namespace

extern "C" {

const char *cac_status_string(cac_status s)
{
    switch (s) {
    case CAC_OK: return "ok";
    case CAC_ERR_ARG: return "invalid argument";
    case CAC_ERR_GEOMETRY: return "invalid geometry";
    case CAC_ERR_HIP: return "HIP runtime error";
    case CAC_ERR_NONFINITE: return "non-finite value in the state";
    case CAC_ERR_STATE: return "call out of order";
    case CAC_ERR_ALLOC: return "device allocation failed";
    }
    return "unknown status";
}

cac_status cac_last_error(cac_handle *h, char *buf, size_t n)
{
    if (!buf || n == 0) return CAC_ERR_ARG;
    snprintf(buf, n, "%s", h ? h->err.c_str() : free_call_error());
    return CAC_OK;
}

cac_status cac_default_params(cac_params *p)
{
    if (!p) return CAC_ERR_ARG;
    *p = cac_params{};
    p->rho_l = p->rho_g = 1.0;
    p->nu_l = p->nu_g = 0.04;
    p->sigma = 0.02;
    p->delta = 4.0;
    p->D = 0.1;
    p->eps_phi = 1e-3;
    p->eps_n = 1e-12;
    p->sin_tol = 1e-6;
    p->cot_max = 1e6;
    p->volume_correction = 1;
    p->wall_compression = 1;
    p->collision = 0;
    p->ghost_localization = 1;
    return CAC_OK;
}

cac_status cac_init(cac_handle **hp, int nx, int ny, int nz, const cac_params *p, cac_alloc_fn alloc,
                    void *alloc_user, void *hip_stream)
{
    if (!hp || !p) return CAC_ERR_ARG;
    *hp = nullptr;
    // every axis needs two nodes: the MUSCL stencil reaches two nodes along each axis
    if (nx < 2 || ny < 2 || nz < 2) return CAC_ERR_ARG;
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    // population index i * N + n is an unsigned 32-bit integer in the kernels
    if (27ull * N > 0xFFFFFFFFull) return CAC_ERR_ARG;
    if (!valid_params(*p)) return CAC_ERR_ARG;
    cac_handle *h = new cac_handle();
    h->prm = *p;
    h->dp = make_dev_params(*p);
    h->g.nx = nx;
    h->g.ny = ny;
    h->g.nz = nz;
    h->g.N = (uint32_t)N;
    h->g.nxny = (uint32_t)nx * (uint32_t)ny;
    int bx, by, bz;
    default_tile(h->g, bx, by, bz);
    h->t = make_tiling(h->g, bx, by, bz);
    h->stream = (hipStream_t)hip_stream;
    h->alloc = alloc;
    h->alloc_user = alloc_user;
    if (hipGetDevice(&h->dev) != hipSuccess) {
        delete h;
        return CAC_ERR_HIP;
    }
    h->t.hyd_lds = hydro_lds_reserve(h->dev, bx * by * bz);
    Fields &F = h->F;
    const size_t Nf = (size_t)N;
    for (int k = 0; k < 2; ++k) {
        F.f[k] = (float *)dev_alloc(h, 27 * Nf * sizeof(float));
        F.phi[k] = (float *)dev_alloc(h, Nf * sizeof(float));
    }
    F.u = (float *)dev_alloc(h, 3 * Nf * sizeof(float));
    F.a = (float *)dev_alloc(h, 3 * Nf * sizeof(float));
    F.nbr = (uint32_t *)dev_alloc(h, Nf * sizeof(uint32_t));
    F.solid = (uint8_t *)dev_alloc(h, Nf);
    F.pstar0 = (float *)dev_alloc(h, Nf * sizeof(float));
    h->partial_cap = std::max({(size_t)(Nf / 64 + 64), (size_t)h->t.ntiles + 64, (size_t)phase_tiles_max(h->g) + 64});
    F.partial = (double2 *)dev_alloc(h, h->partial_cap * sizeof(double2));
    F.scal = (double *)dev_alloc(h, 8 * sizeof(double));
    F.flag = (uint32_t *)dev_alloc(h, 256);
    const size_t nchunk = (Nf + 1023) / 1024;
    F.chunk = (uint8_t *)dev_alloc(h, nchunk);
    F.twall = (uint8_t *)dev_alloc(h, h->partial_cap);
    if (!F.f[0] || !F.f[1] || !F.phi[0] || !F.phi[1] || !F.u || !F.a || !F.nbr || !F.solid || !F.pstar0 ||
        !F.partial || !F.scal || !F.flag || !F.chunk || !F.twall) {
        for (void *q : h->owned) (void)hipFree(q);
        delete h;
        return CAC_ERR_ALLOC;
    }
    if (hipMemsetAsync(F.flag, 0, 256, h->stream) != hipSuccess ||
        hipMemsetAsync(F.scal, 0, 8 * sizeof(double), h->stream) != hipSuccess ||
        hipMemsetAsync(F.chunk, 0, nchunk, h->stream) != hipSuccess ||
        hipMemsetAsync(F.twall, 1, h->partial_cap, h->stream) != hipSuccess) {
        for (void *q : h->owned) (void)hipFree(q);
        delete h;
        return CAC_ERR_HIP;
    }
    *hp = h;
    return CAC_OK;
}

cac_status cac_set_geometry(cac_handle *h, const uint8_t *solid, const float *theta_rad)
{
    if (!h) return CAC_ERR_ARG;
    if (!solid) return fail(h, CAC_ERR_ARG, "solid mask is NULL");
    const uint32_t N = h->g.N;
    uint32_t nfluid = 0;
    for (uint32_t n = 0; n < N; ++n) nfluid += solid[n] ? 0u : 1u;
    if (nfluid == 0) return fail(h, CAC_ERR_GEOMETRY, "the mask has no fluid node");
    std::vector<uint32_t> nbr;
    build_geometry(h->g, solid, nbr, h->widx, h->wn6, h->wdonor, h->nskip);
    const int nb = (int)h->widx.size();
    // device wall tables
    if (nb > h->wall_cap) {
        const int cap = nb + 64;
        h->F.wall_idx = (int32_t *)dev_alloc(h, cap * sizeof(int32_t));
        h->F.wall_q = (uint8_t *)dev_alloc(h, cap);
        h->F.wall_n = (float *)dev_alloc(h, 3 * (size_t)cap * sizeof(float));
        h->F.theta = (float *)dev_alloc(h, cap * sizeof(float));
        if (!h->F.wall_idx || !h->F.wall_q || !h->F.wall_n || !h->F.theta)
            return fail(h, CAC_ERR_ALLOC, "wall tables");
        h->wall_cap = cap;
    }
    std::vector<uint8_t> q(nb);
    std::vector<float> wn(3 * (size_t)nb), th(nb);
    for (int k = 0; k < nb; ++k) {
        q[k] = h->wdonor[k] < 0 ? 255 : (uint8_t)h->wdonor[k];
        const double a = h->wn6[3 * k], b = h->wn6[3 * k + 1], c = h->wn6[3 * k + 2];
        const double nn = std::sqrt(a * a + b * b + c * c);
        wn[3 * k] = nn > 0 ? (float)(a / nn) : 0.f;
        wn[3 * k + 1] = nn > 0 ? (float)(b / nn) : 0.f;
        wn[3 * k + 2] = nn > 0 ? (float)(c / nn) : 0.f;
        th[k] = theta_rad ? theta_rad[h->widx[k]] : (float)(M_PI / 2);
    }
    h->F.nwall = nb;
    HIPCHK(h, hipMemcpyAsync(h->F.nbr, nbr.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->F.solid, solid, N, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_tile_walls(h->g, h->t, h->F, h->stream));
    if (nb) {
        HIPCHK(h, hipMemcpyAsync(h->F.wall_idx, h->widx.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->F.wall_q, q.data(), nb, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->F.wall_n, wn.data(), 3 * nb * sizeof(float), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->F.theta, th.data(), nb * sizeof(float), hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));  // host vectors go out of scope
    h->geometry = true;
    h->state = false;
    h->geom_serial++;
    tape_invalidate(h);
    drop_graphs(h);
    if (h->nskip) fail(h, CAC_OK, "%d wall node(s) with a vanishing normal are skipped", h->nskip);
    return CAC_OK;
}

cac_status cac_num_wall_nodes(cac_handle *h, int *n_b)
{
    if (!h || !n_b) return CAC_ERR_ARG;
    if (!h->geometry) return fail(h, CAC_ERR_STATE, "no geometry");
    *n_b = (int)h->widx.size();
    return CAC_OK;
}

cac_status cac_wall_nodes(cac_handle *h, int32_t *linear_index, int32_t *normal6, int32_t *donor)
{
    if (!h) return CAC_ERR_ARG;
    if (!h->geometry) return fail(h, CAC_ERR_STATE, "no geometry");
    const size_t nb = h->widx.size();
    if (linear_index) std::copy(h->widx.begin(), h->widx.end(), linear_index);
    if (normal6) std::copy(h->wn6.begin(), h->wn6.end(), normal6);
    if (donor) std::copy(h->wdonor.begin(), h->wdonor.end(), donor);
    (void)nb;
    return CAC_OK;
}

cac_status cac_wall_tables(int nx, int ny, int nz, const uint8_t *solid, int *n_b, int32_t *linear_index,
                           int32_t *normal6, int32_t *donor, int cap)
{
    if (nx < 1 || ny < 1 || nz < 1 || !solid || !n_b) return CAC_ERR_ARG;
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    // population index i * N + n is an unsigned 32-bit integer in the kernels
    if (27ull * N > 0xFFFFFFFFull) return CAC_ERR_ARG;
    Grid g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.N = (uint32_t)N;
    g.nxny = (uint32_t)nx * (uint32_t)ny;
    std::vector<uint32_t> nbr;
    std::vector<int32_t> widx, wn6, wd;
    int nskip = 0;
    build_geometry(g, solid, nbr, widx, wn6, wd, nskip);
    const int nb = (int)widx.size();
    *n_b = nb;
    if (cap >= nb) {
        if (linear_index) std::copy(widx.begin(), widx.end(), linear_index);
        if (normal6) std::copy(wn6.begin(), wn6.end(), normal6);
        if (donor) std::copy(wd.begin(), wd.end(), donor);
    }
    return CAC_OK;
}

cac_status cac_set_contact_angles(cac_handle *h, const float *d_theta)
{
    if (!h || !d_theta) return CAC_ERR_ARG;
    if (!h->geometry) return fail(h, CAC_ERR_STATE, "no geometry");
    if (h->F.nwall)
        HIPCHK(h, hipMemcpyAsync(h->F.theta, d_theta, h->F.nwall * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return CAC_OK;
}

cac_status cac_set_state(cac_handle *h, const float *d_phi, const float *d_u, const float *d_pstar)
{
    if (!h) return CAC_ERR_ARG;
    if (!h->geometry) return fail(h, CAC_ERR_STATE, "cac_set_geometry must come first");
    if (!d_phi) return fail(h, CAC_ERR_ARG, "phi is NULL");
    const size_t N = h->g.N;
    Fields &F = h->F;
    HIPCHK(h, hipMemcpyAsync(F.phi[0], d_phi, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(F.phi[1], d_phi, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    if (d_u)
        HIPCHK(h, hipMemcpyAsync(F.u, d_u, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    else
        HIPCHK(h, hipMemsetAsync(F.u, 0, 3 * N * sizeof(float), h->stream));
    if (d_pstar)
        HIPCHK(h, hipMemcpyAsync(F.pstar0, d_pstar, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    else
        HIPCHK(h, hipMemsetAsync(F.pstar0, 0, N * sizeof(float), h->stream));
    HIPCHK(h, hipMemsetAsync(F.a, 0, 3 * N * sizeof(float), h->stream));
    HIPCHK(h, hipMemsetAsync(F.flag, 0, 256, h->stream));
    // the gradient-form path stores no populations: its first step reads p*0 and u0
    if (h->prm.collision == 0) HIPCHK(h, launch_init(h->g, F, 0, d_u, d_pstar, h->stream));
    HIPCHK(h, launch_mass(h->g, h->t, F, F.phi[0], F.scal + 0, h->stream));
    if (h->debug & CAC_DEBUG_POISON) HIPCHK(h, launch_poison(h->g, F, h->stream));
    h->cur = 0;
    h->steps = 0;
    h->sub = 0;
    h->state = true;
    tape_invalidate(h);
    return CAC_OK;
}

cac_status cac_step(cac_handle *h, int nsteps)
{
    if (!h) return CAC_ERR_ARG;
    if (nsteps < 0) return fail(h, CAC_ERR_ARG, "nsteps < 0");
    if (!h->state) return fail(h, CAC_ERR_STATE, "cac_set_state must come first");
    if (h->sub != 0) return fail(h, CAC_ERR_STATE, "a step was started with cac_debug_substep");
    for (int k = 0; k < nsteps; ++k) {
        // the first gradient-form step differs from the others: launched directly
        if (h->use_graph && !(h->prm.collision == 1 && h->steps == 0)) {
            const int par = h->cur;
            if (!h->gexec[par]) {
                cac_status st = capture_step(h, par);
                if (st != CAC_OK) return st;
            }
            HIPCHK(h, hipGraphLaunch(h->gexec[par], h->stream));
            h->cur ^= 1;
            h->steps++;
        } else {
            cac_status st = run_step(h);
            if (st != CAC_OK) return st;
        }
    }
    return CAC_OK;
}

cac_status cac_sync(cac_handle *h)
{
    if (!h) return CAC_ERR_ARG;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    uint32_t flag = 0;
    HIPCHK(h, hipMemcpy(&flag, h->F.flag, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) return fail(h, CAC_ERR_NONFINITE, "non-finite value detected in phi or u");
    return CAC_OK;
}

cac_status cac_volume(cac_handle *h, double *out)
{
    if (!h || !out) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    HIPCHK(h, launch_mass(h->g, h->t, h->F, h->F.phi[h->cur], h->F.scal + 4, h->stream));
    HIPCHK(h, hipMemcpyAsync(out, h->F.scal + 4, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    return cac_sync(h);
}

cac_status cac_get_fields(cac_handle *h, float *d_phi, float *d_u, float *d_pstar)
{
    if (!h) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    if (d_phi || d_pstar) {
        const bool r1 = h->prm.collision == 1;
        HIPCHK(h, launch_gather(h->g, h->F, r1 ? 1 : h->cur, h->cur, h->steps > 0, r1 ? 1 : 27, d_phi, d_pstar,
                                h->stream));
    }
    if (d_u)
        HIPCHK(h, hipMemcpyAsync(d_u, h->F.u, 3 * (size_t)h->g.N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return CAC_OK;
}

cac_status cac_get_populations(cac_handle *h, float *d_f)
{
    if (!h || !d_f) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    if (h->prm.collision != 0) return fail(h, CAC_ERR_STATE, "the gradient-form collision stores no populations");
    HIPCHK(h, hipMemcpyAsync(d_f, h->F.f[h->cur], 27 * (size_t)h->g.N * sizeof(float), hipMemcpyDeviceToDevice,
                             h->stream));
    return CAC_OK;
}

cac_status cac_set_launch(cac_handle *h, int bx, int by, int bz, int phase_tile, int use_graph)
{
    if (!h) return CAC_ERR_ARG;
    const int nt = bx * by * bz;
    if (!pow2(bx) || !pow2(by) || !pow2(bz) || bx < 16 || (nt != 128 && nt != 256 && nt != 512))
        return fail(h, CAC_ERR_ARG, "unsupported tile %dx%dx%d", bx, by, bz);
    if (phase_tile < 0 || phase_tile > 6) return fail(h, CAC_ERR_ARG, "unsupported phase tile %d", phase_tile);
    Tiling t = make_tiling(h->g, bx, by, bz);
    t.phase = phase_tile;
    t.hyd_lds = hydro_lds_reserve(h->dev, nt);
    if (t.ntiles > h->partial_cap) return fail(h, CAC_ERR_ARG, "too many tiles");
    h->t = t;
    if (h->geometry) HIPCHK(h, launch_tile_walls(h->g, h->t, h->F, h->stream));
    h->use_graph = use_graph != 0;
    drop_graphs(h);
    return CAC_OK;
}

cac_status cac_set_debug(cac_handle *h, int flags)
{
    if (!h) return CAC_ERR_ARG;
    if (flags & ~(CAC_DEBUG_POISON | CAC_DEBUG_REVERSE_ORDER)) return fail(h, CAC_ERR_ARG, "unknown debug flag");
    h->debug = flags;
    h->dp.rev_order = (flags & CAC_DEBUG_REVERSE_ORDER) ? 1 : 0;
    drop_graphs(h);  // captured steps carry the kernel arguments
    return CAC_OK;
}

cac_status cac_pull_copy_probe(cac_handle *h, int reps, double *ms)
{
    if (!h || !ms || reps < 1) return CAC_ERR_ARG;
    if (h->sub != 0) return fail(h, CAC_ERR_STATE, "a step was started with cac_debug_substep");
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    cac_status st = CAC_OK;
    if (launch_pull_copy(h->g, h->t, h->F.f[0], h->F.f[1], h->stream) != hipSuccess ||
        hipEventRecord(e0, h->stream) != hipSuccess)
        st = fail(h, CAC_ERR_HIP, "pull-copy launch");
    for (int k = 0; k < reps && st == CAC_OK; ++k)
        if (launch_pull_copy(h->g, h->t, h->F.f[(k + 1) & 1], h->F.f[k & 1], h->stream) != hipSuccess)
            st = fail(h, CAC_ERR_HIP, "pull-copy launch");
    float t = 0.f;
    if (st == CAC_OK && (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = fail(h, CAC_ERR_HIP, "pull-copy timing");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the populations are overwritten: a state must be set again before stepping
    h->state = false;
    tape_invalidate(h);
    if (st == CAC_OK) *ms = (double)t / reps;
    return st;
}

cac_status cac_profile_step(cac_handle *h, int nsteps, double *ms)
{
    if (!h || !ms || nsteps < 0) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    if (h->sub != 0) return fail(h, CAC_ERR_STATE, "a step was started with cac_debug_substep");
    std::vector<hipEvent_t> ev(5 * (size_t)nsteps);
    for (auto &e : ev) HIPCHK(h, hipEventCreate(&e));
    cac_status st = CAC_OK;
    for (int k = 0; k < nsteps && st == CAC_OK; ++k) {
        hipEvent_t *e = &ev[5 * (size_t)k];
        const int c = h->cur;
        HIPCHK(h, hipEventRecord(e[0], h->stream));
        HIPCHK(h, launch_ghost(h->g, h->dp, h->F, c, h->stream));
        HIPCHK(h, hipEventRecord(e[1], h->stream));
        HIPCHK(h, launch_h(h, c));
        HIPCHK(h, hipEventRecord(e[2], h->stream));
        HIPCHK(h, launch_phase(h->g, h->t, h->dp, h->F, c, h->stream));
        HIPCHK(h, hipEventRecord(e[3], h->stream));
        HIPCHK(h, launch_volume(h->g, h->t, h->dp, h->F, c ^ 1, h->stream));
        HIPCHK(h, hipEventRecord(e[4], h->stream));
        h->cur ^= 1;
        h->steps++;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < nsteps; ++k)
        for (int j = 0; j < 4; ++j) {
            float t = 0.f;
            HIPCHK(h, hipEventElapsedTime(&t, ev[5 * (size_t)k + j], ev[5 * (size_t)k + j + 1]));
            ms[j] += t;
        }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return st;
}

// ------------------------------------------------------------------ state save / load
namespace {
constexpr uint64_t kStateMagic = 0x31455441545343ull;  // "CSTATE1"
constexpr size_t kStateHeader = 64;
size_t state_bytes(const cac_handle *h) { return kStateHeader + 33ull * h->g.N * sizeof(float); }
}  // namespace

cac_status cac_state_bytes(cac_handle *h, size_t *bytes)
{
    if (!h || !bytes) return CAC_ERR_ARG;
    *bytes = state_bytes(h);
    return CAC_OK;
}

cac_status cac_save_state(cac_handle *h, void *d_buf, size_t bytes)
{
    if (!h || !d_buf) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    if (h->sub != 0) return fail(h, CAC_ERR_STATE, "a step was started with cac_debug_substep");
    if (bytes < state_bytes(h)) return fail(h, CAC_ERR_ARG, "buffer of %zu bytes, %zu needed", bytes, state_bytes(h));
    const size_t N = h->g.N;
    const int c = h->cur;
    char *b = (char *)d_buf;
    // header: magic, N, step count, target volume (filled from the device below),
    // collision setting, zeros to 64 bytes
    uint64_t hdr[kStateHeader / 8] = {kStateMagic, (uint64_t)N, (uint64_t)h->steps, 0u, (uint64_t)h->prm.collision};
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(b, hdr, sizeof hdr, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpyAsync(b + 24, h->F.scal, sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    float *a = (float *)(b + kStateHeader);
    // the 27 population planes, or the record planes of the gradient-form path
    const float *fsrc = h->prm.collision == 1 ? h->F.f[1] : h->F.f[c];
    HIPCHK(h, hipMemcpyAsync(a, fsrc, 27 * N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(a + 27 * N, h->F.phi[c], N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(a + 28 * N, h->F.phi[c ^ 1], N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(a + 29 * N, h->F.u, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(a + 32 * N, h->F.pstar0, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return CAC_OK;
}

cac_status cac_load_state(cac_handle *h, const void *d_buf, size_t bytes)
{
    if (!h || !d_buf) return CAC_ERR_ARG;
    if (!h->geometry) return fail(h, CAC_ERR_STATE, "cac_set_geometry must come first");
    if (bytes < state_bytes(h)) return fail(h, CAC_ERR_ARG, "buffer of %zu bytes, %zu needed", bytes, state_bytes(h));
    const size_t N = h->g.N;
    const char *b = (const char *)d_buf;
    uint64_t hdr[3], coll = 0;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(hdr, b, sizeof hdr, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(&coll, b + 32, sizeof coll, hipMemcpyDeviceToHost));
    if (hdr[0] != kStateMagic || hdr[1] != (uint64_t)N)
        return fail(h, CAC_ERR_ARG, "not a saved state of a lattice of this size");
    if (coll != (uint64_t)h->prm.collision)
        return fail(h, CAC_ERR_ARG, "state saved with collision = %llu, handle has %d", (unsigned long long)coll,
                    h->prm.collision);
    const float *a = (const float *)(b + kStateHeader);
    HIPCHK(h, hipMemcpyAsync(h->F.scal, b + 24, sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->F.f[h->prm.collision == 1 ? 1 : 0], a, 27 * N * sizeof(float),
                             hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->F.phi[0], a + 27 * N, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->F.phi[1], a + 28 * N, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->F.u, a + 29 * N, 3 * N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->F.pstar0, a + 32 * N, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    // the compressive flux is rebuilt by every ghost update; skipped wall nodes keep zero
    HIPCHK(h, hipMemsetAsync(h->F.a, 0, 3 * N * sizeof(float), h->stream));
    if (h->debug & CAC_DEBUG_POISON) HIPCHK(h, launch_poison(h->g, h->F, h->stream));
    HIPCHK(h, hipMemsetAsync(h->F.flag, 0, 256, h->stream));
    h->cur = 0;
    h->steps = (long long)hdr[2];
    h->sub = 0;
    h->state = true;
    tape_invalidate(h);
    return CAC_OK;
}

// ------------------------------------------------------------------ debug hooks
cac_status cac_debug_substep(cac_handle *h, int which)
{
    if (!h) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    if (which != h->sub) return fail(h, CAC_ERR_STATE, "substep %d expected next, %d requested", h->sub, which);
    const int c = h->cur;
    switch (which) {
    case 0: HIPCHK(h, launch_ghost(h->g, h->dp, h->F, c, h->stream)); break;
    case 1: HIPCHK(h, launch_h(h, c)); break;
    case 2: HIPCHK(h, launch_phase(h->g, h->t, h->dp, h->F, c, h->stream)); break;
    case 3:
        HIPCHK(h, launch_volume(h->g, h->t, h->dp, h->F, c ^ 1, h->stream));
        h->cur ^= 1;
        h->steps++;
        break;
    default: return fail(h, CAC_ERR_ARG, "substep %d", which);
    }
    h->sub = (which + 1) % 4;
    return CAC_OK;
}

cac_status cac_debug_buffer(cac_handle *h, int which, float *d_out)
{
    if (!h || !d_out) return CAC_ERR_ARG;
    if (!h->state) return fail(h, CAC_ERR_STATE, "no state");
    const size_t N = h->g.N;
    const int c = h->cur;
    const float *src = nullptr;
    size_t n = N;
    switch (which) {
    case 0: src = h->F.phi[c]; break;
    case 1: src = h->F.phi[c ^ 1]; break;
    case 2: src = h->F.u; n = 3 * N; break;
    // collision = 1: the rebuilt populations and the record planes, whatever the parity
    case 3: src = h->F.f[h->prm.collision == 1 ? 0 : c]; n = 27 * N; break;
    case 4: src = h->F.f[h->prm.collision == 1 ? 1 : c ^ 1]; n = 27 * N; break;
    case 5: src = h->F.a; n = 3 * N; break;
    default: return fail(h, CAC_ERR_ARG, "buffer %d", which);
    }
    HIPCHK(h, hipMemcpyAsync(d_out, src, n * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return CAC_OK;
}

cac_status cac_destroy(cac_handle *h)
{
    if (!h) return CAC_ERR_ARG;
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    tape_free(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void *q : h->owned) (void)hipFree(q);
    delete h;
    return CAC_OK;
}

}  // extern "C"
