// cac_internal.hpp -- declarations shared by the HIP kernels and the host
// runtime of libcac (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace cac {

// ---------------------------------------------------------------- D3Q27 set
// Canonical order: 0 rest; 1..6 axis pairs; 7..18 face-diagonal pairs;
// 19..26 body-diagonal pairs; the opposite of odd i is i + 1.
struct Lat {
    static constexpr int Q = 27;
    static constexpr int cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
    __host__ __device__ static constexpr int norm2(int i) { return cx[i] * cx[i] + cy[i] * cy[i] + cz[i] * cz[i]; }
    __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
    // lattice weight as a rational: w = 8/27, 2/27, 1/54, 1/216 by |c|^2
    __host__ __device__ static constexpr float w(int i)
    {
        return norm2(i) == 0 ? 8.0f / 27.0f : norm2(i) == 1 ? 2.0f / 27.0f : norm2(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f;
    }
    // link index of the offset (dx, dy, dz) in {-1,0,1}^3
    __host__ __device__ static constexpr int idx(int dx, int dy, int dz)
    {
        for (int i = 0; i < 27; ++i)
            if (cx[i] == dx && cy[i] == dy && cz[i] == dz) return i;
        return -1;
    }
};

// compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1
template <class F, int... Is>
__host__ __device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------- parameters
// Single-precision coefficients derived once on the host from cac_params.
struct DevParams {
    float rho_g, drho;       // rho = rho_g + drho * phi
    float mu_g, dmu;         // dynamic viscosity mu = mu_g + dmu * phi
    float beta4, kappa_phi;  // 4 beta and kappa_phi of the chemical potential
    float D, kappa;          // CAC diffusivity and compression (kappa = 4 D / delta)
    float gx, gy, gz;        // body acceleration
    float eps_phi, eps_n2;   // interface band, squared normal guard
    float sin_tol, cot_max;
    int volume_correction;
    int wall_compression;
    int ghost_lambda;        // 1: lambda_s of Eq. (47) in the ghost extrapolation; 0: lambda_s = 1
    int variable_density;    // drho != 0: pressure and viscous corrections are live
    int rev_order;           // debug: W, H and P take their workgroups in reverse order
};

struct Grid {
    int nx, ny, nz;
    uint32_t N, nxny;
};

// Tiling of the bulk kernels: workgroup = one tile of bx*by*bz nodes.
struct Tiling {
    int bx, by, bz;
    int tx, ty, tz;   // tiles per axis
    uint32_t ntiles;  // tx*ty*tz
    int phase;        // column tile code of the phase kernel (0 = automatic)
    uint32_t hyd_lds; // LDS bytes each collide-stream workgroup reserves (unused) to hold it at 4 waves per SIMD
};

// Column tiling of the phase kernel: ntx x nty column tiles, z-chunks of zc planes.
struct PhaseTiling {
    int ntx, nty, nzc, zc;
    uint32_t ntiles;
};

// Device buffers of one lattice (plain handle or one batched domain).
struct Fields {
    float *f[2];        // post-collision populations, 27 planes each
    float *phi[2];      // phase field A/B buffers (fluid values + ghosts)
    float *u;           // 3 planes
    float *a;           // compressive flux on wall nodes (3 planes, written by W; zero elsewhere)
    uint32_t *nbr;      // bit 0: node solid; bit i: node + c_i solid
    uint8_t *solid;     // 1 = solid
    int32_t *wall_idx;  // wall-node list (ascending node index)
    uint8_t *wall_q;    // donor link (255: skipped)
    float *wall_n;      // unit wall normal, 3 per node
    float *theta;       // contact angle per wall node
    double2 *partial;   // per-tile (sum phi*, sum chi)
    double *scal;       // [0] M_target, [1] lambda, [2] M*, [3] W
    uint32_t *flag;     // watchdog: nonzero after a non-finite value
    uint8_t *chunk;     // per 1024 nodes: set by P where it wrote an interface node, cleared by V
    uint8_t *twall;     // per hydrodynamic tile: 1 when a node of the tile is solid or next to a solid node
    float *pstar0;      // p* of the initial state (reported before the first step)
    int nwall;
};

// ---------------------------------------------------------------- batches
// Device descriptor of one domain of a batch.  All domains live in shared
// concatenated arrays; domain k's fields start at node offset `off` (its
// populations at 27*off, vectors at 3*off) and keep the single-lattice layout.
struct BatchDomain {
    Grid g;
    Tiling t;         // hydrodynamic tiling
    PhaseTiling pt;   // phase tiling
    DevParams p;
    uint32_t off;     // node offset
    uint32_t p_item0; // first FP64 partial of this domain's phase tiles
};

struct BatchPtrs {
    float *f[2], *phi[2], *u, *a;
    uint32_t *nbr;
    uint8_t *solid;
    int32_t *wall_idx;   // domain-local node index of each wall node
    uint8_t *wall_q;
    float *wall_n, *theta;
    uint16_t *wall_dom;  // domain of each wall node
    double2 *partial;    // per phase tile, at BatchDomain::p_item0 + tile
    double *scal;        // 8 per domain: [0] M_target, [1] lambda, [2] M*, [3] W, [4] volume
    uint32_t *flag;
    uint8_t *chunk;      // per 1024 nodes of the concatenated arrays: set by P at interface nodes, cleared by V
    const BatchDomain *dom;
    const uint32_t *dom_start;  // ndom + 1 node offsets: domain k holds nodes [dom_start[k], dom_start[k + 1])
    const uint16_t *blk_dom;    // domain of the first node of each 256-node block of the concatenated arrays
    uint32_t ntot;              // total nodes
    int ndom;
};

// Work items of the persistent batched kernels: (domain, tile) pairs in the
// order of the block schedule.  grid = number of persistent workgroups.
hipError_t launch_bghost(const BatchPtrs &B, uint32_t nwall, int cur, hipStream_t s);
hipError_t launch_bitem_walls(const BatchPtrs &B, int nt, uint2 *items, uint32_t nitems, hipStream_t s);
hipError_t launch_bhydro(const BatchPtrs &B, int nt, const uint2 *items, uint32_t nitems, uint32_t grid, uint32_t lds, int cur,
                         hipStream_t s);
hipError_t launch_bphase(const BatchPtrs &B, int phase_code, const uint2 *items, uint32_t nitems, uint32_t grid,
                         int cur, hipStream_t s);
hipError_t launch_bvolume(const BatchPtrs &B, int nt, const uint2 *items, uint32_t nitems, uint32_t grid, int cur_next,
                          hipStream_t s);
// resident workgroups per CU of a batched kernel (kind 0 hydro / 1 phase), 0 on failure
int batch_blocks_per_cu(int kind, int code, uint32_t lds = 0);
// LDS bytes a collide-stream workgroup of nt threads reserves (see Tiling::hyd_lds)
uint32_t hydro_lds_reserve(int dev, int nt);
void phase_shape_of(int code, int &bx, int &by);  // code 1..6
PhaseTiling phase_tiling(const Grid &g, int bx, int by);

// ---------------------------------------------------------------- launchers
// All enqueue on `s`; return the launch status.
hipError_t launch_ghost(const Grid &g, const DevParams &p, const Fields &F, int cur, hipStream_t s);
hipError_t launch_hydro(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, int fcur, int pcur,
                        hipStream_t s);
// Gradient-form hydrodynamic substep (collision = 1): coefficients of the
// post-collision populations from the record in F.f[1] and the velocity
// field into F.f[0]; then pull, moments and collision into the record and u
// (self = the first step after the state is set: each node pulls its own
// equilibrium).
hipError_t launch_r1_rebuild(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, hipStream_t s);
hipError_t launch_r1_stream(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, int pcur, bool self,
                            hipStream_t s);
hipError_t launch_phase(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, int pcur,
                        hipStream_t s);
uint32_t phase_tiles(const Grid &g, const Tiling &t);  // workgroups (and FP64 partials) of the phase kernel
uint32_t phase_tiles_max(const Grid &g);                // over every phase tile shape
hipError_t launch_tile_walls(const Grid &g, const Tiling &t, const Fields &F, hipStream_t s);
hipError_t launch_volume(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, int pnext,
                         hipStream_t s);
hipError_t launch_poison(const Grid &g, const Fields &F, hipStream_t s);  // debug (k_poison)
hipError_t launch_init(const Grid &g, const Fields &F, int fcur, const float *u0, const float *ps0,
                       hipStream_t s);
hipError_t launch_mass(const Grid &g, const Tiling &t, const Fields &F, const float *phi, double *out,
                       hipStream_t s);
// The same FP64 fluid sum of phi with the block partials in `partial`
// (mass_partials(N) entries, all written before they are read); out: device.
uint32_t mass_partials(uint32_t N);
hipError_t launch_mass_into(uint32_t N, const uint8_t *solid, const float *phi, double2 *partial, double *out,
                            hipStream_t s);
// p* on fluid nodes after a step: the sum of the first `npl` planes of
// F.f[fcur] (27: the post-collision populations; 1: the record of the
// gradient-form path).
hipError_t launch_gather(const Grid &g, const Fields &F, int fcur, int pcur, int stepped, int npl, float *phi_out,
                         float *pstar_out, hipStream_t s);

// ---------------------------------------------------------------- adjoint
// One reverse step (the transpose of the Jacobian of W -> H -> P -> V at the
// recorded forward state).  Cotangents of the populations are kept as the
// cotangents of the ten moments the collision reads (p*, j, P = sum f c c):
// the collision depends on f only through them, so the cotangent of the
// pulled population f_i(x) is  mb0 + c_i.(mb1..3) + c_i c_i : (mb4..9).
struct AdjStep {
    // recorded forward state of the step
    const float *fprev;    // post-collision populations entering the step (pull layout)
    const float *phihat;   // phi^n on fluid nodes with this step's ghosts on wall nodes
    const float *phiold;   // previous ghosts (read on wall nodes)
    const float *u;        // velocity of the step (zero on solid nodes)
    const float *phistar;  // phase field before the volume correction (fluid nodes)
    // cotangents
    const float *pb_in;    // of phi^{n+1} (all nodes)
    const float *mb_in;    // of the moments of step n+1: N float4 (p*, j), N float4 (P_xx, P_yy, P_zz, P_xy),
                           // N float2 (P_xz, P_yz)
    float *psi;            // of phi* on fluid nodes (0 on solid nodes)
    float *pb_out;         // of phi-hat, then (after the wall pass) of phi^n
    float *mb_out;         // of the moments of step n (layout of mb_in)
    float *rec;            // N float4 (cotangents of grad x, y, z and of the Laplacian), then N floats (local)
    float *awb;            // 3 planes: of the compressive flux on wall nodes
    // geometry
    const uint32_t *nbr;
    const uint8_t *solid;
    const int32_t *widx;
    const uint8_t *wq;
    const float *wn, *theta;
    const int32_t *don_start, *don_wall, *don_node;  // donors with their wall nodes (CSR)
    int ndon;
    const int32_t *don_map;  // node -> donor slot or -1
    float4 *dg;              // per donor: (cotangent of phi_f, of grad phi at the donor)
    const uint32_t *near;    // nodes within one link of a donor; bit 31: active wall node
    uint32_t nnear;
    double *thb;             // dL/dtheta per wall node (accumulated)
    double *red;             // reduction partials
    double *rs;              // [0] lambda, [1] cotangent mean of the correction, [3] dL/dM_target, [4] loss
    const double *scal;      // forward scalars ([0] M_target)
};

hipError_t launch_volume_copy(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F,
                              const float *phistar, const float *phihat, float *out, hipStream_t s);
uint32_t adj_red_blocks(const Grid &g);  // partial entries (3 doubles each) of the reductions
// reduction of the correction's transpose (lambda, cbar into S.rs) and the psi field
hipError_t launch_adj_vsum(const Grid &g, const DevParams &p, const AdjStep &S, hipStream_t s);
hipError_t launch_adj_main(const Grid &g, const Tiling &t, const DevParams &p, const AdjStep &S, hipStream_t s);
hipError_t launch_adj_assemble(const Grid &g, const Tiling &t, const AdjStep &S, hipStream_t s);
hipError_t launch_adj_wall(const Grid &g, const DevParams &p, const AdjStep &S, hipStream_t s);
hipError_t launch_adj_fix(const Grid &g, const AdjStep &S, hipStream_t s);
// dst = src on the fluid nodes of `planes` planes of N floats (solid entries untouched)
hipError_t launch_copy_fluid(const Grid &g, const uint8_t *solid, int planes, const float *src, float *dst,
                             hipStream_t s);
// pb += rs[3] on fluid nodes (the path of dL/dphi0 through the target volume)
hipError_t launch_adj_mtarget(const Grid &g, const uint8_t *solid, float *pb, const double *rs, hipStream_t s);
// seed = phi - target on fluid nodes (0 elsewhere) and out[0] = 1/2 sum_fluid (phi - target)^2 in FP64
hipError_t launch_loss_seed(const Grid &g, const uint8_t *solid, const float *phi, const float *target, float *seed,
                            double *red, double *out, hipStream_t s);

}  // namespace cac
