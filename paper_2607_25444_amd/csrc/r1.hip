// r1.hip -- the hydrodynamic substep with the gradient-form non-equilibrium
// moment (collision = 1): the thread-safe formulation of Sec. II A, in which
// both parts of the populations are rebuilt from macroscopic quantities.
//
// No populations are kept from one step to the next.  The state of a node is
// its record (p*, u, a, omega) of the last collision.  A step takes two
// kernels:
//   k_r1_rebuild A2 = -(c_s^2/omega)(grad u + grad u^T) (Eq. (15)) from the
//                isotropic stencil (Eq. (22)) of the stored velocity field
//                (a solid neighbour holds the node's mirror image -u; the
//                planes staged through LDS in column tiles), then the node's
//                post-collision populations (Eqs. (3), (11), (14), (16),
//                (17)), written once;
//   k_r1_stream  pull f_i(x) = f*_i(x - c_i) (halfway bounce-back: f*_opp(i)
//                of x itself), the kinetic moments, forces and velocity of
//                the collision at x (Eqs. (6)-(10), (18)-(21)); writes the
//                new record.  On the first step after the state is set, the
//                pulled populations are the node's own equilibrium
//                f^eq(p*0, u0) (the initial condition of the local-moment
//                path).
// Rebuilding each population at the pulling node instead (from the 17
// Hermite coefficients of its source, 68 bytes per node) needs 314 gathers
// per node against 27 here; on gfx950 that substep took 1.49 ms against
// 0.49 ms here on 256 x 256 x 128.
//
// Layout (structure of arrays, node index n):
//   rebuilt populations P[i*N + n] (27 planes) in the first population buffer;
//   record planes R[k*N + n], k = 0..4: p*, a (3), omega, in the second; u in
//   its own array.
#include "r1_device.hpp"

namespace cac {

// One workgroup per column tile (r1_rebuild_tile), tiles in XCD-contiguous order.
template <int CX, int CY>
__global__ __launch_bounds__(CX *CY) void k_r1_rebuild(Grid g, PhaseTiling pt, DevParams p, const float *__restrict__ rec,
                                                    const float *__restrict__ u, const uint32_t *__restrict__ nbr,
                                                    float *__restrict__ fout)
{
    const uint32_t b = p.rev_order ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
    r1_rebuild_tile<CX, CY>(g, pt, xcd_tile(b, pt.ntiles), rec, u, nbr, fout);
}

// Workgroup order as in the local-moment kernel: the hardware's (on 64x8
// tiles of the 192-wide orifice lattice 3% faster than XCD-contiguous tiles).
template <int NT, bool SELF, bool NTL>
__global__ __launch_bounds__(NT) void k_r1_stream(Grid g, Tiling t, DevParams p, const float *__restrict__ fin,
                                                  const float *__restrict__ phi, const uint32_t *__restrict__ nbr,
                                                  const uint8_t *__restrict__ twall, const float *__restrict__ pstar0,
                                                  float *__restrict__ u, float *__restrict__ rec,
                                                  uint32_t *__restrict__ flag)
{
    const uint32_t tile = p.rev_order ? gridDim.x - 1u - blockIdx.x : blockIdx.x;
    r1_stream_node<SELF, NTL>(g, p, tile_node(g, t, tile), fin, phi, nbr, pstar0, u, rec, flag, twall[tile] != 0);
}

// The rebuilt populations live in the first population buffer, the record in
// the second.
hipError_t launch_r1_rebuild(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, hipStream_t s)
{
    (void)t;
    const PhaseTiling pt = phase_tiling(g, 64, 8);
    k_r1_rebuild<64, 8><<<pt.ntiles, 512, 0, s>>>(g, pt, p, F.f[1], F.u, F.nbr, F.f[0]);
    return hipGetLastError();
}

hipError_t launch_r1_stream(const Grid &g, const Tiling &t, const DevParams &p, const Fields &F, int pcur, bool self,
                            hipStream_t s)
{
    const bool ntl = t.bx >= g.nx;
#define CAC_R1S(NT_)                                                                                              \
    if (self)                                                                                                     \
        k_r1_stream<NT_, true, false><<<t.ntiles, NT_, t.hyd_lds, s>>>(g, t, p, F.f[0], F.phi[pcur], F.nbr, F.twall, F.pstar0,     \
                                                               F.u, F.f[1], F.flag);                              \
    else if (ntl)                                                                                                 \
        k_r1_stream<NT_, false, true><<<t.ntiles, NT_, t.hyd_lds, s>>>(g, t, p, F.f[0], F.phi[pcur], F.nbr, F.twall, F.pstar0,     \
                                                               F.u, F.f[1], F.flag);                              \
    else                                                                                                          \
        k_r1_stream<NT_, false, false><<<t.ntiles, NT_, t.hyd_lds, s>>>(g, t, p, F.f[0], F.phi[pcur], F.nbr, F.twall, F.pstar0,    \
                                                                F.u, F.f[1], F.flag);
    switch (t.bx * t.by * t.bz) {
    case 128: CAC_R1S(128) break;
    case 256: CAC_R1S(256) break;
    case 512: CAC_R1S(512) break;
    default: return hipErrorInvalidValue;
    }
#undef CAC_R1S
    return hipGetLastError();
}

}  // namespace cac
