// adjoint.hip -- gfx950 kernels of the reverse (adjoint) step.
//
// One reverse step at the recorded forward state of step n:
//   k_adj_vsum / k_adj_vfin  FP64 sums sum(pb chi), sum(phi*), sum(chi) of the
//                            volume correction's transpose -> lambda, cbar
//   k_adj_main               per node: transposes of V, P and the collision;
//                            the transpose of the pull streaming is a gather
//                            of the neighbours' moment cotangents
//   k_adj_assemble           transpose of the gradient / Laplacian stencils
//   k_adj_wall               transpose of the ghost update per donor node,
//                            dL/dtheta accumulated in FP64 per wall node
//   k_adj_fix                donor-stencil transpose on the nodes next to donors
// plus the loss / seed kernel of L = 1/2 sum_fluid (phi - phi_T)^2.
// Node bodies live in adjoint_device.hpp; all kernels are deterministic
// (no atomics, fixed reduction order).
#include "adjoint_device.hpp"

namespace cac {

template <int NT>
__device__ __forceinline__ void block_sum3(double &x, double &y, double &z)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
        z += __shfl_xor(z, off, 64);
    }
    __shared__ double sx[NT / 64], sy[NT / 64], sz[NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sx[wid] = x;
        sy[wid] = y;
        sz[wid] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) {
            tx += sx[k];
            ty += sy[k];
            tz += sz[k];
        }
        x = tx;
        y = ty;
        z = tz;
    }
}

static inline unsigned nblocks(uint32_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// Per-block sums over fluid nodes of pb chi(phi*), phi*, chi(phi*) (Eqs. (49), (51)).
__global__ __launch_bounds__(256) void k_adj_vsum(uint32_t N, const uint8_t *__restrict__ solid,
                                                  const float *__restrict__ pb, const float *__restrict__ phistar,
                                                  float eps, double *__restrict__ red)
{
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    if (n < N && !solid[n]) {
        const float v = phistar[n];
        b = (double)v;
        if (v > eps && v < 1.0f - eps) {
            c = (double)v * (1.0 - (double)v);
            a = (double)pb[n] * c;
        }
    }
    block_sum3<256>(a, b, c);
    if (threadIdx.x == 0) {
        red[3 * blockIdx.x] = a;
        red[3 * blockIdx.x + 1] = b;
        red[3 * blockIdx.x + 2] = c;
    }
}

// lambda = (M_target - sum phi*) / W and cbar = sum(pb chi) / W, zero when W = 0
// or the correction is off.
__global__ __launch_bounds__(1024) void k_adj_vfin(const double *__restrict__ red, uint32_t np,
                                                   const double *__restrict__ scal, double *__restrict__ rs, int vc)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (uint32_t k = threadIdx.x; k < np; k += 1024) {
        a += red[3 * k];
        b += red[3 * k + 1];
        c += red[3 * k + 2];
    }
    block_sum3<1024>(a, b, c);
    if (threadIdx.x == 0) {
        const bool on = vc && c > 0.0;
        rs[0] = on ? (scal[0] - b) / c : 0.0;
        rs[1] = on ? a / c : 0.0;
        rs[3] += rs[1];  // dL/dM_target summed over the steps (lambda grows by 1/W per unit of M)
    }
}

// Add the target-volume path to dL/dphi0: M_target is the fluid sum of phi0.
__global__ __launch_bounds__(256) void k_add_fluid(uint32_t N, const uint8_t *__restrict__ solid,
                                                   float *__restrict__ pb, const double *__restrict__ rs)
{
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    if (n < N && !solid[n]) pb[n] += (float)rs[3];
}

template <int NT>
__global__ __launch_bounds__(NT) void k_adj_main(Grid g, Tiling t, DevParams p, AdjStep S)
{
    const Node nd = tile_node(g, t, xcd_tile(blockIdx.x, t.ntiles));
    if (nd.in) adj_main_node(g, p, S, nd.x, nd.y, nd.z);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_adj_assemble(Grid g, Tiling t, AdjStep S)
{
    const Node nd = tile_node(g, t, xcd_tile(blockIdx.x, t.ntiles));
    if (nd.in) adj_assemble_node(g, S, nd.x, nd.y, nd.z);
}

__global__ __launch_bounds__(256) void k_adj_wall(Grid g, DevParams p, AdjStep S)
{
    const int d = (int)(blockIdx.x * 256u + threadIdx.x);
    if (d < S.ndon) adj_wall_donor(g, p, S, d);
}

__global__ __launch_bounds__(256) void k_adj_fix(Grid g, AdjStep S)
{
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e < S.nnear) adj_fix_node(g, S, e);
}

// seed = phi - phi_T on fluid nodes (0 on solid), per-block sums of 1/2 (phi - phi_T)^2.
__global__ __launch_bounds__(256) void k_loss_seed(uint32_t N, const uint8_t *__restrict__ solid,
                                                   const float *__restrict__ phi, const float *__restrict__ target,
                                                   float *__restrict__ seed, double *__restrict__ red)
{
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    if (n < N) {
        float d = 0.f;
        if (!solid[n]) {
            d = phi[n] - target[n];
            a = 0.5 * (double)d * (double)d;
        }
        seed[n] = d;
    }
    block_sum3<256>(a, b, c);
    if (threadIdx.x == 0) {
        red[3 * blockIdx.x] = a;
        red[3 * blockIdx.x + 1] = b;
        red[3 * blockIdx.x + 2] = c;
    }
}

__global__ __launch_bounds__(1024) void k_loss_fin(const double *__restrict__ red, uint32_t np, double *__restrict__ out)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (uint32_t k = threadIdx.x; k < np; k += 1024) a += red[3 * k];
    block_sum3<1024>(a, b, c);
    if (threadIdx.x == 0) out[0] = a;
}

// ------------------------------------------------------------------ launchers

uint32_t adj_red_blocks(const Grid &g) { return nblocks(g.N, 256); }

hipError_t launch_adj_vsum(const Grid &g, const DevParams &p, const AdjStep &S, hipStream_t s)
{
    const unsigned nb = nblocks(g.N, 256);
    k_adj_vsum<<<nb, 256, 0, s>>>(g.N, S.solid, S.pb_in, S.phistar, p.eps_phi, S.red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_adj_vfin<<<1, 1024, 0, s>>>(S.red, nb, S.scal, S.rs, p.volume_correction);
    return hipGetLastError();
}

hipError_t launch_adj_main(const Grid &g, const Tiling &t, const DevParams &p, const AdjStep &S, hipStream_t s)
{
    switch (t.bx * t.by * t.bz) {
    case 128: k_adj_main<128><<<t.ntiles, 128, 0, s>>>(g, t, p, S); break;
    case 256: k_adj_main<256><<<t.ntiles, 256, 0, s>>>(g, t, p, S); break;
    case 512: k_adj_main<512><<<t.ntiles, 512, 0, s>>>(g, t, p, S); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adj_assemble(const Grid &g, const Tiling &t, const AdjStep &S, hipStream_t s)
{
    switch (t.bx * t.by * t.bz) {
    case 128: k_adj_assemble<128><<<t.ntiles, 128, 0, s>>>(g, t, S); break;
    case 256: k_adj_assemble<256><<<t.ntiles, 256, 0, s>>>(g, t, S); break;
    case 512: k_adj_assemble<512><<<t.ntiles, 512, 0, s>>>(g, t, S); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adj_wall(const Grid &g, const DevParams &p, const AdjStep &S, hipStream_t s)
{
    if (S.ndon <= 0) return hipSuccess;
    k_adj_wall<<<nblocks((uint32_t)S.ndon, 256), 256, 0, s>>>(g, p, S);
    return hipGetLastError();
}

hipError_t launch_adj_fix(const Grid &g, const AdjStep &S, hipStream_t s)
{
    if (S.nnear == 0) return hipSuccess;
    k_adj_fix<<<nblocks(S.nnear, 256), 256, 0, s>>>(g, S);
    return hipGetLastError();
}

hipError_t launch_adj_mtarget(const Grid &g, const uint8_t *solid, float *pb, const double *rs, hipStream_t s)
{
    k_add_fluid<<<nblocks(g.N, 256), 256, 0, s>>>(g.N, solid, pb, rs);
    return hipGetLastError();
}

hipError_t launch_loss_seed(const Grid &g, const uint8_t *solid, const float *phi, const float *target, float *seed,
                            double *red, double *out, hipStream_t s)
{
    const unsigned nb = nblocks(g.N, 256);
    k_loss_seed<<<nb, 256, 0, s>>>(g.N, solid, phi, target, seed, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_loss_fin<<<1, 1024, 0, s>>>(red, nb, out);
    return hipGetLastError();
}

}  // namespace cac
