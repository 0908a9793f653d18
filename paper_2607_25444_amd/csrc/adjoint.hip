// adjoint.hip -- gfx950 kernels of the reverse (adjoint) step.
//
// One reverse step at the recorded forward state of step n:
//   k_adj_vsum               FP64 sums sum(pb chi), sum(phi*), sum(chi) of the
//                            volume correction's transpose
//   k_adj_psi                lambda, cbar from those sums; psi = cotangent of
//                            phi* (fluid nodes)
//   k_adj_main               per node: transposes of V, P and the collision;
//                            the transpose of the pull streaming is a gather
//                            of the neighbours' moment cotangents
//   k_adj_assemble_lds       transpose of the gradient / Laplacian stencils (2.5-D LDS)
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

// Per-block FP64 sums over fluid nodes of pb chi(phi*), phi*, chi(phi*)
// (Eqs. (49), (51)); each thread covers ADJ_VSUM_PER_THREAD nodes.
constexpr uint32_t ADJ_VSUM_PER_THREAD = 8;

__global__ __launch_bounds__(256) void k_adj_vsum(uint32_t N, const uint8_t *__restrict__ solid,
                                                  const float *__restrict__ pb, const float *__restrict__ phistar,
                                                  float eps, double *__restrict__ red)
{
    // all loads first, at in-range indices (a node past N reads node 0 and is
    // then skipped), so that they are in flight together
    uint8_t so[ADJ_VSUM_PER_THREAD];
    float v[ADJ_VSUM_PER_THREAD], q[ADJ_VSUM_PER_THREAD];
#pragma unroll
    for (uint32_t r = 0; r < ADJ_VSUM_PER_THREAD; ++r) {
        const uint32_t n = (blockIdx.x * ADJ_VSUM_PER_THREAD + r) * 256u + threadIdx.x;
        const uint32_t m = n < N ? n : 0u;
        so[r] = n < N ? solid[m] : (uint8_t)1;
        v[r] = phistar[m];
        q[r] = pb[m];
    }
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (uint32_t r = 0; r < ADJ_VSUM_PER_THREAD; ++r) {
        if (!so[r]) {
            b += (double)v[r];
            if (v[r] > eps && v[r] < 1.0f - eps) {
                const double ch = (double)v[r] * (1.0 - (double)v[r]);
                c += ch;
                a += (double)q[r] * ch;
            }
        }
    }
    block_sum3<256>(a, b, c);
    if (threadIdx.x == 0) {
        red[3 * blockIdx.x] = a;
        red[3 * blockIdx.x + 1] = b;
        red[3 * blockIdx.x + 2] = c;
    }
}

// psi, the cotangent of phi* on fluid nodes (0 on solid nodes), with
// lambda = (M_target - sum phi*) / W and cbar = sum(pb chi) / W (zero when
// W = 0 or the correction is off).  Every workgroup sums the np partials of
// k_adj_vsum itself, in the same fixed order, so that no separate launch has
// to finish the sums first; workgroup 0 records lambda and cbar and adds cbar
// to dL/dM_target (summed over the steps: lambda grows by 1/W per unit of M).
// ADJ_VSUM_PER_THREAD nodes per thread, in k_adj_vsum's order.
__global__ __launch_bounds__(256) void k_adj_psi(uint32_t N, DevParams p, AdjStep S, uint32_t np)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (uint32_t k = threadIdx.x; k < np; k += 256u) {
        a += S.red[3 * k];
        b += S.red[3 * k + 1];
        c += S.red[3 * k + 2];
    }
    block_sum3<256>(a, b, c);
    __shared__ float slc[2];
    if (threadIdx.x == 0) {
        const bool on = p.volume_correction && c > 0.0;
        const double lam = on ? (S.scal[0] - b) / c : 0.0, cb = on ? a / c : 0.0;
        slc[0] = (float)lam;
        slc[1] = (float)cb;
        if (blockIdx.x == 0) {
            S.rs[0] = lam;
            S.rs[1] = cb;
            S.rs[3] += cb;
        }
    }
    __syncthreads();
    const float lam = slc[0], cb = slc[1];
#pragma unroll
    for (uint32_t r = 0; r < ADJ_VSUM_PER_THREAD; ++r) {
        const uint32_t n = (blockIdx.x * ADJ_VSUM_PER_THREAD + r) * 256u + threadIdx.x;
        if (n < N) S.psi[n] = S.solid[n] ? 0.0f : psi_of(S.pb_in[n], S.phistar[n], lam, cb, p.eps_phi);
    }
}

// Add the target-volume path to dL/dphi0: M_target is the fluid sum of phi0.
__global__ __launch_bounds__(256) void k_add_fluid(uint32_t N, const uint8_t *__restrict__ solid,
                                                   float *__restrict__ pb, const double *__restrict__ rs)
{
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    if (n < N && !solid[n]) pb[n] += (float)rs[3];
}

// dst = src on the fluid nodes of `planes` planes of N floats; the solid
// entries of dst keep their values (no step writes them).
__global__ __launch_bounds__(256) void k_copy_fluid(uint32_t N, uint32_t planes, const uint8_t *__restrict__ solid,
                                                    const float *__restrict__ src, float *__restrict__ dst)
{
    const uint32_t n = blockIdx.x * 256u + threadIdx.x;
    if (n >= N || solid[n]) return;
    for (uint32_t q = 0; q < planes; ++q) dst[(size_t)q * N + n] = src[(size_t)q * N + n];
}

template <int NT>
__global__ __launch_bounds__(NT) void k_adj_main(Grid g, Tiling t, DevParams p, AdjStep S)
{
    const Node nd = tile_node(g, t, xcd_tile(blockIdx.x, t.ntiles));
    if (nd.in) adj_main_node(g, p, S, nd.x, nd.y, nd.z);
}

// Transpose of the gradient / Laplacian stencils as a 2.5-D LDS stencil: a
// workgroup owns a BX x BY column tile and marches up a z-chunk; LDS holds a
// ring of three planes of the (grad x, y, z; Laplacian) cotangent records with
// a halo of one.  The sums of adj_assemble_node, regrouped plane by plane with
// the tensor-product weights t(0) = 4, t(+-1) = 1: per plane, from the 3 x 3
// patch q around the column,
//   X = sum_dy t(dy) [q.x(+1, dy) - q.x(-1, dy)],  Y likewise with q.y,
//   Z = sum t(dx) t(dy) q.z,  tq = sum t(dx) t(dy) [q.w - q.w(0, 0)],  c = q.w(0, 0),
// then over planes -1, 0, +1 (rolled up the column):
//   -div = -(X_- + 4 X_0 + X_+ + Y_- + 4 Y_0 + Y_+ + Z_+ - Z_-) / 72,
//   lap  = (tq_- + 4 tq_0 + tq_+ + 36 ((c_- - c_0) + (c_+ - c_0))) / 36.
template <int BX, int BY>
__global__ __launch_bounds__(BX *BY) void k_adj_assemble_lds(Grid g, PhaseTiling pt, AdjStep S)
{
    constexpr int NT = BX * BY;
    constexpr int AX = BX + 2, AY = BY + 2;
    constexpr int PA = (AX * AY + NT - 1) / NT;
    __shared__ float4 sr[3][AY * AX];
    const uint32_t tile = xcd_tile(blockIdx.x, pt.ntiles);
    const int tcx = (int)(tile % (uint32_t)pt.ntx);
    const int tcy = (int)((tile / (uint32_t)pt.ntx) % (uint32_t)pt.nty);
    const int tcz = (int)(tile / ((uint32_t)pt.ntx * (uint32_t)pt.nty));
    const int x0 = tcx * BX, y0 = tcy * BY, z0 = tcz * pt.zc;
    const int z1 = min(z0 + pt.zc, g.nz);
    const int tid = threadIdx.x;
    const int lx = tid % BX, ly = tid / BX;
    const int x = x0 + lx, y = y0 + ly;
    const bool col_in = x < g.nx && y < g.ny;
    const float4 *rec4 = reinterpret_cast<const float4 *>(S.rec);
    const float *recl = S.rec + 4u * g.N;
    static_assert(PA <= 2, "two halo points per thread");
    // this thread's (up to) two halo points of a plane: in-plane global offset
    const int k0 = tid, k1 = tid + NT;
    const bool h0 = k0 < AX * AY, h1 = k1 < AX * AY;
    const uint32_t a0 = h0 ? (uint32_t)wrapc(x0 - 1 + k0 % AX, g.nx) + (uint32_t)wrapc(y0 - 1 + k0 / AX, g.ny) * (uint32_t)g.nx : 0u;
    const uint32_t a1 = h1 ? (uint32_t)wrapc(x0 - 1 + k1 % AX, g.nx) + (uint32_t)wrapc(y0 - 1 + k1 / AX, g.ny) * (uint32_t)g.nx : 0u;
    auto slot = [&](int zz) { return (zz - z0 + 4) % 3; };
    float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
    auto fetch = [&](int zz) {
        const uint32_t zo = (uint32_t)wrapc(zz, g.nz) * g.nxny;
        if (h0) v0 = rec4[a0 + zo];
        if (h1) v1 = rec4[a1 + zo];
    };
    auto store = [&](int zz) {
        float4 *dst = sr[slot(zz)];
        if (h0) dst[k0] = v0;
        if (h1) dst[k1] = v1;
    };
    struct PS {
        float X, Y, Z, tq, c;
    };
    const int c0 = (ly + 1) * AX + lx + 1;
    auto psums = [&](int zz) {
        const float4 *pl = sr[slot(zz)];
        float4 q[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) q[j] = pl[c0 + (j / 3 - 1) * AX + (j % 3 - 1)];
        PS r;
        r.c = q[4].w;
        r.X = (q[2].x - q[0].x) + 4.0f * (q[5].x - q[3].x) + (q[8].x - q[6].x);
        r.Y = (q[6].y - q[0].y) + 4.0f * (q[7].y - q[1].y) + (q[8].y - q[2].y);
        r.Z = (q[0].z + q[2].z + q[6].z + q[8].z) + 4.0f * (q[1].z + q[3].z + q[5].z + q[7].z) + 16.0f * q[4].z;
        r.tq = (q[0].w - r.c) + (q[2].w - r.c) + (q[6].w - r.c) + (q[8].w - r.c) +
               4.0f * ((q[1].w - r.c) + (q[3].w - r.c) + (q[5].w - r.c) + (q[7].w - r.c));
        return r;
    };
    fetch(z0 - 1);
    store(z0 - 1);
    fetch(z0);
    store(z0);
    fetch(z0 + 1);
    __syncthreads();
    PS sm = psums(z0 - 1), sc = psums(z0);
    for (int z = z0; z < z1; ++z) {
        // One barrier per plane: this plane reads only the slot of z + 1; the
        // store below (slot of z + 1) overwrites plane z - 2, which no wave
        // still reads (waves are at most one plane apart).
        store(z + 1);
        __syncthreads();
        if (z + 1 < z1) fetch(z + 2);  // lands while this plane computes
        const PS sp = psums(z + 1);
        if (col_in) {
            const float dv = (sm.X + 4.0f * sc.X + sp.X + sm.Y + 4.0f * sc.Y + sp.Y + sp.Z - sm.Z) * (1.0f / 72.0f);
            const float lp = (sm.tq + 4.0f * sc.tq + sp.tq + 36.0f * ((sm.c - sc.c) + (sp.c - sc.c))) * (1.0f / 36.0f);
            const uint32_t n = (uint32_t)x + (uint32_t)y * (uint32_t)g.nx + (uint32_t)z * g.nxny;
            S.pb_out[n] = recl[n] + lp - dv;
        }
        sm = sc;
        sc = sp;
    }
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
    const unsigned nr = nblocks(g.N, 256 * ADJ_VSUM_PER_THREAD);
    k_adj_vsum<<<nr, 256, 0, s>>>(g.N, S.solid, S.pb_in, S.phistar, p.eps_phi, S.red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_adj_psi<<<nr, 256, 0, s>>>(g.N, p, S, nr);
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
    (void)t;
    if (g.nx >= 64) {
        const PhaseTiling pt = phase_tiling(g, 64, 4);
        k_adj_assemble_lds<64, 4><<<pt.ntiles, 256, 0, s>>>(g, pt, S);
    } else {
        const PhaseTiling pt = phase_tiling(g, 16, 16);
        k_adj_assemble_lds<16, 16><<<pt.ntiles, 256, 0, s>>>(g, pt, S);
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

hipError_t launch_copy_fluid(const Grid &g, const uint8_t *solid, int planes, const float *src, float *dst,
                             hipStream_t s)
{
    k_copy_fluid<<<nblocks(g.N, 256), 256, 0, s>>>(g.N, (uint32_t)planes, solid, src, dst);
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
