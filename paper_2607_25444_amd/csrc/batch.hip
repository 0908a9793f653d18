// batch.hip -- persistent batched kernels: many independent lattices of
// uneven size and contact angle advanced by one launch per substep.
//
// A fixed grid of workgroups (sized from the occupancy of the kernel) walks a
// host-built list of (domain, tile) work items with stride gridDim.x; each
// item runs the same device body as the single-lattice kernels on that
// domain's slice of the concatenated arrays.  Volume sums are kept per domain
// (partial index = the domain's first partial + its tile), so the FP64 totals
// do not depend on the schedule.
#include "batch_r1.hpp"
#include "r1_device.hpp"
#include "step_device.hpp"

namespace cac {

// Pointers of one domain for buffer parity `cur`, chosen with selects (a
// runtime-indexed local array would be placed in scratch memory).
struct DomPtrs {
    const float *fin;
    float *fout;
    float *phi_cur, *phi_oth;
    float *u, *a;
    const uint32_t *nbr;
    const uint8_t *solid;
};

__device__ __forceinline__ DomPtrs domain_ptrs(const BatchPtrs &B, const BatchDomain &d, int cur)
{
    DomPtrs P;
    float *f0 = B.f[0], *f1 = B.f[1], *p0 = B.phi[0], *p1 = B.phi[1];
    P.fin = (cur ? f1 : f0) + 27u * d.off;
    P.fout = (cur ? f0 : f1) + 27u * d.off;
    P.phi_cur = (cur ? p1 : p0) + d.off;
    P.phi_oth = (cur ? p0 : p1) + d.off;
    P.u = B.u + 3u * d.off;
    P.a = B.a + 3u * d.off;
    P.nbr = B.nbr + d.off;
    P.solid = B.solid + d.off;
    return P;
}

// Items of this workgroup.  One workgroup per item: the XCD-aware renumbering
// of the single-lattice kernels.  Persistent grid (a multiple of 8): XCD x =
// blockIdx % 8 owns the contiguous eighth x of the item list and its
// workgroups stride through it, so neighbouring tiles share that XCD's L2.
struct ItemRange {
    uint32_t first, end, stride;
};

__device__ __forceinline__ ItemRange item_range(uint32_t nitems)
{
    const uint32_t G = gridDim.x, b = blockIdx.x;
    ItemRange r;
    if (G >= nitems) {
        r.first = b < nitems ? xcd_tile(b, nitems) : nitems;
        r.end = r.first < nitems ? r.first + 1 : nitems;
        r.stride = 1;
    } else if ((G & 7u) == 0) {
        const uint32_t x = b & 7u;
        r.first = (uint32_t)(((uint64_t)nitems * x) >> 3) + (b >> 3);
        r.end = (uint32_t)(((uint64_t)nitems * (x + 1)) >> 3);
        r.stride = G >> 3;
    } else {
        r.first = b;
        r.end = nitems;
        r.stride = G;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_bghost(BatchPtrs B, const BatchDomain *__restrict__ dom, uint32_t nwall,
                                                int cur)
{
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= nwall) return;
    const BatchDomain d = dom[B.wall_dom[k]];
    const DomPtrs P = domain_ptrs(B, d, cur);
    ghost_node(d.g, d.p, (int)k, B.wall_idx, B.wall_q, B.wall_n, B.theta, P.phi_cur, P.phi_oth, P.nbr, P.a);
}

// Hydrodynamic items carry, in the top bit of the tile index, whether the tile
// holds a solid node or a node next to one (set on the device by
// k_bitem_walls whenever the item list changes); other tiles skip the
// neighbour-mask load.
constexpr uint32_t ITEM_WALLS = 0x80000000u;

// The descriptor array is a separate read-only, non-aliased argument so that
// its uniform fields are fetched with scalar loads into scalar registers.
template <int NT>
__global__ __launch_bounds__(NT) void k_bhydro(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                               const uint2 *__restrict__ items, uint32_t nitems, int cur)
{
    const ItemRange r = item_range(nitems);
    uint2 nxt = r.first < r.end ? items[r.first] : make_uint2(0u, 0u);
    for (uint32_t it = r.first; it < r.end; it += r.stride) {
        const uint2 dt = nxt;
        if (it + r.stride < r.end) nxt = items[it + r.stride];  // next record loads during this item
        const BatchDomain d = dom[dt.x];
        const DomPtrs P = domain_ptrs(B, d, cur);
        hydro_node<false>(d.g, d.p, tile_node(d.g, d.t, dt.y & ~ITEM_WALLS), P.fin, P.fout, P.phi_cur, P.nbr, P.u,
                          B.flag, (dt.y & ITEM_WALLS) != 0u);
    }
}

// One workgroup per item (the schedule's grid multiplier 0): no loop state.
// Items keep the hardware workgroup order (round-robin over the XCDs), and a
// domain whose tile spans its rows reads populations with non-temporal
// loads, as in the single-lattice kernel (the branch is uniform per
// workgroup): 17.0 -> 17.6 GLUPS on the 64-domain batch.
template <int NT>
__global__ __launch_bounds__(NT) void k_bhydro1(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                                const uint2 *__restrict__ items, uint32_t nitems, int cur)
{
    const uint2 dt = items[blockIdx.x];
    const BatchDomain d = dom[dt.x];
    const DomPtrs P = domain_ptrs(B, d, cur);
    const Node nd = tile_node(d.g, d.t, dt.y & ~ITEM_WALLS);
    const bool walls = (dt.y & ITEM_WALLS) != 0u;
    if (d.t.bx >= d.g.nx)
        hydro_node<true>(d.g, d.p, nd, P.fin, P.fout, P.phi_cur, P.nbr, P.u, B.flag, walls);
    else
        hydro_node<false>(d.g, d.p, nd, P.fin, P.fout, P.phi_cur, P.nbr, P.u, B.flag, walls);
}

// Sets the wall bit of every hydrodynamic item: one workgroup per item, one
// thread per node of its tile.
template <int NT>
__global__ __launch_bounds__(NT) void k_bitem_walls(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                                    uint2 *__restrict__ items)
{
    const uint2 dt = items[blockIdx.x];
    const uint32_t tile = dt.y & ~ITEM_WALLS;
    const BatchDomain d = dom[dt.x];
    const Node nd = tile_node(d.g, d.t, tile);
    const int any = nd.in && B.nbr[d.off + (uint32_t)nd.x +
                                   (uint32_t)d.g.nx * ((uint32_t)nd.y + (uint32_t)d.g.ny * (uint32_t)nd.z)] != 0u;
    const int r = __syncthreads_or(any);
    if (threadIdx.x == 0) items[blockIdx.x].y = tile | (r ? ITEM_WALLS : 0u);
}

template <int BX, int BY>
__global__ __launch_bounds__(BX *BY) void k_bphase(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                                   const uint2 *__restrict__ items, uint32_t nitems, int cur)
{
    const ItemRange r = item_range(nitems);
    uint2 nxt = r.first < r.end ? items[r.first] : make_uint2(0u, 0u);
    for (uint32_t it = r.first; it < r.end; it += r.stride) {
        __syncthreads();  // the previous item is done with the workgroup's LDS
        const uint2 dt = nxt;
        if (it + r.stride < r.end) nxt = items[it + r.stride];
        const BatchDomain d = dom[dt.x];
        const DomPtrs P = domain_ptrs(B, d, cur);
        phase_tile<BX, BY>(d.g, d.pt, d.p, dt.y, P.phi_cur, P.phi_oth, P.u, P.a, P.solid,
                           B.partial + d.p_item0 + dt.y, B.flag, B.chunk, d.off);
    }
}

// One workgroup per item (the schedule's grid multiplier 0).  Without the item
// loop of k_bphase the kernel keeps the register budget of the single-lattice
// phase kernel (about 120 VGPRs instead of 170-200), so twice the waves fit.
template <int BX, int BY>
__global__ __launch_bounds__(BX *BY) void k_bphase1(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                                    const uint2 *__restrict__ items, uint32_t nitems, int cur)
{
    const uint2 dt = items[xcd_tile(blockIdx.x, nitems)];
    const BatchDomain d = dom[dt.x];
    const DomPtrs P = domain_ptrs(B, d, cur);
    phase_tile<BX, BY>(d.g, d.pt, d.p, dt.y, P.phi_cur, P.phi_oth, P.u, P.a, P.solid, B.partial + d.p_item0 + dt.y,
                       B.flag, B.chunk, d.off);
}

// One workgroup per domain: lambda_k from its tile partials in a fixed order.
__global__ __launch_bounds__(256) void k_bvol_finalize(BatchPtrs B, const BatchDomain *__restrict__ dom)
{
    const BatchDomain d = dom[blockIdx.x];
    double x = 0.0, y = 0.0;
    for (uint32_t k = threadIdx.x; k < d.pt.ntiles; k += 256u) {
        const double2 v = B.partial[d.p_item0 + k];
        x += v.x;
        y += v.y;
    }
    block_sum2<256>(x, y);
    if (threadIdx.x == 0) {
        double *sc = B.scal + 8u * blockIdx.x;
        const double lam = (d.p.volume_correction && y > 0.0) ? (sc[0] - x) / y : 0.0;
        sc[1] = lam;
        sc[2] = x;
        sc[3] = y;
    }
}

// phi <- phi* + lambda_k chi(phi*) on fluid nodes (Eq. (53)), four consecutive
// nodes of the concatenated arrays per thread (VEC: 16-byte phi and 4-byte
// mask loads).  A workgroup covers one 1024-node chunk; when the phase update
// wrote no interface node there (chunk byte clear) it returns at once, else it
// clears the byte for the next step.  The domain of the first node comes from
// a host-built table of the domain of each 256-node block; a later node past
// the domain's end belongs to a following domain (quads straddle domains only
// at their boundaries).  The population and mask loads do not depend on the
// lookup.
template <bool VEC>
__global__ __launch_bounds__(256) void k_bvol_apply(BatchPtrs B, const BatchDomain *__restrict__ dom, int cur_next)
{
    if (B.chunk) {
        if (!B.chunk[blockIdx.x]) return;  // the same for the whole workgroup
        __syncthreads();                    // every thread has read the byte before it is cleared
        if (threadIdx.x == 0) B.chunk[blockIdx.x] = 0;
    }
    const uint32_t n0 = 4u * (blockIdx.x * 256u + threadIdx.x);
    if (n0 >= B.ntot) return;
    float *phi = cur_next ? B.phi[1] : B.phi[0];
    uint8_t s[4];
    float v[4];
    const int cnt = (int)min(4u, B.ntot - n0);
    if (VEC && cnt == 4) {
        const uchar4 s4 = *reinterpret_cast<const uchar4 *>(B.solid + n0);
        const float4 v4 = *reinterpret_cast<const float4 *>(phi + n0);
        s[0] = s4.x, s[1] = s4.y, s[2] = s4.z, s[3] = s4.w;
        v[0] = v4.x, v[1] = v4.y, v[2] = v4.z, v[3] = v4.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[k] = k < cnt ? B.solid[n0 + k] : (uint8_t)1;
            v[k] = k < cnt ? phi[n0 + k] : 0.f;
        }
    }
    uint32_t lo = B.blk_dom[n0 >> 8];
    uint32_t end = B.dom_start[lo + 1];
    while (n0 >= end) end = B.dom_start[++lo + 1];
    float eps = dom[lo].p.eps_phi;
    double lam = B.scal[8u * lo + 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t n = n0 + (uint32_t)k;
        if (k > 0 && k < cnt && n >= end) {
            while (n >= end) end = B.dom_start[++lo + 1];
            eps = dom[lo].p.eps_phi;
            lam = B.scal[8u * lo + 1];
        }
        if (!s[k] && v[k] > eps && v[k] < 1.0f - eps)
            phi[n] = (float)((double)v[k] + lam * ((double)v[k] * (1.0 - (double)v[k])));
    }
}

// ------------------------------------------------------------------ gradient form
// collision = 1 (all domains of the batch): the record of each domain in its
// slice of the second population buffer, its rebuilt populations in the first.

template <int BX, int BY>
__global__ __launch_bounds__(BX *BY) void k_br1_rebuild(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                                        const uint2 *__restrict__ items)
{
    const uint2 dt = items[blockIdx.x];
    const BatchDomain d = dom[dt.x];
    r1_rebuild_tile<BX, BY>(d.g, d.pt, dt.y, B.f[1] + 27u * d.off, B.u + 3u * d.off, B.nbr + d.off,
                            B.f[0] + 27u * d.off);
}

template <int NT, bool SELF>
__global__ __launch_bounds__(NT) void k_br1_stream(BatchPtrs B, const BatchDomain *__restrict__ dom,
                                                   const uint2 *__restrict__ items, const float *__restrict__ pstar0,
                                                   int cur)
{
    const uint2 dt = items[blockIdx.x];
    const BatchDomain d = dom[dt.x];
    const Node nd = tile_node(d.g, d.t, dt.y & ~ITEM_WALLS);
    const float *fin = B.f[0] + 27u * d.off;
    const float *phi = (cur ? B.phi[1] : B.phi[0]) + d.off;
    float *rec = B.f[1] + 27u * d.off;
    if (d.t.bx >= d.g.nx)
        r1_stream_node<SELF, true>(d.g, d.p, nd, fin, phi, B.nbr + d.off, pstar0 + d.off, B.u + 3u * d.off, rec,
                                   B.flag, (dt.y & ITEM_WALLS) != 0u);
    else
        r1_stream_node<SELF, false>(d.g, d.p, nd, fin, phi, B.nbr + d.off, pstar0 + d.off, B.u + 3u * d.off, rec,
                                    B.flag, (dt.y & ITEM_WALLS) != 0u);
}

hipError_t launch_br1_rebuild(const BatchPtrs &B, int code, const uint2 *items, uint32_t nitems, hipStream_t s)
{
    if (!nitems) return hipSuccess;
    int bx, by;
    phase_shape_of(code, bx, by);
#define CAC_BR1R(BX_, BY_)                                                        \
    if (bx == BX_ && by == BY_) {                                                 \
        k_br1_rebuild<BX_, BY_><<<nitems, BX_ * BY_, 0, s>>>(B, B.dom, items);    \
        return hipGetLastError();                                                 \
    }
    CAC_BR1R(64, 8)
    CAC_BR1R(64, 4)
    CAC_BR1R(32, 8)
    CAC_BR1R(32, 16)
    CAC_BR1R(16, 16)
    CAC_BR1R(128, 4)
#undef CAC_BR1R
    return hipErrorInvalidValue;
}

hipError_t launch_br1_stream(const BatchPtrs &B, const float *pstar0, int nt, const uint2 *items, uint32_t nitems,
                             uint32_t lds, int cur, bool self, hipStream_t s)
{
    if (!nitems) return hipSuccess;
#define CAC_BR1S(NT_)                                                                        \
    if (self)                                                                                \
        k_br1_stream<NT_, true><<<nitems, NT_, lds, s>>>(B, B.dom, items, pstar0, cur);       \
    else                                                                                     \
        k_br1_stream<NT_, false><<<nitems, NT_, lds, s>>>(B, B.dom, items, pstar0, cur);
    switch (nt) {
    case 128: CAC_BR1S(128) break;
    case 256: CAC_BR1S(256) break;
    case 512: CAC_BR1S(512) break;
    default: return hipErrorInvalidValue;
    }
#undef CAC_BR1S
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers

hipError_t launch_bghost(const BatchPtrs &B, uint32_t nwall, int cur, hipStream_t s)
{
    if (!nwall) return hipSuccess;
    k_bghost<<<(nwall + 255u) / 256u, 256, 0, s>>>(B, B.dom, nwall, cur);
    return hipGetLastError();
}

hipError_t launch_bhydro(const BatchPtrs &B, int nt, const uint2 *items, uint32_t nitems, uint32_t grid, uint32_t lds, int cur,
                         hipStream_t s)
{
    if (!nitems) return hipSuccess;
    switch (nt) {
    case 128:
        if (grid >= nitems) k_bhydro1<128><<<nitems, 128, lds, s>>>(B, B.dom, items, nitems, cur);
        else k_bhydro<128><<<grid, 128, lds, s>>>(B, B.dom, items, nitems, cur);
        break;
    case 256:
        if (grid >= nitems) k_bhydro1<256><<<nitems, 256, lds, s>>>(B, B.dom, items, nitems, cur);
        else k_bhydro<256><<<grid, 256, lds, s>>>(B, B.dom, items, nitems, cur);
        break;
    case 512:
        if (grid >= nitems) k_bhydro1<512><<<nitems, 512, lds, s>>>(B, B.dom, items, nitems, cur);
        else k_bhydro<512><<<grid, 512, lds, s>>>(B, B.dom, items, nitems, cur);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bitem_walls(const BatchPtrs &B, int nt, uint2 *items, uint32_t nitems, hipStream_t s)
{
    if (!nitems) return hipSuccess;
    switch (nt) {
    case 128: k_bitem_walls<128><<<nitems, 128, 0, s>>>(B, B.dom, items); break;
    case 256: k_bitem_walls<256><<<nitems, 256, 0, s>>>(B, B.dom, items); break;
    case 512: k_bitem_walls<512><<<nitems, 512, 0, s>>>(B, B.dom, items); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bphase(const BatchPtrs &B, int code, const uint2 *items, uint32_t nitems, uint32_t grid, int cur,
                         hipStream_t s)
{
    if (!nitems) return hipSuccess;
    int bx, by;
    phase_shape_of(code, bx, by);
#define CAC_BPHASE(BX_, BY_)                                                        \
    if (bx == BX_ && by == BY_) {                                                   \
        if (grid >= nitems)                                                         \
            k_bphase1<BX_, BY_><<<nitems, BX_ * BY_, 0, s>>>(B, B.dom, items, nitems, cur); \
        else                                                                        \
            k_bphase<BX_, BY_><<<grid, BX_ * BY_, 0, s>>>(B, B.dom, items, nitems, cur); \
        return hipGetLastError();                                                   \
    }
    CAC_BPHASE(64, 8)
    CAC_BPHASE(64, 4)
    CAC_BPHASE(32, 8)
    CAC_BPHASE(32, 16)
    CAC_BPHASE(16, 16)
    CAC_BPHASE(128, 4)
#undef CAC_BPHASE
    return hipErrorInvalidValue;
}

hipError_t launch_bvolume(const BatchPtrs &B, int nt, const uint2 *items, uint32_t nitems, uint32_t grid, int cur_next,
                          hipStream_t s)
{
    (void)nt;
    (void)items;
    (void)nitems;
    (void)grid;
    k_bvol_finalize<<<B.ndom, 256, 0, s>>>(B, B.dom);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !B.ntot) return e;
    const unsigned nb = ((B.ntot + 3u) / 4u + 255u) / 256u;
    const float *phi = cur_next ? B.phi[1] : B.phi[0];
    if ((((uintptr_t)B.solid | (uintptr_t)phi) & 15u) == 0)
        k_bvol_apply<true><<<nb, 256, 0, s>>>(B, B.dom, cur_next);
    else
        k_bvol_apply<false><<<nb, 256, 0, s>>>(B, B.dom, cur_next);
    return hipGetLastError();
}

int batch_blocks_per_cu(int kind, int code, uint32_t lds)
{
    int nb = 0;
    hipError_t e = hipSuccess;
    if (kind == 0) {
        switch (code) {
        case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bhydro<128>, 128, lds); break;
        case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bhydro<256>, 256, lds); break;
        case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bhydro<512>, 512, lds); break;
        default: return 0;
        }
    } else {
        int bx, by;
        phase_shape_of(code, bx, by);
        if (bx == 64 && by == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bphase<64, 8>, 512, 0);
        else if (bx == 64 && by == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bphase<64, 4>, 256, 0);
        else if (bx == 32 && by == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bphase<32, 8>, 256, 0);
        else if (bx == 32 && by == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bphase<32, 16>, 512, 0);
        else if (bx == 16 && by == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bphase<16, 16>, 256, 0);
        else if (bx == 128 && by == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bphase<128, 4>, 512, 0);
        else return 0;
    }
    return e == hipSuccess ? nb : 0;
}

}  // namespace cac
