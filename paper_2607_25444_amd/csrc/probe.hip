// probe.hip -- bandwidth ceiling of the collide-stream's access pattern.
#include "probe.hpp"
#include "step_device.hpp"

namespace cac {

// Bandwidth probe with the memory access pattern of k_hydro and none of its
// arithmetic: each node pulls its 27 populations from the upstream
// neighbours (periodic wrap, no bounce-back) and stores them, 216 bytes per
// node.  Same tiling, workgroup order and load hints as k_hydro.
template <int NT, bool NTL>
__global__ __launch_bounds__(NT) void k_pull_copy(Grid g, Tiling t, const float *__restrict__ fin,
                                                  float *__restrict__ fout)
{
    const Node nd = tile_node(g, t, blockIdx.x);
    if (!nd.in) return;
    const Offs o = node_offsets(g, nd.x, nd.y, nd.z);
    const uint32_t n = at<0, 0, 0>(o), N = g.N;
    float f[27];
    static_for<27>([&](auto I) {
        constexpr int i = I;
        const uint32_t k = (uint32_t)i * N + at<-Lat::cx[i], -Lat::cy[i], -Lat::cz[i]>(o);
        if constexpr (NTL)
            f[i] = __builtin_nontemporal_load(&fin[k]);
        else
            f[i] = fin[k];
    });
    static_for<27>([&](auto I) {
        constexpr int i = I;
        __builtin_nontemporal_store(f[i], &fout[(uint32_t)i * N + n]);
    });
}

hipError_t launch_pull_copy(const Grid &g, const Tiling &t, const float *fin, float *fout, hipStream_t s)
{
    const int nt = t.bx * t.by * t.bz;
    const bool ntl = t.bx >= g.nx;
#define CAC_COPY(NT_)                                                                   \
    if (ntl)                                                                            \
        k_pull_copy<NT_, true><<<t.ntiles, NT_, t.hyd_lds, s>>>(g, t, fin, fout);               \
    else                                                                                \
        k_pull_copy<NT_, false><<<t.ntiles, NT_, t.hyd_lds, s>>>(g, t, fin, fout);
    switch (nt) {
    case 128: CAC_COPY(128) break;
    case 256: CAC_COPY(256) break;
    case 512: CAC_COPY(512) break;
    default: return hipErrorInvalidValue;
    }
#undef CAC_COPY
    return hipGetLastError();
}

}  // namespace cac
