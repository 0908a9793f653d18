// adjoint_tables.hpp -- host-side tables of the ghost-update transpose:
// wall nodes grouped by donor (CSR), the node -> donor map and the list of
// nodes that a donor stencil reads.  Header-only (host code).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "cac_internal.hpp"

namespace cac {

struct DonorTables {
    std::vector<int32_t> don_node;   // donor node of each slot, ascending
    std::vector<int32_t> don_start;  // CSR offsets into don_wall (ndon + 1)
    std::vector<int32_t> don_wall;   // wall-node indices, grouped by donor, ascending within a donor
    std::vector<int32_t> don_map;    // N: donor slot of a node, -1 if it is no donor
    std::vector<uint32_t> near;      // nodes within one link of a donor, ascending; bit 31: active wall node
};

// widx: wall-node list (node index, ascending); wdonor: donor link per wall
// node (-1: skipped).  Donor of wall node b: b + c_q with periodic wrap.
inline void build_donor_tables(const Grid &g, const int32_t *widx, const int32_t *wdonor, int nwall, DonorTables &T)
{
    auto wrapn = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    auto node = [&](int x, int y, int z) {
        return (uint32_t)wrapn(x, g.nx) + (uint32_t)g.nx * ((uint32_t)wrapn(y, g.ny) + (uint32_t)g.ny * (uint32_t)wrapn(z, g.nz));
    };
    std::vector<std::pair<uint32_t, int32_t>> pairs;  // (donor node, wall index)
    std::vector<uint8_t> active(g.N, 0);
    for (int k = 0; k < nwall; ++k) {
        const int q = wdonor[k];
        if (q < 0) continue;
        const uint32_t b = (uint32_t)widx[k];
        const int x = (int)(b % (uint32_t)g.nx), y = (int)((b / (uint32_t)g.nx) % (uint32_t)g.ny),
                  z = (int)(b / g.nxny);
        pairs.emplace_back(node(x + Lat::cx[q], y + Lat::cy[q], z + Lat::cz[q]), k);
        active[b] = 1;
    }
    std::sort(pairs.begin(), pairs.end());
    T.don_node.clear();
    T.don_start.clear();
    T.don_wall.clear();
    T.don_map.assign(g.N, -1);
    for (size_t e = 0; e < pairs.size(); ++e) {
        if (e == 0 || pairs[e].first != pairs[e - 1].first) {
            T.don_map[pairs[e].first] = (int32_t)T.don_node.size();
            T.don_node.push_back((int32_t)pairs[e].first);
            T.don_start.push_back((int32_t)e);
        }
        T.don_wall.push_back(pairs[e].second);
    }
    T.don_start.push_back((int32_t)pairs.size());
    std::vector<uint8_t> mark(g.N, 0);
    for (int32_t d : T.don_node) {
        const uint32_t dn = (uint32_t)d;
        const int x = (int)(dn % (uint32_t)g.nx), y = (int)((dn / (uint32_t)g.nx) % (uint32_t)g.ny),
                  z = (int)(dn / g.nxny);
        for (int i = 0; i < 27; ++i) mark[node(x + Lat::cx[i], y + Lat::cy[i], z + Lat::cz[i])] = 1;
    }
    T.near.clear();
    for (uint32_t n = 0; n < g.N; ++n)
        if (mark[n]) T.near.push_back(n | (active[n] ? 0x80000000u : 0u));
}

}  // namespace cac
