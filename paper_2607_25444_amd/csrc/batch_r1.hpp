// batch_r1.hpp -- launchers of the gradient-form hydrodynamic substep
// (collision = 1) for batches of domains.  Not part of the public ABI.
#pragma once

#include "cac_internal.hpp"

namespace cac {

// Rebuild pass, one workgroup per phase item (domain, column tile of the
// domain's phase tiling, whose shape is the phase code's): the record planes
// in B.f[1] and the velocity give the post-collision populations in B.f[0].
hipError_t launch_br1_rebuild(const BatchPtrs &B, int phase_code, const uint2 *items, uint32_t nitems,
                              hipStream_t s);

// Stream pass, one workgroup per hydrodynamic item (domain, tile of nt
// nodes): pull, moments and collision into the record and u.  self: the first
// step after the initial state, which pulls each node's own equilibrium
// (p*0 from pstar0, u0 from B.u).  cur: parity of the phase-field buffers.
hipError_t launch_br1_stream(const BatchPtrs &B, const float *pstar0, int nt, const uint2 *items, uint32_t nitems,
                             uint32_t lds, int cur, bool self, hipStream_t s);

}  // namespace cac
