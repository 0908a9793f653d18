// probe.hpp -- measurement kernel launcher (not part of the step).
#pragma once

#include <hip/hip_runtime.h>

#include "cac_internal.hpp"

namespace cac {

// 27-plane pull copy fin -> fout with the tiling and load hints of k_hydro.
hipError_t launch_pull_copy(const Grid &g, const Tiling &t, const float *fin, float *fout, hipStream_t s);

}  // namespace cac
