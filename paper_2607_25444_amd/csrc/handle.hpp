// handle.hpp -- the plain handle of libcac and the host helpers that the
// runtime sources share.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/cac.h"
#include "cac_internal.hpp"

namespace cac {
struct AdjTape;  // recording of a forward sweep for the reverse pass
void tape_free(cac_handle *h);
void tape_invalidate(cac_handle *h);  // the recorded sweep no longer matches the state
}  // namespace cac

struct cac_handle {
    int dev = 0;
    cac::Grid g{};
    cac::Tiling t{};
    cac_params prm{};
    cac::DevParams dp{};
    cac::Fields F{};
    hipStream_t stream = nullptr;
    cac_alloc_fn alloc = nullptr;
    void *alloc_user = nullptr;
    std::vector<void *> owned;  // hipMalloc'd when no callback
    bool geometry = false, state = false;
    int cur = 0;                // parity of the A/B buffers holding the current state
    long long steps = 0;
    size_t partial_cap = 0;     // entries of F.partial
    int wall_cap = 0;
    // host copies of the wall tables
    std::vector<int32_t> widx, wn6, wdonor;
    int nskip = 0;
    // graph replay of two steps (even/odd buffer parity)
    bool use_graph = false;
    int debug = 0;              // CAC_DEBUG_* flags (cac_set_debug)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;  // capture needs a stream other than the null stream
    long long geom_serial = 0;   // incremented by every cac_set_geometry
    int sub = 0;                 // next substep of cac_debug_substep (0 = W ... 3 = V)
    cac::AdjTape *tape = nullptr;  // created by the first recorded sweep
    std::string err;
};


namespace cac {
// Record an error message on the handle and return the status.
cac_status fail(cac_handle *h, cac_status s, const char *fmt, ...);
// Device memory from the allocation callback (or hipMalloc, freed at destroy), 256-byte aligned.
void *dev_alloc(cac_handle *h, size_t bytes);
// Enqueue one plain step W -> H -> P -> V on h->stream and flip the buffer parity.
cac_status run_step(cac_handle *h);
}  // namespace cac

#define HIPCHK(h, call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return cac::fail(h, CAC_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)
