// noalloc.hip -- the allocation-free entry point of libcac: the phase-field
// volume of Eq. (48) for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// It runs the kernels of cac_volume (per-block FP64 partials, then one
// workgroup that sums them in a fixed order), with the partials in a
// file-scope device array instead of handle memory.  Each device holds its own
// copy of the array until the process ends; host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address is looked up once per device with hipGetSymbolAddress and
// kept in g_scratch_ptr.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "../../include/cac.h"
#include "cac_internal.hpp"

namespace {

// 2^19 block partials of 16 bytes (8 MiB per device): one partial per 256
// nodes, so lattices of up to 2^27 nodes (512^3).
constexpr uint32_t kScratchPartials = 1u << 19;
constexpr unsigned long long kMaxNodes = 256ull * kScratchPartials;

static __device__ __align__(256) double2 scratch[kScratchPartials];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

thread_local char g_err[256] = "";

cac_status fail_free(cac_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

// Device address of this device's copy of `scratch` (looked up once, with the
// device current).
hipError_t scratch_of(int dev, double2 **out)
{
    std::call_once(g_scratch_once[dev], [dev] {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = p;
    });
    *out = static_cast<double2 *>(g_scratch_ptr[dev]);
    return g_scratch_err[dev];
}

}  // namespace

namespace cac {
// message of the last failed handle-free call on this thread
const char *free_call_error() { return g_err; }
}  // namespace cac

extern "C" cac_status cac_volume_noalloc(int nx, int ny, int nz, const uint8_t *d_solid, const float *d_phi,
                                         double *d_out, void *hip_stream)
{
    if (nx < 1 || ny < 1 || nz < 1)
        return fail_free(CAC_ERR_ARG, "cac_volume_noalloc: lattice %d x %d x %d has an empty axis", nx, ny, nz);
    const unsigned long long N = (unsigned long long)nx * ny * nz;
    if (N > kMaxNodes)
        return fail_free(CAC_ERR_ARG,
                         "cac_volume_noalloc: %llu nodes exceed the limit of %llu nodes of its static scratch "
                         "(%u partials)",
                         N, kMaxNodes, kScratchPartials);
    if (!d_solid || !d_phi || !d_out) return fail_free(CAC_ERR_ARG, "cac_volume_noalloc: null pointer");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_free(CAC_ERR_HIP, "cac_volume_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail_free(CAC_ERR_ARG, "cac_volume_noalloc: device %d out of range", dev);
    double2 *part = nullptr;
    e = scratch_of(dev, &part);
    if (e != hipSuccess || !part)
        return fail_free(CAC_ERR_HIP, "cac_volume_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    e = cac::launch_mass_into((uint32_t)N, d_solid, d_phi, part, d_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail_free(CAC_ERR_HIP, "cac_volume_noalloc: launch: %s", hipGetErrorString(e));
    return CAC_OK;
}
