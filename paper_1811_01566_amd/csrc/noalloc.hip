// wf_das_noalloc: the DAS calls for callers that cannot allocate device
// memory.  Its geometry tables and split partial frames live in one static
// device array per GPU instead of library-allocated or caller-given memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>

#include "wf_internal.h"

namespace {

// The geometry tables of the largest geometry the calls accept (1024
// transmits and channels, a split work list) take about 2.1 MiB; the rest
// holds split partial frames of the small grids that split.
constexpr size_t kScratchBytes = WF_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each GPU the library has run on.  In host
// code the array's name is only a host-side stand-in: kernels and copies
// use these addresses.
std::mutex g_mu;
std::unordered_map<int, void*> g_scratch;

wf_status scratch_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return wf::report_hip(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return WF_OK;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return wf::report_hip(e, "hipGetSymbolAddress(scratch)");
    g_scratch.emplace(dev, p);
    *out = p;
    return WF_OK;
}

}  // namespace

extern "C" wf_status wf_das_noalloc(int32_t mode, const void* rf, const wf_probe* probe,
                                    const wf_acq* acq, const int32_t* tx_elem,
                                    const double* angles_rad, int32_t tref, const wf_grid* grid,
                                    float* out, void* stream) {
    // the arguments are validated before the scratch address is looked up
    return wf::das_scratch(mode, rf, probe, acq, tx_elem, angles_rad, tref, grid, out,
                           scratch_of_current_device, kScratchBytes, (hipStream_t)stream);
}
