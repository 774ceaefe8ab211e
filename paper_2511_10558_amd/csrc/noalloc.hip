// The workspace of abdf_solve_noalloc: a file-scope device array (one copy on
// every device the library runs on, held until the process ends) and static
// host buffers, so that the entry point calls no allocating routine.
#include "noalloc.hpp"

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/astrobdf.h"

namespace abdf {

// In host code `scratch` names a host-side stand-in, not device memory: every
// use goes through the device address that noalloc_workspace looks up.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 16;

struct HostState {
    int32_t cnt[kCountSlots];
    int32_t fin[kNoAllocMaxSlots];
    int32_t admit_slots[kNoAllocMaxSlots];
    long long admit_cells[kNoAllocMaxSlots];
    int32_t free_list[kNoAllocMaxSlots];
    double atol[kMaxSpecies];
};

std::mutex g_mu;
void *g_scratch[kMaxDevices];       // device address of `scratch` on each device, null until looked up
HostState g_host[kMaxDevices];

}  // namespace

int noalloc_workspace(int device, void **scratch_ptr, HostBuffers *host, std::string &err) {
    if (device < 0 || device >= kMaxDevices) {
        err = "device index beyond the no-allocation entry point's table";
        return ABDF_E_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        // the array's name is a host-side stand-in; its address on this
        // device (current) comes from the runtime
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return ABDF_E_DEVICE;
        }
        g_scratch[device] = p;
    }
    *scratch_ptr = g_scratch[device];
    HostState &h = g_host[device];
    *host = HostBuffers{h.cnt, h.fin, h.admit_slots, h.admit_cells, h.free_list, h.atol, kNoAllocMaxSlots};
    return ABDF_OK;
}

}  // namespace abdf
