// kf_noalloc.hip -- kf_run_noalloc: run a compiled plan on a fixed device
// array owned by the library instead of a caller workspace, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation).
//
// The array lives in this code object, so every GPU the library runs on holds
// its own copy, at its own address, until the process ends. Host code never
// passes the array's name to a kernel or a copy: it is a host-side stand-in.
// The device address is looked up once per device with hipGetSymbolAddress
// (the device current at that moment) and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kf_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[KF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device (null until looked up)

// The current device's address of `scratch`, looked up on first use.
kf_status scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return kf::set_error(KF_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return kf::set_error(KF_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return kf::set_error(KF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return KF_OK;
}

}  // namespace

extern "C" kf_status kf_run_noalloc(kf_plan* p, void* stream) {
    size_t need = 0;
    kf_status st = kf_plan_workspace_bytes(p, &need);
    if (st != KF_OK) return st;
    if (need > (size_t)KF_NOALLOC_SCRATCH_BYTES)
        return kf::set_error(KF_ERR_WORKSPACE, "plan needs " + std::to_string(need) +
                                                   " bytes of workspace; kf_run_noalloc has " +
                                                   std::to_string((size_t)KF_NOALLOC_SCRATCH_BYTES));
    st = kf::plan_loaded(p);
    if (st != KF_OK) return st;
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != KF_OK) return st;
    return kf::run_on_workspace(p, ws, stream);
}
