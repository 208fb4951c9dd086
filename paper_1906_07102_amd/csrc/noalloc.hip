// Gridding through a plan without any allocation: the call's scratch (work
// counters, visibilities in entry order, per-item patches) lives in a
// file-scope device array of fixed size instead of a caller workspace.
//
// The array's name is a host-side stand-in in host code, not a device
// address; its address on a device comes from hipGetSymbolAddress, taken once
// per device with that device current and kept here. Each device that runs
// this call holds its own copy of the array until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lmgrid.h"

namespace lmg {
namespace noalloc {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;   // LMG_STATIC_SCRATCH_BYTES in lmgrid.h

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

}  // namespace noalloc
}  // namespace lmg

namespace {

using lmg::noalloc::kStaticScratchBytes;
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
lmg_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LMG_EHIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(lmg::noalloc::scratch)) != hipSuccess || !p) return LMG_EHIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LMG_OK;
}

}  // namespace

extern "C" {

lmg_status lmg_grid_planned_noalloc(const lmg_plan* p, const void* vis, const float* w, void* grid, int accumulate,
                                    void* stream) {
    if (!p) return LMG_EINVAL;
    size_t need = 0;
    lmg_status st = lmg_plan_scratch_size(p, LMG_OP_GRID, &need);
    if (st != LMG_OK) return st;
    if (need > kStaticScratchBytes) return LMG_ENOTSUP;
    void* sc = nullptr;
    st = scratch_address(&sc);
    if (st != LMG_OK) return st;
    return lmg_grid_planned(p, vis, w, grid, accumulate, sc, kStaticScratchBytes, stream);
}

}  // extern "C"
