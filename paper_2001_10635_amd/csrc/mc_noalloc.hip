// Monte Carlo without any allocation, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// reach_montecarlo_noalloc runs the kernels of reach_montecarlo_range (the
// per-sample RK4 and the min / max reduction of Algorithm 4) with their
// per-wave partial minima and maxima in `scratch`, a fixed array of this file
// in device memory, instead of a caller workspace.  Each device the library
// runs on holds its own copy of the array from the module's load until the
// process ends.  In host code the name `scratch` is only a host-side stand-in:
// the device address of each device's copy is looked up once per device, with
// that device current (reach_ctx_create calls noalloc_setup), and only that
// address is ever handed to kernels.
//
// Nothing in the array needs clearing between calls: every partial a
// reduction reads is written by the same call's sampling kernel first.  Calls
// that overlap on one device (two streams, two host threads) share the array
// and race; serialise them.
#include <mutex>

#include "../../include/reach.h"
#include "kernels.hpp"
#include "rt.hpp"

namespace reach {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];
bool g_done[kMaxDevices];

}  // namespace

// With `device` current: looks up that device's copy of `scratch` once.
// Returns the lookup's error (the same one on every later call).
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        g_err[device] = e;
        g_done[device] = true;
    }
    return g_err[device];
}

}  // namespace reach

extern "C" {

size_t reach_noalloc_scratch_bytes(void) { return reach::kScratchBytes; }

reach_status reach_montecarlo_noalloc(reach_ctx* c, const reach_system* s, reach_dtype dtype,
                                      const void* x_lo, const void* x_hi, const void* p_lo,
                                      const void* p_hi, double t0, double dt, int64_t nsteps,
                                      int64_t s0, int64_t m, uint64_t seed, void* r_min,
                                      void* r_max, void* stream) {
    if (!c) return REACH_E_INVAL;
    const int device = reach::rt::ctx_device(c);
    // Arguments reach_montecarlo_range rejects are left to it (same errors);
    // a valid call whose partials do not fit the array is refused here.
    const size_t need = reach_workspace_bytes(c, s, dtype, m);
    if (need != (size_t)-1 && need > reach::kScratchBytes)
        return reach::rt::set_error(
            c, REACH_E_NOMEM,
            "Monte Carlo partials need " + std::to_string(need) +
                " bytes; the no-allocation scratch holds " + std::to_string(reach::kScratchBytes) +
                " (lower the option mc.waves)");
    if (hipSetDevice(device) != hipSuccess)
        return reach::rt::set_error(c, REACH_E_DEVICE, "hipSetDevice failed");
    const hipError_t e = reach::noalloc_setup(device);
    if (e != hipSuccess)
        return reach::rt::set_error(c, REACH_E_DEVICE,
                                    std::string("scratch address lookup: ") + hipGetErrorString(e));
    void* ptr = reach::g_ptr[device];
    return reach_montecarlo_range(c, s, dtype, x_lo, x_hi, p_lo, p_hi, t0, dt, nsteps, s0, m, seed,
                                  r_min, r_max, ptr, reach::kScratchBytes, stream);
}

}  // extern "C"
