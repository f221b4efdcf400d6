// Allocation-free variant of fwi_gradient.  The workspace that fwi_gradient
// takes from its caller (coefficients, geometry tables, forward and adjoint
// states, checkpoints, segment buffer, correlation planes, residual, misfit
// partials) lives here in one file-scope device array instead, for callers
// that cannot allocate device memory at all.
//
// The array is resolved to a device address once per device, on the first
// call made with that device current, with hipGetSymbolAddress; host code
// only ever passes that address on (the array's own name in host code is a
// host-side stand-in, not a device address).  Every call on one device
// shares that device's array: fwi_gradient writes every part of the
// workspace it later reads within the same call (states and correlation
// planes are cleared by fill kernels, checkpoints and the segment buffer are
// written before they are read), so what a previous call left behind never
// reaches a result.  Calls that overlap in time on one device race on the
// array and must be ordered by the caller.
#include "fwi.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

__device__ __align__(256) unsigned char scratch[FWI_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FWI_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FWI_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FWI_OK;
}

}  // namespace

extern "C" int fwi_gradient_static(const fwi_grid *grid, const fwi_geom *geom,
                                   const float *eps_r, const float *sigma,
                                   const float *observed, double *misfit,
                                   float *grad_eps_r, float *grad_sigma,
                                   float *traces_out, void *stream) {
    // host-only checks first: an invalid or oversized problem launches
    // nothing and makes no HIP call
    size_t need = 0;
    int rc = fwi_workspace_bytes(grid, geom, -1, &need);
    if (rc != FWI_OK) return rc;
    if (need > (size_t)FWI_STATIC_SCRATCH_BYTES) return FWI_ESCRATCH;
    if (!eps_r || !sigma || !observed || !misfit || !grad_eps_r || !grad_sigma)
        return FWI_EINVAL;
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != FWI_OK) return rc;
    // one shot group: no streams or events are created
    return fwi_gradient_ex(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                           traces_out, ws, (size_t)FWI_STATIC_SCRATCH_BYTES, stream, nullptr, 1);
}
