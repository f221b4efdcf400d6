// Definitions behind the host-only HIP stand-in (see hip/hip_runtime.h in
// this directory) and inert kernel launchers, for the sanitizer build of the
// library's host code.  TEST INFRASTRUCTURE ONLY.
#include <hip/hip_runtime.h>

#include <cstring>

#include "fwi_internal.h"

struct ihipStream_t { int unused; };
struct ihipEvent_t { int unused; };

extern "C++" {

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t) {
    if (bytes) std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new ihipStream_t{0};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
// graph capture is refused: batched plans then issue their steps one by one
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorUnknown; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    *g = nullptr;
    return hipErrorUnknown;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, hipGraphNode_t *, char *, size_t) {
    return hipErrorUnknown;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorUnknown; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new ihipEvent_t{0};
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    *e = new ihipEvent_t{0};
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *device) {
    *device = 0;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol) {
    *ptr = const_cast<void *>(symbol);
    return hipSuccess;
}

}  // extern "C++"

namespace fwi {

// Kernels do not run here.  Fills and the values the host reads back are
// written, so that the host code sees well-defined memory.
hipError_t launch_fill(float *dst, size_t n, float v, hipStream_t) {
    for (size_t i = 0; i < n; ++i) dst[i] = v;
    return hipSuccess;
}
hipError_t launch_coefficients(const float *, const float *, float *, float *, int, int, int,
                               double, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_profiles(const Dims &, const Profiles &, hipStream_t) { return hipSuccess; }
hipError_t launch_gradient_finalize(const float *, const float *, const float *, const float *,
                                    int, size_t, float *, float *, int, int, int, double,
                                    hipStream_t) {
    return hipSuccess;
}
hipError_t launch_residual_misfit(const float *, const float *, float *, size_t, double *,
                                  double *misfit, hipStream_t) {
    *misfit = 0.0;
    return hipSuccess;
}
hipError_t launch_finite_check(const float *, size_t, const float *, size_t, const double *,
                               double *, int *flag, hipStream_t) {
    *flag = 0;
    return hipSuccess;
}
// The merged copies are carried out, so the sanitizer checks every entry
// against its buffers.
hipError_t launch_copy_table(const CopyEntry *tab, const unsigned long long *cum, int nent,
                             unsigned long long total, hipStream_t) {
    if (nent < 1 || cum[nent] != total) return hipErrorInvalidValue;
    for (int e = 0; e < nent; ++e) {
        if (cum[e + 1] - cum[e] != tab[e].n) return hipErrorInvalidValue;
        std::memcpy(tab[e].dst, tab[e].src, tab[e].n * sizeof(float));
    }
    return hipSuccess;
}
hipError_t launch_fwd_stream(const FwdStreamArgs &a, hipStream_t) {
    return a.nlev >= 1 && a.nlev <= a.tl.depth ? hipSuccess : hipErrorInvalidValue;
}
hipError_t launch_adj_stream(const AdjStreamArgs &a, hipStream_t) {
    return a.nlev >= 1 && a.nlev <= a.tl.depth ? hipSuccess : hipErrorInvalidValue;
}
unsigned stream_blocks(int S, const Tiling &tl) { return (unsigned)S * tl.nstrip * tl.nband; }
// The forward table is read, so the sanitizer checks it and its block
// offsets, and every entry must make the launch's level-store choice.
hipError_t launch_fwd_table(const FwdStreamArgs *tab, const unsigned *boff, int nm,
                            unsigned nblocks, int, bool, int lev, hipStream_t) {
    if (nm < 1 || boff[0] != 0 || boff[nm] != nblocks) return hipErrorInvalidValue;
    if (lev != 0 && lev != 1) return hipErrorInvalidValue;
    for (int m = 0; m < nm; ++m)
        if ((tab[m].E_lev != nullptr) != (lev == 1)) return hipErrorInvalidValue;
    return hipSuccess;
}
hipError_t launch_adj_table(const AdjStreamArgs *, const unsigned *, int, unsigned, int, bool,
                            hipStream_t) {
    return hipSuccess;
}

}  // namespace fwi
