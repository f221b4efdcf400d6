/*
 * Host-only stand-in for the HIP runtime header, for the sanitizer build of
 * the library's host code (tests/test_sanitizers.py).  TEST INFRASTRUCTURE:
 * the product is always built with hipcc against the real HIP runtime.
 *
 * It declares only what the host code of the library uses.  The matching
 * definitions (hip_host_stub.cpp) treat "device" memory as host memory:
 * copies are memcpy, streams and events are inert, graph capture is
 * refused, and the kernel launchers do nothing except where the host code
 * reads back what a kernel wrote (fills, the finiteness flag).  So the
 * host code - validation, workspace layout, geometry sorting, the pass
 * loops, checkpoint copies, the batch schedule - runs on the CPU with every
 * copy checked by AddressSanitizer against the buffers' real extents.
 */
#ifndef FWI_HOST_ASAN_HIP_RUNTIME_H
#define FWI_HOST_ASAN_HIP_RUNTIME_H

#include <stddef.h>

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorUnknown = 999
} hipError_t;

typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph *hipGraph_t;
typedef struct hipGraphExec *hipGraphExec_t;
typedef struct hipGraphNode *hipGraphNode_t;

typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

#define hipStreamNonBlocking 0x1
#define hipEventDisableTiming 0x2

/* device-side qualifiers of a file-scope array: plain host storage here */
#define __device__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))

hipError_t hipGetDevice(int *device);
hipError_t hipSetDevice(int device);
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol);

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t stream);
hipError_t hipStreamSynchronize(hipStream_t stream);
hipError_t hipStreamCreateWithFlags(hipStream_t *stream, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t stream);
hipError_t hipStreamBeginCapture(hipStream_t stream, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t stream, hipGraph_t *graph);
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t graph, hipGraphNode_t *node,
                               char *log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t stream);
hipError_t hipGraphDestroy(hipGraph_t graph);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipEventCreate(hipEvent_t *event);
hipError_t hipEventCreateWithFlags(hipEvent_t *event, unsigned flags);
hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t event);
hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream);
hipError_t hipEventSynchronize(hipEvent_t event);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t start, hipEvent_t stop);
hipError_t hipGetLastError(void);

#endif
