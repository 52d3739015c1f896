// A host-only stand-in for the part of the HIP runtime API that libacs's
// host sources call, for building those sources with the address and
// undefined-behaviour sanitizers on a machine without a GPU.  Test
// infrastructure only (see fake_hip.cpp): "device" memory is host memory,
// streams are queues of host closures that make progress only when the
// caller queries or synchronises, and kernels run the few task bodies the
// host logic depends on.
#pragma once
#include <stddef.h>
#include <stdint.h>

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
    hipErrorInvalidResourceHandle = 400,
    hipErrorUnknown = 999
} hipError_t;

typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipDeviceAttribute_t {
    hipDeviceAttributeMultiprocessorCount = 1,
    hipDeviceAttributeWallClockRate = 2
} hipDeviceAttribute_t;

struct dim3 {
    uint32_t x, y, z;
    constexpr dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph *hipGraph_t;
typedef struct hipGraphNode *hipGraphNode_t;
typedef struct hipGraphExec *hipGraphExec_t;

typedef struct hipKernelNodeParams {
    dim3 blockDim;
    void **extra;
    void *func;
    dim3 gridDim;
    void **kernelParams;
    unsigned int sharedMemBytes;
} hipKernelNodeParams;

#define hipStreamNonBlocking 0x01
#define hipEventDefault 0x0
#define hipEventDisableTiming 0x2
#define hipHostMallocMapped 0x2
#define hipHostMallocCoherent 0x40000000

hipError_t hipSetDevice(int device);
hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t attr, int device);
hipError_t hipRuntimeGetVersion(int *version);
hipError_t hipDeviceSynchronize(void);
const char *hipGetErrorString(hipError_t e);

hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned int flags);
hipError_t hipHostFree(void *p);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemset(void *dst, int value, size_t bytes);

hipError_t hipStreamCreate(hipStream_t *s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamQuery(hipStream_t s);
typedef int hipDevice_t;
hipError_t hipStreamGetDevice(hipStream_t s, hipDevice_t *device);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int flags);

hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);

hipError_t hipGraphCreate(hipGraph_t *g, unsigned int flags);
hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t g, const hipGraphNode_t *deps, size_t n_deps,
                                 const hipKernelNodeParams *params);
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *err_node, char *log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t g);
