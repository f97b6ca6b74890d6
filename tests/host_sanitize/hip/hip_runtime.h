// Host-only stand-in for the subset of the HIP runtime API that the serving
// loop (server.hip) and the headers it includes use, so that the scheduler
// can be built with g++ under AddressSanitizer, UndefinedBehaviorSanitizer
// and ThreadSanitizer on a machine without a GPU.  "Device" memory is host
// memory; streams run their work at enqueue time and advance a simulated
// clock, and events complete when that clock time has passed in real time
// (see stub_runtime.cpp).  Test infrastructure only.
#pragma once

#include <stddef.h>
#include <stdint.h>

#define __host__
#define __device__
#define __global__

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
} hipError_t;

typedef struct StubStream *hipStream_t;
typedef struct StubEvent *hipEvent_t;

typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 } hipMemcpyKind;
enum { hipStreamNonBlocking = 1, hipHostMallocDefault = 0 };

struct float2 { float x, y; };
struct double2 { double x, y; };
struct int2 { int x, y; };
struct int4 { int x, y, z, w; };

hipError_t hipMalloc(void **ptr, size_t bytes);
hipError_t hipFree(void *ptr);
hipError_t hipHostMalloc(void **ptr, size_t bytes, unsigned flags);
hipError_t hipHostFree(void *ptr);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetDevice(int *d);
hipError_t hipSetDevice(int d);
hipError_t hipGetLastError(void);
