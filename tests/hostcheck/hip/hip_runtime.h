// Minimal host-only stand-in for the HIP runtime API used by api.hip, for a
// CPU check of the host logic (allocations are host memory).
#pragma once
#include <stddef.h>
#include <stdint.h>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __align__(x) alignas(x)
#define HIP_SYMBOL(x) (&(x))
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph_t* hipGraph_t;
typedef struct ihipGraphExec_t* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipMemoryType { hipMemoryTypeHost, hipMemoryTypeDevice, hipMemoryTypeManaged };
struct hipPointerAttribute_t { int type; };
enum { hipHostMallocDefault = 0, hipStreamNonBlocking = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal };
hipError_t hipMalloc(void** p, size_t b);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t b, unsigned f);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t b, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t b, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void* d, int v, size_t b, hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned f);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
// registry query used by the launch checks
bool fake_in_alloc(const void* p, size_t bytes);
extern bool fake_poison;
