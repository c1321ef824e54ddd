// Host-memory stand-in of the HIP runtime calls the library's host code
// makes: device allocations are host allocations kept in a registry, so
// launch checks can test that a range lies inside a live allocation.
#include <hip/hip_runtime.h>
#include <map>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
static std::map<uintptr_t, size_t> g_alloc;
void fake_describe(const void* p) {
    uintptr_t a = (uintptr_t)p;
    auto it = g_alloc.upper_bound(a);
    if (it == g_alloc.begin()) { fprintf(stderr, "  no allocation below %p\n", p); return; }
    --it;
    fprintf(stderr, "  nearest allocation %p size %zu (offset %zd)\n", (void*)it->first, it->second, (ssize_t)(a - it->first));
}
bool fake_in_alloc(const void* p, size_t bytes) {
    uintptr_t a = (uintptr_t)p;
    auto it = g_alloc.upper_bound(a);
    if (it == g_alloc.begin()) return false;
    --it;
    return a >= it->first && a + bytes <= it->first + it->second;
}
// Device allocations start as NaN bytes when set (a GPU leaves them
// uninitialized), zeros otherwise.
bool fake_poison = false;
hipError_t hipMalloc(void** p, size_t b) {
    *p = calloc(1, b ? b : 1);
    if (fake_poison) memset(*p, 0xff, b);
    g_alloc[(uintptr_t)*p] = b;
    return 0;
}
hipError_t hipFree(void* p) { g_alloc.erase((uintptr_t)p); free(p); return 0; }
hipError_t hipHostMalloc(void** p, size_t b, unsigned) { *p = calloc(1, b ? b : 1); return 0; }
hipError_t hipHostFree(void* p) { free(p); return 0; }
static void chk(const void* p, size_t b, const char* what) {
    if (b && !fake_in_alloc(p, b)) { fprintf(stderr, "BAD %s %p %zu\n", what, p, b); abort(); }
}
hipError_t hipMemcpy(void* d, const void* s, size_t b, hipMemcpyKind k) {
    if (k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice) chk(d, b, "memcpy dst");
    if (k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice) chk(s, b, "memcpy src");
    memcpy(d, s, b); return 0;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t b, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, b, k); }
hipError_t hipMemsetAsync(void* d, int v, size_t b, hipStream_t) { chk(d, b, "memset"); memset(d, v, b); return 0; }
hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
hipError_t hipDeviceSynchronize() { return 0; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)malloc(8); return 0; }
hipError_t hipEventDestroy(hipEvent_t e) { free(e); return 0; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return 0; }
hipError_t hipEventSynchronize(hipEvent_t) { return 0; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return 0; }
hipError_t hipGetLastError() { return 0; }
const char* hipGetErrorString(hipError_t) { return "fake"; }
hipError_t hipSetDevice(int) { return 0; }
hipError_t hipGetDevice(int* d) { *d = 0; return 0; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return 0; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) { a->type = fake_in_alloc(p, 1) ? hipMemoryTypeDevice : hipMemoryTypeHost; return 0; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = (void*)sym; g_alloc[(uintptr_t)sym] = 32u << 20; return 0; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)malloc(8); return 0; }
hipError_t hipStreamDestroy(hipStream_t s) { free(s); return 0; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return 0; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)malloc(8); return 0; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, void*, size_t) { *e = (hipGraphExec_t)malloc(8); return 0; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return 0; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); return 0; }
hipError_t hipGraphDestroy(hipGraph_t g) { free(g); return 0; }
