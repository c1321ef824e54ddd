// Host stand-in of the HIP runtime that runs one-wavefront kernels: the
// host-check API (allocations are host memory), plus a launch that runs the
// threads of each block concurrently, one OS thread per lane, with a block
// barrier, a shared-memory qualifier and the cross-lane shuffles built on
// it.  Every lane must reach every barrier and shuffle, as on the device.
#pragma once
#include "../../hostcheck/hip/hip_runtime.h"
#include <math.h>
#include <pthread.h>
#include <string.h>
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

using std::isnan;
using std::max;
using std::min;

#define __shared__ static
#define __launch_bounds__(x)
// dynamic shared memory: one buffer of the launch's requested size
extern std::vector<char> wave_dyn_shared;
#define HIP_DYNAMIC_SHARED(type, var) type* var = (type*)wave_dyn_shared.data();

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_index {
    unsigned x, y, z;
};
extern thread_local emu_index blockIdx, threadIdx;
extern thread_local dim3 blockDim, gridDim;
extern pthread_barrier_t wave_barrier;
extern unsigned long long wave_slot[1024];

inline void __syncthreads() { pthread_barrier_wait(&wave_barrier); }

template <typename T> inline T wave_exchange(T v, int src) {
    static_assert(sizeof(T) <= sizeof(unsigned long long), "shuffle of a wide type");
    memcpy(&wave_slot[threadIdx.x], &v, sizeof(T));
    __syncthreads();
    T r;
    memcpy(&r, &wave_slot[src & 63], sizeof(T));
    __syncthreads();
    return r;
}
template <typename T> inline T __shfl_xor(T v, int mask, int = 64) { return wave_exchange(v, (int)threadIdx.x ^ mask); }
template <typename T> inline T __shfl(T v, int src, int = 64) { return wave_exchange(v, src); }

template <typename K, typename... A>
inline void wave_launch(K kernel, dim3 g, dim3 b, size_t shared_bytes, A... args) {
    const unsigned nt = b.x * b.y * b.z;
    // NaN bytes, as the device allocations of the stand-in start
    wave_dyn_shared.assign(shared_bytes ? shared_bytes : 1, (char)0xFF);
    for (unsigned bz = 0; bz < g.z; ++bz)
        for (unsigned by = 0; by < g.y; ++by)
            for (unsigned bx = 0; bx < g.x; ++bx) {
                pthread_barrier_init(&wave_barrier, nullptr, nt);
                std::vector<std::thread> th;
                for (unsigned t = 0; t < nt; ++t)
                    th.emplace_back([=] {
                        gridDim = g;
                        blockDim = b;
                        blockIdx = {bx, by, bz};
                        threadIdx = {t % b.x, (t / b.x) % b.y, t / (b.x * b.y)};
                        kernel(args...);
                    });
                for (auto& x : th) x.join();
                pthread_barrier_destroy(&wave_barrier);
            }
}
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) wave_launch(k, dim3(g), dim3(b), (size_t)(sh), __VA_ARGS__)
