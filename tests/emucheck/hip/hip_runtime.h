// Host-only stand-in for the HIP runtime that also runs kernels: the API of
// the host-check stand-in, plus a launch that calls the kernel function once
// per (block, thread) index in order.  Only kernels without shared memory,
// barriers or cross-lane operations are meaningful under it.
#pragma once
#include "../../hostcheck/hip/hip_runtime.h"
#include <math.h>

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_index {
    unsigned x, y, z;
};
extern thread_local emu_index blockIdx, threadIdx;
extern thread_local dim3 blockDim, gridDim;

template <typename K, typename... A>
inline void emu_launch(K kernel, dim3 g, dim3 b, A... args) {
    gridDim = g;
    blockDim = b;
    for (unsigned bz = 0; bz < g.z; ++bz)
        for (unsigned by = 0; by < g.y; ++by)
            for (unsigned bx = 0; bx < g.x; ++bx)
                for (unsigned tz = 0; tz < b.z; ++tz)
                    for (unsigned ty = 0; ty < b.y; ++ty)
                        for (unsigned tx = 0; tx < b.x; ++tx) {
                            blockIdx = {bx, by, bz};
                            threadIdx = {tx, ty, tz};
                            kernel(args...);
                        }
}
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) emu_launch(k, dim3(g), dim3(b), __VA_ARGS__)
