// Block and thread indices of the emulated kernel launch.
#include <hip/hip_runtime.h>

thread_local emu_index blockIdx, threadIdx;
thread_local dim3 blockDim, gridDim;
