// Factorization kernels for complex128.
#include "factor_impl.hpp"

template void factor_kernels_init<double>();
template int launch_factor_layer<double>(const InstDesc<double>*, const Plan*, int, int, hipStream_t, hipEvent_t);
