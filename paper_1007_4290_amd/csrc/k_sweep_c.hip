// Compiled sweep instantiations, list C (see sweep_impl.hpp).
#include "sweep_impl.hpp"

HSWEEP_SWEEP_LIST_C(HSWEEP_SWEEP_DEFINE)
