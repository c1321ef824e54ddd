// Compiled sweep instantiations, list B (see sweep_impl.hpp).
#include "sweep_impl.hpp"

HSWEEP_SWEEP_LIST_B(HSWEEP_SWEEP_DEFINE)
