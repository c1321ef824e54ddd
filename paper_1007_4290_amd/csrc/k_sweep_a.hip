// Compiled sweep instantiations, list A (see sweep_impl.hpp).
#include "sweep_impl.hpp"

HSWEEP_SWEEP_LIST_A(HSWEEP_SWEEP_DEFINE)
