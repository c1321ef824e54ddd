// Compiled sweep instantiations for groups of 4 right-hand sides (see sweep_impl.hpp).
#include "sweep_impl.hpp"

HSWEEP_SWEEP_LIST_G4(HSWEEP_SWEEP_DEFINE4)
