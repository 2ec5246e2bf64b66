// Kernel instantiations of the single-instance launchers for dense cost matrices (FP32 and FP64).
#include "launchers.h"

using namespace otk;

OT_LAUNCHERS(, DenseSrc<float>)
OT_LAUNCHERS(, DenseSrc<double>)
