// Kernel instantiations of the single-instance launchers for rate matrices (FP32 and FP64).
#include "launchers.h"

using namespace otk;

OT_LAUNCHERS(, RatesSrc<float>)
OT_LAUNCHERS(, RatesSrc<double>)
