// Kernel instantiations of the single-instance launchers for costs regenerated from positions (rates of the downlink model, distances).
#include "launchers.h"

using namespace otk;

OT_LAUNCHERS(, GeoSrc)
OT_LAUNCHERS(, EuclidSrc)
