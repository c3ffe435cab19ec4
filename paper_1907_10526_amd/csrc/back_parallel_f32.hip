// Back projection kernels for the parallel beam, FP32, and their quarter-turn and octant forms.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(float, FP_PARALLEL)
FANPROJ_INSTANTIATE_BACK_QUARTER(FP_PARALLEL)
FANPROJ_INSTANTIATE_BACK_OCTANT(FP_PARALLEL)
