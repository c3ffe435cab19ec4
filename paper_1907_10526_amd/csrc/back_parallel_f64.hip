// Back projection kernels for the parallel beams, FP64.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(double, FP_PARALLEL)
