// Back projection kernels for the parallel beams, FP32.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(float, FP_PARALLEL)
