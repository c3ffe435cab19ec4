// Back projection kernels for the flat detector, FP32.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(float, FP_FAN_FLAT)
