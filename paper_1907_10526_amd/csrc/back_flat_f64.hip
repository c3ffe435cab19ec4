// Back projection kernels for the flat detector, FP64.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(double, FP_FAN_FLAT)
