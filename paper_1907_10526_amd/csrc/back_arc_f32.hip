// Back projection kernels for the arc detector, FP32.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(float, FP_FAN_ARC)
