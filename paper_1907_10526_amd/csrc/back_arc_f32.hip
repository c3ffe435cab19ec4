// Back projection kernels for the arc detector, FP32, and their quarter-turn and octant forms.
#include "back_launch.h"

FANPROJ_INSTANTIATE_BACK(float, FP_FAN_ARC)
FANPROJ_INSTANTIATE_BACK_QUARTER(FP_FAN_ARC)
FANPROJ_INSTANTIATE_BACK_OCTANT(FP_FAN_ARC)
