// Rotation-accelerated M2L kernels, orders 14 (instantiation unit).
#include "m2l_rot_impl.h"

FMM_M2L_ROT_DEFINE(14)
