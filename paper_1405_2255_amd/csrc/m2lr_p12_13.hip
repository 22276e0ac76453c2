// Rotation-accelerated M2L kernels, orders 12 13 (instantiation unit).
#include "m2l_rot_impl.h"

FMM_M2L_ROT_DEFINE(12)
FMM_M2L_ROT_DEFINE(13)
