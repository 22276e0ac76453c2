// Rotation-accelerated M2L kernels, orders 9 10 11 (instantiation unit).
#include "m2l_rot_impl.h"

FMM_M2L_ROT_DEFINE(9)
FMM_M2L_ROT_DEFINE(10)
FMM_M2L_ROT_DEFINE(11)
