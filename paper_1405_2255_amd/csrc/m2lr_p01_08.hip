// Rotation-accelerated M2L kernels, orders 1 2 3 4 5 6 7 8 (instantiation unit).
#include "m2l_rot_impl.h"

FMM_M2L_ROT_DEFINE(1)
FMM_M2L_ROT_DEFINE(2)
FMM_M2L_ROT_DEFINE(3)
FMM_M2L_ROT_DEFINE(4)
FMM_M2L_ROT_DEFINE(5)
FMM_M2L_ROT_DEFINE(6)
FMM_M2L_ROT_DEFINE(7)
FMM_M2L_ROT_DEFINE(8)
