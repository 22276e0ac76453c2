// Instantiation of the mixed-precision M2L kernel for expansion orders 9 and 10.
#include "m2l32_impl.h"

FMM_M2L32_FIXED_DEFINE(9)
FMM_M2L32_FIXED_DEFINE(10)
