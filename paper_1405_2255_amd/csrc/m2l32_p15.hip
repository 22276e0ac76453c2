// Instantiation of the mixed-precision M2L kernel for expansion order 15.
#include "m2l32_impl.h"

FMM_M2L32_FIXED_DEFINE(15)
