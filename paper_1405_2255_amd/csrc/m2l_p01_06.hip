// Instantiation of the register-resident M2L kernel for expansion order(s) 1 2 3 4 5 6.
#include "m2l_impl.h"

FMM_M2L_FIXED_DEFINE(1)
FMM_M2L_FIXED_DEFINE(2)
FMM_M2L_FIXED_DEFINE(3)
FMM_M2L_FIXED_DEFINE(4)
FMM_M2L_FIXED_DEFINE(5)
FMM_M2L_FIXED_DEFINE(6)
