// Instantiation of the register-resident M2L kernel for expansion order(s) 14.
#include "m2l_impl.h"

FMM_M2L_FIXED_DEFINE(14)
