// Internal declarations shared by the host sources of liblbm.so (not part of the C ABI).
#pragma once

#include "lbm.h"

// thread-local message returned by lbm_last_error()
void lbm_set_error(const char* msg);

// d(b1, a1^2)/d(rho_max, p_max) -> J1, d(b3, a3^2)/d(rho_min, p_min) -> J3 (rows b, a^2)
void lbm_knot_jacobians(const lbm_eos* e, double J1[2][2], double J3[2][2]);
