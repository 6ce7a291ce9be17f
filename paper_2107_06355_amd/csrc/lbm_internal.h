// Internal declarations shared by the host sources of liblbm.so (not part of the C ABI).
#pragma once

#include "lbm.h"

// thread-local message returned by lbm_last_error()
void lbm_set_error(const char* msg);
