// validate.hpp -- host-side parameter checks of sim_create (validate.cpp).
#pragma once

#include <stddef.h>

#include "cuesim.h"

namespace cuesim {

// SIM_OK, or the status sim_create returns for *p with a message in msg[0..cap).
sim_status validate_params(const sim_params* p, char* msg, size_t cap);

}  // namespace cuesim
