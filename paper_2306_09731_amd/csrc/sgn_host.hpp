// Host-side helpers shared by the C-ABI sources of libsgn.
#pragma once
#include "sgn.h"
#include "sgn_internal.hpp"

namespace sgn {

// Validates a configuration: SGN_OK, SGN_ERR_INVALID_ARG or SGN_ERR_UNSUPPORTED.
int check_config(const sgn_config* c);
// Geometry, spectral constants and launch shapes of a valid configuration;
// the twiddle-table pointers are left null for the caller to set.
void geom_init(const sgn_config& c, Geom& g);
// Message reported by sgn_last_error(NULL) for calls that take no context.
void set_global_error(const char* msg);
const char* global_error();

}  // namespace sgn
