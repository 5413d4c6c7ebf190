// Internal C++ entry points shared between the runtime's translation units.
#pragma once
#include <stddef.h>

#include <string>

#include "ppp.h"

namespace ppp {

// Workspace bytes of a single-problem handle for p (0 if p is invalid).
size_t workspace_bytes_for(const ppp_problem *p);

}  // namespace ppp
