// Internal C++ entry points shared between the runtime's translation units.
#pragma once
#include <stddef.h>

#include <string>

#include "ppp.h"

namespace ppp {

// ppp_run on a single-problem handle without creating its timing events (no
// allocation of any kind on the way); PPP_E_OUT_OF_MEMORY with a message if the
// problem needs more than `bytes`.
ppp_status run_without_allocation(ppp_handle *h, void *ws, size_t bytes, void *stream);

// Sets the handle's last-error message (what ppp_last_error returns).
void set_error(ppp_handle *h, const std::string &msg);

// Workspace bytes of a single-problem handle for p (0 if p is invalid).
size_t workspace_bytes_for(const ppp_problem *p);

}  // namespace ppp
