// Shared host-side helpers of the mgrav library (not part of the ABI).
#pragma once

#include <string>

#include "../../include/mgrav.h"

namespace mgrav_internal {

// Records `msg` as the calling thread's last host-side error (what
// mgrav_last_error(NULL) returns) and passes the status through.
mgrav_status set_host_error(mgrav_status s, const std::string& msg);

}  // namespace mgrav_internal
