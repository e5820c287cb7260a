// The thread-local error text of libsem, shared by the translation units that
// hold C-ABI entry points (defined in sem_api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace semk {

// Record the text sem_last_error() returns and return `code`; set_hip_error
// returns SEM_ERR_HIP with the HIP error string appended to `what`.
int set_error(int code, const std::string &msg);
int set_hip_error(hipError_t e, const char *what);

}  // namespace semk
