// Error handling shared by the host-side translation units of libdmrg.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "../../include/dmrg.h"

namespace dmrg {

// Thrown inside the library, caught at the C-ABI boundary and turned into a status code.
struct Error : std::runtime_error {
    dmrg_status code;
    Error(dmrg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Stores e's message as the thread's dmrg_last_error() and returns its code.
dmrg_status record_error(const Error& e);
void clear_error();
// The calling thread's last-error message (what dmrg_last_error returns), writable.
std::string& last_error();
double now_seconds();

}  // namespace dmrg

#define HIPCHK(x)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess)                                                                          \
            throw ::dmrg::Error(DMRG_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));     \
    } while (0)
