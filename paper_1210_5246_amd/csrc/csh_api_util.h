// Error plumbing shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <string>

#include "cshydro.h"

// record a message for csh_last_error() and return code
int csh_fail(int code, const std::string& msg);

#define CSH_HIP(call)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return csh_fail(CSH_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// geometry the adjoint needs, copied out of the grid handle
struct csh_grid_view {
    int nx, ny, bcx, bcy;
    double dx, dy;
    double vc, rc, x0, y0;
};
