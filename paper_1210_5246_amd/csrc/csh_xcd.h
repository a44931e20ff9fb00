// XCD-aware workgroup numbering for gfx950.
#pragma once

#include <hip/hip_runtime.h>

namespace csh {

// Logical index of the calling workgroup, XCD-aware.  The MI355X deals the
// workgroups of a launch round-robin to its 8 XCDs (workgroup b to XCD b % 8),
// each XCD with its own L2; renumbered this way each XCD takes one contiguous
// range of logical workgroups, so tiles that share stencil rows run on the
// same L2 at the same time.  A bijection of [0, nb) for any nb.  The
// adjoint's one-thread-per-cell kernels run 10% faster with it, and the 3-D
// sweep reads 2.6x fewer bytes past L2 (3% slower); the 2-D row-marching
// sweep kernels measured 4-8% slower and keep the hardware order.
__host__ __device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    constexpr unsigned kXcds = 8;
    const unsigned x = b % kXcds, i = b / kXcds, per = nb / kXcds, rem = nb % kXcds;
    return x * per + (x < rem ? x : rem) + i;
}

}  // namespace csh
