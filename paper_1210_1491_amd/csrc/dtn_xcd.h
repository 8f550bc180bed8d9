// XCD-aware order of a traversal's work items (the treecode's target
// groups).  Workgroups are dispatched to the 8 XCDs round-robin (workgroup i
// to XCD i mod 8), each with its own L2; neighbouring items share data
// across a whole eighth of the range, so each XCD takes one contiguous
// eighth, in order.
#pragma once

#include <cstdint>

#include "dtn_device.h"

namespace dtn {

// n items (a multiple of kXcds * W) in blocks of W waves: block ib (XCD
// ib mod 8) and its wave wv take item (ib mod 8) n/8 + (ib / 8) W + wv, so
// XCD x works through [x n/8, (x + 1) n/8) in order.
__host__ __device__ __forceinline__ int64_t xcd_contiguous(int64_t ib, int wv, int64_t n, int W)
{
    return (ib % kXcds) * (n / kXcds) + (ib / kXcds) * W + wv;
}

}  // namespace dtn
