// Device helpers shared by the HIP sources (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace pts {

// XCD-aware block order.  The chip's 8 XCDs (each with its own L2) receive
// the blocks of a launch round-robin: hardware block b runs on XCD b % 8.
// Returning b % 8 * (G / 8) + b / 8 (with the remainder spread over the first
// XCDs) gives each XCD one contiguous range of logical blocks, so
// neighbouring work items - which read overlapping image windows or the same
// leaf rows - share an L2.  A bijection on [0, G).
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

}  // namespace pts
