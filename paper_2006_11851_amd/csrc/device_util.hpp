// Device helpers shared by the HIP sources (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

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

// (score, id) order: ties to the lower id
__device__ __forceinline__ bool lex_lt(float a, int ia, float b, int ib) { return a < b || (a == b && ia < ib); }

template <int K>
struct TopLex {
  float d[K];
  int i[K];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      d[t] = FLT_MAX;
      i[t] = INT_MAX;
    }
  }
  __device__ __forceinline__ void insert(float v, int id) {
    bool lt[K];
#pragma unroll
    for (int t = 0; t < K; ++t) lt[t] = lex_lt(v, id, d[t], i[t]);
#pragma unroll
    for (int t = K - 1; t > 0; --t) {
      d[t] = lt[t - 1] ? d[t - 1] : (lt[t] ? v : d[t]);
      i[t] = lt[t - 1] ? i[t - 1] : (lt[t] ? id : i[t]);
    }
    d[0] = lt[0] ? v : d[0];
    i[0] = lt[0] ? id : i[0];
  }
};
using Top8Lex = TopLex<8>;

}  // namespace pts
