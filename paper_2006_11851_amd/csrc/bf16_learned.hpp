// The two accelerated search forms (internal): BF16 brute force with top-k
// and FP32 re-rank; MLP leaf proposal with fallback to the tree.
#pragma once

#include "api_internal.hpp"

namespace pts {

// nn[q] for projected queries qp [nq][ix.dp] (qb: their bf16(-2 q') [nq][ix.dk]).  When the form re-ranks in full
// dimension it also writes the winner distance to dist (if non-null) and
// returns true; otherwise the caller computes it.  *scan_overflows and work
// as for search_learned below (its exact BF16 scan over the exemplar splits).
bool search_brute_bf16(Ctx* c, ExView ex, const Index& ix, const float* x, int H, int W, const pts_estep_params& p,
                       const float* qp, const uint16_t* qb, int64_t nq, int32_t* nn, float* dist,
                       int32_t** scan_overflows, int64_t* work);
// returns the number of queries that fell back to the tree; *dist_done as
// the return value above; *scan_overflows (if non-null) receives the device
// counter of queries the BF16 scan sent to its per-query pass (null if none ran);
// work (if non-null): [0] = scores of the leaf scan (BF16: its bound pass),
// [1] = scores of the BF16 collect pass (synchronises).  class_candidates
// (with bf16_scan): class-minimum candidates from one pass instead of the
// exact BF16 top-8
int64_t search_learned(Ctx* c, ExView ex, const Index& ix, const float* x, int H, int W, const pts_estep_params& p,
                       const float* qp, const uint16_t* qb, int64_t nq, int32_t* nn, float* dist, bool* dist_done,
                       bool bf16_scan, bool class_candidates, bool count_fallbacks, int32_t** scan_overflows,
                       int64_t* work);

}  // namespace pts
