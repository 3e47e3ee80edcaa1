// Launchers of the BF16 search kernels (internal).
#pragma once

#include "kernels.hpp"

namespace pts {

#define PTS_DP_SWITCH(dp, ...)                                                                     \
  switch (dp) {                                                                                    \
    case 16: { constexpr int DPC = 16; __VA_ARGS__; } break;                                       \
    case 24: { constexpr int DPC = 24; __VA_ARGS__; } break;                                       \
    case 32: { constexpr int DPC = 32; __VA_ARGS__; } break;                                       \
    case 48: { constexpr int DPC = 48; __VA_ARGS__; } break;                                       \
    case 64: { constexpr int DPC = 64; __VA_ARGS__; } break;                                       \
    case 96: { constexpr int DPC = 96; __VA_ARGS__; } break;                                       \
    case 128: { constexpr int DPC = 128; __VA_ARGS__; } break;                                     \
    default: ::pts::fail(PTS_ERR_UNSUPPORTED, "padded PCA width must be 16/24/32/48/64/96/128");   \
  }

// The rows the exact BF16 scan collects per (query, leaf) pair and half-wave:
// hits [pairs][2][hs] (score bits, leaf position), hit_cnt [pairs][2]; a
// query's K smallest (score, position) keys among them are the exact BF16
// top-K over its scanned rows.
struct ScanHits {
  const int2* hits = nullptr;
  const int32_t* hit_cnt = nullptr;
  const int32_t* pair_leaf = nullptr;
  int P = 0, hs = 0;
};
// number of exemplar splits for the brute-force top-k kernel
int brute_splits(int64_t nq);
// partial top-kt (score, leaf position) per (split, query), kt = 8 or 16:
// part [S][nq][kt]; tau_q (optional, [nq]): a bound on each query's kt-th
// smallest key, scores above it skipped (its rows cannot be among them)
void launch_brute_bf16_topk(Ctx* c, const uint16_t* Qb, int64_t nq, const uint16_t* Zb, const float* zbn, int64_t N,
                            int dk, int S, int kt, const uint64_t* tau_q, float* part_d, int32_t* part_i);
// merge S partial lists per query (list s of query q = row q*qs + s*ss of
// part [..][list_len]; lists with valid[row] < 0 skipped), re-rank the best k
// in FP32 PCA space; nn = exemplar id.  cand_out (optional) [nq][8]: the k
// candidates as exemplar ids (-1 beyond k).  sh non-null: the candidates are
// the k smallest keys of the collected rows instead.
void launch_merge_rerank_pca(Ctx* c, const float* part_d, const int32_t* part_i, int64_t nq, int S, int64_t qs,
                             int64_t ss, const int32_t* valid, const ScanHits* sh, int k, const float* Qp, int dp,
                             const float* Zp, const float* zres, const int32_t* perm, int64_t N, int32_t* cand_out,
                             int32_t* nn, int list_len = 0);
// pairs per tile of the leaf scan (the bucketing chunk)
int leaf_scan_bf16_chunk();
// sum of the leaf sizes over the pairs with pair_leaf >= 0 (synchronous)
int64_t count_scan_rows(Ctx* c, const int32_t* pair_leaf, int64_t n, const int32_t* leaf_off);
// Exact BF16 top-K (K = 8 or 16) of every query over the members of its
// bucketed leaves (pair_leaf [nq*P], P <= 16, negative = not scanned; a
// "leaf" is any row range of leaf_off: a tree leaf, or a split of the whole
// exemplar set), in two passes.  Bound: every pair's 16 class minima; the
// K-th smallest over the query's pairs bounds its K-th key from above (tau);
// pairs that cannot hold a row within tau get pair_leaf2 = -1, the others
// their leaf.  Collect (over the pairs bucketed from pair_leaf2): the rows
// within tau, hc slots per pair and half (0..14); queries with more rows go
// to a per-query pass.  n_overflow: device int32, the number of such queries.
void launch_leaf_scan_bf16_bound(Ctx* c, const uint16_t* Qb, int64_t nq, int P, const uint16_t* Zb, const float* zbn,
                                 int dk, const int32_t* leaf_off, const BucketBufs& b, int max_tiles,
                                 const int32_t* pair_leaf, int32_t* pair_leaf2, int K);
void launch_leaf_scan_bf16_collect(Ctx* c, const uint16_t* Qb, int64_t nq, int P, const uint16_t* Zb,
                                   const float* zbn, int dk, const int32_t* leaf_off, const BucketBufs& b,
                                   int max_tiles, const int32_t* pair_leaf2, int hc, ScanHits* sh,
                                   int32_t* n_overflow, int K);
// pair_leaf[i] = i % S for i < n: every query scans every one of S splits
void launch_fill_splits(Ctx* c, int32_t* pair_leaf, int64_t n, int S);
// off [S + 1]: the row ranges of S equal splits of N rows (the last shorter)
void launch_split_offsets(Ctx* c, int32_t* off, int S, int64_t N);
// Class-minimum candidates of the learned form's BF16 scan in one pass:
// per pair (the pair_leaf layout: P per query), its 16 class minima as
// (score, leaf position) in part_d / part_i [nq * P][16] (classes: rows i
// and i + 16 of every 32-row tile, i < 16; each keeps its smallest score and
// the row of its first occurrence; a class with no row: FLT_MAX, INT_MAX).
void launch_leaf_scan_bf16_class(Ctx* c, const uint16_t* Qb, int64_t nq, int P, const uint16_t* Zb, const float* zbn,
                                 int dk, const int32_t* leaf_off, const BucketBufs& b, int max_tiles, float* part_d,
                                 int32_t* part_i);
// merge S partial lists per query as above and re-rank the best k by the
// full-D FP32 distance gathered from the images x [H][W][4] and ex
// [Hz][Wz][4] (read from its 8-bit form ex_pk / ex_srow when given: the same
// values); nn = exemplar id, dist (optional) = its full-D distance.
// list_len: entries per list (8 or 16; 0: 8 for k <= 8, else 16)
void launch_select_rerank_full(Ctx* c, const float* part_d, const int32_t* part_i, int64_t nq, int S, int64_t qs,
                               int64_t ss, const int32_t* valid, const ScanHits* sh, int k, const int32_t* perm,
                               int64_t npos,
                               const float* x, int H, int W, int w, int s, const float* ex, const uint32_t* ex_pk,
                               const float* ex_srow, int Hz, int Wz, int32_t* nn, float* dist, int list_len = 0);

}  // namespace pts
