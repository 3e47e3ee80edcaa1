// The accelerated search forms: BF16 brute force and the learned leaf
// proposal, each ending in an FP32 re-rank.
#include "bf16_learned.hpp"
#include "kernels_bf16.hpp"
#include "kernels_mlp.hpp"

namespace pts {

bool search_brute_bf16(Ctx* c, ExView ex, const Index& ix, const float* x, int H, int W, const pts_estep_params& p,
                       const float* qp, const uint16_t* qb, int64_t nq, int32_t* nn, float* dist,
                       int32_t** scan_overflows, int64_t* work) {
  const int k = p.topk <= 0 ? 8 : p.topk;
  PTS_REQUIRE(k >= 1 && k <= 16, PTS_ERR_ARG, "topk must be 1..16");
  const int kt = k <= 8 ? 8 : 16;  // the exact BF16 top-kt, of which the best k are re-ranked
  const int64_t N = ix.N;
  PTS_REQUIRE(N > 0 && N < INT_MAX, PTS_ERR_ARG, "brute: bad N");
  if (scan_overflows) *scan_overflows = nullptr;
  const float* zbn = p.residual ? ix.zbnorm_res.as<float>() : ix.zbnorm.as<float>();
  const float* zres = p.residual ? ix.zres.as<float>() : nullptr;
  // Pass 1, the bound: the exemplar rows (leaf order) in S contiguous splits
  // of at least 8192 rows, at most 16, every query scanning every split as it
  // would the leaves proposed to it; the kt-th smallest of a query's class
  // minima over all splits bounds its kt-th smallest key from above.
  const int S = (int)std::min<int64_t>(16, std::max<int64_t>(1, N / 8192));
  int32_t* soff = c->buf<int32_t>("bb_split_off", (size_t)S + 1);
  launch_split_offsets(c, soff, S, N);
  const int64_t npairs = nq * S;
  int32_t* pair_leaf = c->buf<int32_t>("bb_pair_leaf", (size_t)std::max<int64_t>(1, npairs));
  int32_t* pair_leaf2 = c->buf<int32_t>("bb_pair_leaf2", (size_t)std::max<int64_t>(1, npairs));
  launch_fill_splits(c, pair_leaf, npairs, S);
  const int chunk = leaf_scan_bf16_chunk();
  int max_tiles = 0;
  BucketBufs b = bucket_buffers(c, npairs, S, chunk, &max_tiles, "bbk");
  launch_bucket(c, pair_leaf, npairs, S, chunk, b);
  launch_leaf_scan_bf16_bound(c, qb, nq, S, ix.zbf.as<uint16_t>(), zbn, ix.dk, soff, b, max_tiles, pair_leaf,
                              pair_leaf2, kt);
  const uint64_t* tau = c->buf<uint64_t>("ls_tau_q", (size_t)std::max<int64_t>(1, nq));
  if (work) work[0] = count_scan_rows(c, pair_leaf, npairs, soff);
  // Pass 2: every (query, exemplar) score again, only those within the bound
  // entering each lane's sorted top-kt (rare once the bound is known)
  const int S2 = brute_splits(nq);
  float* pd = c->buf<float>("bb_pd", (size_t)S2 * nq * kt);
  int32_t* pi = c->buf<int32_t>("bb_pi", (size_t)S2 * nq * kt);
  launch_brute_bf16_topk(c, qb, nq, ix.zbf.as<uint16_t>(), zbn, N, ix.dk, S2, kt, tau, pd, pi);
  if (work) work[1] = work[0];
  if (p.rerank_full) {
    launch_select_rerank_full(c, pd, pi, nq, S2, 1, nq, nullptr, nullptr, k, ix.perm.as<int32_t>(), N, x, H, W, ix.w,
                              p.stride, ex.img, ex.pk, ex.srow, ex.Hz, ex.Wz, nn, dist);
    return dist != nullptr;
  }
  launch_merge_rerank_pca(c, pd, pi, nq, S2, 1, nq, nullptr, nullptr, k, qp, ix.dp, ix.zproj.as<float>(), zres,
                          ix.perm.as<int32_t>(), N, nullptr, nn);
  return false;
}

int64_t search_learned(Ctx* c, ExView ex, const Index& ix, const float* x, int H, int W, const pts_estep_params& p,
                       const float* qp, const uint16_t* qb, int64_t nq, int32_t* nn, float* dist, bool* dist_done,
                       bool bf16_scan, bool class_candidates, bool count_fallbacks, int32_t** scan_overflows,
                       int64_t* work) {
  *dist_done = false;
  if (scan_overflows) *scan_overflows = nullptr;
  const int P = p.n_proposals <= 0 ? 4 : p.n_proposals;
  PTS_REQUIRE(P >= 1 && P <= 8 && P <= ix.tree.n_leaves(), PTS_ERR_ARG, "n_proposals must be 1..8 (and <= leaves)");
  const int L = ix.tree.n_leaves();
  // proposals and softmax margins
  int32_t* prop = c->buf<int32_t>("ln_prop", (size_t)nq * P);
  float* margin = c->buf<float>("ln_margin", (size_t)nq);
  mlp_propose_rows(c, qp, ix.dp, nq, P, prop, margin);
  // the tree's own leaf, needed only where the margin is low
  int32_t* dleaf = c->buf<int32_t>("ln_dleaf", (size_t)nq);
  int32_t* lowq = c->buf<int32_t>("ln_lowq", (size_t)nq);
  int32_t* nlow = c->buf<int32_t>("ln_nlow", 1);
  launch_zero_i32(c, nlow, 1);
  launch_descend_low_margin(c, qp, nq, ix.dp, margin, p.margin, ix.cent.as<float>(), ix.first_child.as<int32_t>(),
                            ix.n_children.as<int32_t>(), ix.leaf_of_node.as<int32_t>(), ix.tree.n_nodes(), lowq, nlow,
                            dleaf);
  const int P1 = P + 1;  // proposals + the tree's leaf for low-margin queries
  int32_t* pair_leaf = c->buf<int32_t>("ln_pair_leaf", (size_t)nq * P1);
  // the fallback count (one atomic per wave) only when statistics are asked for
  int32_t* fb = count_fallbacks ? c->buf<int32_t>("ln_fallbacks", 1) : nullptr;
  if (fb) launch_zero_i32(c, fb, 1);
  launch_learned_pairs(c, prop, margin, dleaf, nq, P, p.margin, L, pair_leaf, fb);
  const int chunk = bf16_scan ? leaf_scan_bf16_chunk() : leaf_scan_f32_chunk(ix.dp);
  int max_tiles = 0;
  BucketBufs b = bucket_buffers(c, nq * P1, L, chunk, &max_tiles);
  b.tile_order = ix.leaf_by_rows.as<int32_t>();
  launch_bucket(c, pair_leaf, nq * P1, L, chunk, b);
  if (!bf16_scan && p.rerank_full) {
    // the exact FP32 top-k over the members of the scanned leaves (PCA space),
    // re-ranked by the full-dimension FP32 distance
    const int k = p.topk <= 0 ? 8 : p.topk;
    PTS_REQUIRE(k >= 1 && k <= 8, PTS_ERR_ARG, "topk must be 1..8");
    float* pdd = c->buf<float>("ln_pair_cd", (size_t)nq * P1 * 8);
    int32_t* pii = c->buf<int32_t>("ln_pair_ci", (size_t)nq * P1 * 8);
    launch_leaf_scan_f32(c, qp, ix.dp, ix.zproj.as<float>(), ix.perm.as<int32_t>(), ix.leaf_off.as<int32_t>(), b,
                         max_tiles, P1, p.residual ? ix.zres.as<float>() : nullptr, nullptr, nullptr, pdd, pii);
    launch_select_rerank_full(c, pdd, pii, nq, P1, P1, 1, pair_leaf, nullptr, k, ix.perm.as<int32_t>(), ix.N, x, H, W,
                              ix.w, p.stride, ex.img, ex.pk, ex.srow, ex.Hz, ex.Wz, nn, dist);
    *dist_done = dist != nullptr;
    if (work) work[0] = count_scan_rows(c, pair_leaf, nq * P1, ix.leaf_off.as<int32_t>());
  } else if (!bf16_scan) {
    int32_t* pid = c->buf<int32_t>("ln_pair_id", (size_t)nq * P1);
    float* pdd = c->buf<float>("ln_pair_d", (size_t)nq * P1);
    launch_leaf_scan_f32(c, qp, ix.dp, ix.zproj.as<float>(), ix.perm.as<int32_t>(), ix.leaf_off.as<int32_t>(), b,
                         max_tiles, P1, p.residual ? ix.zres.as<float>() : nullptr, pid, pdd);
    launch_merge_pairs_f32(c, pair_leaf, pid, pdd, nq, P1, nn);
    if (work) work[0] = count_scan_rows(c, pair_leaf, nq * P1, ix.leaf_off.as<int32_t>());
  } else if (class_candidates) {
    // one BF16 pass: the query's k smallest class minima over its pairs (16
    // per pair) as candidates, re-ranked as below
    PTS_REQUIRE(ix.has_bf16 && qb, PTS_ERR_STATE, "LEARNED_BF16_CLASS needs an index built with make_bf16");
    const int k = p.topk <= 0 ? 8 : p.topk;
    PTS_REQUIRE(k >= 1 && k <= 16, PTS_ERR_ARG, "topk must be 1..16");
    const float* zbn = p.residual ? ix.zbnorm_res.as<float>() : ix.zbnorm.as<float>();
    float* pdd = c->buf<float>("ln_pair_cd16", (size_t)nq * P1 * 16);
    int32_t* pii = c->buf<int32_t>("ln_pair_ci16", (size_t)nq * P1 * 16);
    launch_leaf_scan_bf16_class(c, qb, nq, P1, ix.zbf.as<uint16_t>(), zbn, ix.dk, ix.leaf_off.as<int32_t>(), b,
                                max_tiles, pdd, pii);
    if (p.rerank_full) {
      launch_select_rerank_full(c, pdd, pii, nq, P1, P1, 1, pair_leaf, nullptr, k, ix.perm.as<int32_t>(), ix.N, x, H,
                                W, ix.w, p.stride, ex.img, ex.pk, ex.srow, ex.Hz, ex.Wz, nn, dist, 16);
      *dist_done = dist != nullptr;
    } else {
      launch_merge_rerank_pca(c, pdd, pii, nq, P1, P1, 1, pair_leaf, nullptr, k, qp, ix.dp, ix.zproj.as<float>(),
                              p.residual ? ix.zres.as<float>() : nullptr, ix.perm.as<int32_t>(), ix.N, nullptr, nn, 16);
    }
    if (work) work[0] = count_scan_rows(c, pair_leaf, nq * P1, ix.leaf_off.as<int32_t>());
  } else {
    PTS_REQUIRE(ix.has_bf16 && qb, PTS_ERR_STATE, "LEARNED_BF16 needs an index built with make_bf16");
    const int k = p.topk <= 0 ? 8 : p.topk;
    PTS_REQUIRE(k >= 1 && k <= 8, PTS_ERR_ARG, "topk must be 1..8");
    const float* zbn = p.residual ? ix.zbnorm_res.as<float>() : ix.zbnorm.as<float>();
    const float* zres = p.residual ? ix.zres.as<float>() : nullptr;
    const int hc = p.scan_slots <= 0 ? 14 : p.scan_slots;
    ScanHits sh;
    int32_t* novf = c->buf<int32_t>("ln_scan_overflow", 1);
    // bound pass over every pair, then the collect pass over the pairs that
    // can hold a row within the query's bound (bucketed again)
    int32_t* pair_leaf2 = c->buf<int32_t>("ln_pair_leaf2", (size_t)nq * P1);
    launch_leaf_scan_bf16_bound(c, qb, nq, P1, ix.zbf.as<uint16_t>(), zbn, ix.dk, ix.leaf_off.as<int32_t>(), b,
                                max_tiles, pair_leaf, pair_leaf2, 8);
    int max_tiles2 = 0;
    BucketBufs b2 = bucket_buffers(c, nq * P1, L, chunk, &max_tiles2, "bk2");
    b2.tile_order = ix.leaf_by_rows.as<int32_t>();
    launch_bucket(c, pair_leaf2, nq * P1, L, chunk, b2);
    launch_leaf_scan_bf16_collect(c, qb, nq, P1, ix.zbf.as<uint16_t>(), zbn, ix.dk, ix.leaf_off.as<int32_t>(), b2,
                                  max_tiles2, pair_leaf2, hc, &sh, novf, 8);
    if (work) {
      work[0] = count_scan_rows(c, pair_leaf, nq * P1, ix.leaf_off.as<int32_t>());
      work[1] = count_scan_rows(c, pair_leaf2, nq * P1, ix.leaf_off.as<int32_t>());
    }
    if (scan_overflows) *scan_overflows = novf;
    if (p.rerank_full) {
      launch_select_rerank_full(c, nullptr, nullptr, nq, 0, 0, 0, nullptr, &sh, k, ix.perm.as<int32_t>(), ix.N, x, H,
                                W, ix.w, p.stride, ex.img, ex.pk, ex.srow, ex.Hz, ex.Wz, nn, dist);
      *dist_done = dist != nullptr;
    } else {
      launch_merge_rerank_pca(c, nullptr, nullptr, nq, 0, 0, 0, nullptr, &sh, k, qp, ix.dp, ix.zproj.as<float>(),
                              zres, ix.perm.as<int32_t>(), ix.N, nullptr, nn);
    }
  }
  int32_t fbh = 0;
  if (count_fallbacks) {
    PTS_HIP(hipMemcpyAsync(&fbh, fb, 4, hipMemcpyDeviceToHost, c->stream));
    PTS_HIP(hipStreamSynchronize(c->stream));
  }
  return fbh;
}

}  // namespace pts

