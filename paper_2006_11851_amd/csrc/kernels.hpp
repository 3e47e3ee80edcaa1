// Launchers of the gfx950 kernels (internal).  Every launcher enqueues on
// ctx->stream and brackets itself for profiling.
#pragma once

#include "common.hpp"

namespace pts {

// ---- images (k_image.hip)
void launch_rgbs_from_u8(Ctx* c, const uint8_t* u8, int H, int W, float gw, float* out);
// the 8-bit form of an exemplar (see Ctx::ex_pk): u8 [H][W][3], img its RGBS floats
void launch_pack_exemplar(Ctx* c, const uint8_t* u8, int H, int W, const float* img, uint32_t* pk, float* srow);
// number of non-finite values in x [n] (synchronous)
int64_t count_nonfinite(Ctx* c, const float* x, int64_t n);
void launch_fill_guidance(Ctx* c, float* x, int H, int W, float gw);
void launch_blur_decimate(Ctx* c, const float* in, int H, int W, float gw, float* out);
void launch_upsample2(Ctx* c, const float* in, int H, int W, float gw, float* out);

// ---- perspective scale map (k_scale.hip)
// Eqs. 1-2 of an exemplar of ref_h x ref_w pixels under a slant and a tilt
// (radians), evaluated on the host; scale_geom validates the ranges.
struct ScaleGeom {
  double smax, smin, sd, ymax, sin_t, cos_t;
  int ref_h, ref_w;
};
ScaleGeom scale_geom(double slant, double tilt, int ref_h, int ref_w);
// channel 3 of x [H][W][4] = gw * the normalised map resampled to H x W
void launch_scale_guidance(Ctx* c, float* x, int H, int W, const ScaleGeom& g, float gw);
// x [H][W][4]: t x t tiles copied from the scale-matched windows of ex
// [Hz][Wz][4] (the map's size), rnd [tiles][2] uniform uint32 draws
void launch_scale_init(Ctx* c, const float* ex, int Hz, int Wz, float* x, int H, int W, int t, const uint32_t* rnd,
                       const ScaleGeom& g, float gw);

// ---- windows and exhaustive search (k_search.hip)
// Materialise windows as rows of float32 [n][D]: output grid (stride s, x
// wrap) when wrap, else the exemplar grid (all corners at stride s).
void launch_gather_windows(Ctx* c, const float* img, int H, int W, int w, int s, bool wrap, float* out);
// Exhaustive argmin of the direct squared distance between rows of Q [nq][D]
// and rows of Z [N][D]; zid maps a Z row to the id reported and used in
// tie-breaks (NULL = row index).
void launch_argmin_direct(Ctx* c, const float* Q, int64_t nq, const float* Z, int64_t N, int D,
                          const int32_t* zid, int32_t* best_id, float* best_d2);
// dist[q] = || x_q - z_nn[q] || over the full window (NaN for an invalid id)
void launch_winner_dist(Ctx* c, const float* x, int H, int W, int w, int s, const float* ex, int Hz, int Wz,
                        const int32_t* nn, float* dist);
// exhaustive full-D search of listed output windows: nn, dist = sqrt(d2)
void launch_exact_subset(Ctx* c, const float* x, int H, int W, int w, int s, const float* ex, int Hz, int Wz,
                         const int32_t* qids, int64_t n, int32_t* nn, float* dist);
// number of i with a[i] != b[i], added to *count (int32)
void launch_count_diff(Ctx* c, const int32_t* a, const int32_t* b, int64_t n, int32_t* count);
void launch_zero_i32(Ctx* c, int32_t* p, int64_t n);

// ---- histogram matching (k_hist.hip)
// counts [3][bins] of the R, G, B channels of img [n][4] (2 <= bins <= 256)
void launch_channel_hist(Ctx* c, const float* img, int64_t n, int bins, unsigned* counts);
// Eq. 9 factors 1 / (1 + excess) of the matched windows nn [nq] for output x
// and exemplar ex: both histograms and the factors (context scratch)
const float* hist_weight_factors(Ctx* c, const int32_t* nn, int64_t nq, const float* x, int H, int W,
                                 const float* ex, int Hz, int Wz, int w, int bins);
// W = max(dist, delta)^(r-2) [* factor]
void launch_irls_weights(Ctx* c, const float* dist, const float* factor, int64_t nq, float r, float delta, float* W);
// the final match: x's R, G, B take the exemplar's distribution rank for rank
void histogram_match(Ctx* c, float* x, int H, int W, const float* ex, int Hz, int Wz);

// ---- blend and energy (k_mstep.hip)
// ex_pk (optional): the exemplar's 8-bit form (Ctx::ex_pk), read instead of ex's RGB
void launch_mstep(Ctx* c, const int32_t* nn, const float* dist, float* x, int H, int W, int w, int s,
                  const float* ex, const uint32_t* ex_pk, int Hz, int Wz, float r, float delta, int o,
                  const float* wscale = nullptr);
void launch_energy(Ctx* c, const float* dist, int64_t n, float r, float delta, float* out2);
// The same energy with its partial sums in the library's fixed per-device
// array (no allocation); energy_scratch_init returns that array's device
// address for `device`, which must be current at the first call.
float* energy_scratch_init(int device);
void launch_energy_scratch(Ctx* c, const float* dist, int64_t n, float r, float delta, float* out2,
                           float* scratch_ptr);

// ---- index (k_index.hip)
void launch_mean_cov_image(Ctx* c, const float* img, int H, int W, int w, double* mean, double* cov);
// P = (window - mu) B for every window of the grid; B is [D][dp]; Qb
// (optional) [n][dk] = bf16(-2 P), zero past dp
void launch_project_image(Ctx* c, const float* img, int H, int W, int w, int s, bool wrap, const float* mu,
                          const float* B, int dp, float* P, uint16_t* Qb = nullptr, int dk = 0);
void launch_kmeans_mindist(Ctx* c, const float* P, int dp, const int32_t* members, int64_t m, const int32_t* seg_of,
                           const float* cand, float* mind, int first);
void launch_kmeans_assign(Ctx* c, const float* P, int dp, const int32_t* members, int64_t m, const int32_t* seg_of,
                          const int32_t* seg_cent_off, const int32_t* seg_k, const float* cents, int32_t* assign,
                          int32_t* changed);
void launch_kmeans_accumulate(Ctx* c, const float* P, int dp, const int32_t* members, int64_t m,
                              const int32_t* seg_of, const int32_t* seg_cent_off, const int32_t* assign,
                              unsigned long long* sums, int32_t* counts, int ncent);
// dst[i] = src[perm[i]] (rows of dp floats); norm[i] = ||dst[i]||^2 if non-null
void launch_permute_rows(Ctx* c, const float* src, const int32_t* perm, int64_t n, int dp, float* dst, float* norm);
void launch_to_bf16_rows(Ctx* c, const float* P, int64_t n, int dp, int dk, uint16_t* out, float* norm);
// ||z - mu||^2 per exemplar window (original id order)
void launch_centered_norm(Ctx* c, const float* img, int H, int W, int w, const float* mu, float* out);
// leaf order: res = max(0, cn[perm] - zn), bres = bn + res (bres optional)
void launch_residual(Ctx* c, const float* cn, const int32_t* perm, const float* zn, const float* bn, int64_t n,
                     float* res, float* bres);
void launch_leaf_of_ids(Ctx* c, const int32_t* leaf_of_ex, const int32_t* nn, int64_t n, int32_t* leaf, int64_t N);

// ---- tree search (k_tree.hip)
struct BucketBufs {
  int32_t* counts;    // [n_leaves]
  int32_t* off;       // [n_leaves + 1] query offsets per leaf
  int32_t* cursor;    // [n_leaves]
  int32_t* tile_off;  // [n_leaves + 1]
  int32_t* ntiles;    // [1]
  int32_t* order;     // [n] query ids grouped by leaf
  int2* tiles;        // [max_tiles] (leaf, first position in order)
  // optional [n_leaves]: the order of the leaves in the tile list (largest
  // leaves first, so that persistent scans end on short tiles); null: leaf order
  const int32_t* tile_order = nullptr;
};
void launch_descend(Ctx* c, const float* Qp, int64_t nq, int dp, const float* cent, const int32_t* first_child,
                    const int32_t* n_children, const int32_t* leaf_of_node, int n_nodes, int32_t* leaf);
// descent of the queries with margin < thr only (others: leaf -1); list, n scratch
void launch_descend_low_margin(Ctx* c, const float* Qp, int64_t nq, int dp, const float* margin, float thr,
                               const float* cent, const int32_t* first_child, const int32_t* n_children,
                               const int32_t* leaf_of_node, int n_nodes, int32_t* list, int32_t* n, int32_t* leaf);
void launch_bucket(Ctx* c, const int32_t* leaf, int64_t n, int n_leaves, int chunk, BucketBufs b);
// order[] holds pair indices (query * P + slot); results per pair: the best
// id and distance (nn, best_d2), or with top_d non-null the 8 best
// (distance, leaf position) sorted into top_d / top_i [pair][8].  The
// bucketing for it must use chunks of leaf_scan_f32_chunk(dp) pairs.
int leaf_scan_f32_chunk(int dp);
void launch_leaf_scan_f32(Ctx* c, const float* Qp, int dp, const float* Zp, const int32_t* perm,
                          const int32_t* leaf_off, const BucketBufs& b, int max_tiles, int P, const float* zres,
                          int32_t* nn, float* best_d2, float* top_d = nullptr, int32_t* top_i = nullptr);
void launch_learned_pairs(Ctx* c, const int32_t* prop, const float* margin, const int32_t* dleaf, int64_t nq, int P,
                          float thr, int n_leaves, int32_t* pair_leaf, int32_t* fallbacks);
void launch_merge_pairs_f32(Ctx* c, const int32_t* pair_leaf, const int32_t* pair_id, const float* pair_d, int64_t nq,
                            int P, int32_t* nn);

}  // namespace pts
