// Search phase (E-step) orchestration: for every output window, find the
// exemplar window it matches (Methodology 2.1, Eq. 4), by the chosen search
// form, then its full-dimension distance (used by the weights and the
// energy whatever space the search ran in).
#include <algorithm>
#include <string>

#include "api_internal.hpp"
#include "bf16_learned.hpp"

namespace pts {

namespace {

void require_index(Ctx* c, Index* ix, int w) {
  (void)c;
  PTS_REQUIRE(ix && ix->valid, PTS_ERR_STATE, "search mode needs an index (pts_build_index / pts_import_index)");
  PTS_REQUIRE(ix->w == w, PTS_ERR_ARG, "estep w differs from the index's w");
}

}  // namespace

BucketBufs bucket_buffers(Ctx* c, int64_t n, int n_leaves, int chunk, int* max_tiles, const char* tag) {
  const std::string t(tag);
  BucketBufs b;
  b.counts = c->buf<int32_t>((t + "_counts").c_str(), n_leaves);
  b.off = c->buf<int32_t>((t + "_off").c_str(), n_leaves + 1);
  b.cursor = c->buf<int32_t>((t + "_cursor").c_str(), n_leaves);
  b.tile_off = c->buf<int32_t>((t + "_tile_off").c_str(), n_leaves + 1);
  b.ntiles = c->buf<int32_t>((t + "_ntiles").c_str(), 1);
  b.order = c->buf<int32_t>((t + "_order").c_str(), std::max<int64_t>(1, n));
  *max_tiles = (int)(ceil_div(n, chunk) + n_leaves);
  b.tiles = c->buf<int2>((t + "_tiles").c_str(), *max_tiles);
  return b;
}

void project_on(Ctx* c, const Index& ix, const float* x, int H, int W, int stride, float* qp, uint16_t* qb = nullptr) {
  launch_project_image(c, x, H, W, ix.w, stride, true, ix.mu_f.as<float>(), ix.basis_f.as<float>(), ix.dp, qp, qb,
                       ix.dk);
}

EstepStats estep_on(Ctx* c, ExView ex, Index* ix, const float* x, int H, int W, const pts_estep_params& p,
                    int32_t* nn, float* dist, bool timing, bool count_work) {
  validate_grid(H, W, p.w, p.stride);
  PTS_REQUIRE(p.w <= ex.Hz && p.w <= ex.Wz, PTS_ERR_ARG, "estep: window larger than the exemplar");
  const Grid g{H, W, p.w, p.stride};
  const int64_t nq = g.nq();
  const int w = p.w, D = 4 * w * w;
  const int64_t N = (int64_t)(ex.Hz - w + 1) * (ex.Wz - w + 1);
  EstepStats st;
  st.nq = nq;
  bool dist_done = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timing) {
    PTS_HIP(hipEventCreate(&e0));
    PTS_HIP(hipEventCreate(&e1));
    PTS_HIP(hipEventRecord(e0, c->stream));
  }
  switch (p.mode) {
    case PTS_MODE_EXACT_FULL: {
      PTS_REQUIRE(N < (int64_t)1 << 31, PTS_ERR_UNSUPPORTED, "exact search: too many windows");
      float* zw = c->buf<float>("exact_zw", (size_t)N * D);
      float* qw = c->buf<float>("exact_qw", (size_t)nq * D);
      launch_gather_windows(c, ex.img, ex.Hz, ex.Wz, w, 1, false, zw);
      launch_gather_windows(c, x, H, W, w, p.stride, true, qw);
      launch_argmin_direct(c, qw, nq, zw, N, D, nullptr, nn, nullptr);
      break;
    }
    case PTS_MODE_EXACT_PCA: {
      require_index(c, ix, w);
      float* qp = c->buf<float>("qproj", (size_t)nq * ix->dp);
      project_on(c, *ix, x, H, W, p.stride, qp);
      launch_argmin_direct(c, qp, nq, ix->zproj.as<float>(), ix->N, ix->dp, ix->perm.as<int32_t>(), nn, nullptr);
      break;
    }
    case PTS_MODE_TREE: {
      require_index(c, ix, w);
      float* qp = c->buf<float>("qproj", (size_t)nq * ix->dp);
      project_on(c, *ix, x, H, W, p.stride, qp);
      int32_t* leaf = c->buf<int32_t>("qleaf", nq);
      launch_descend(c, qp, nq, ix->dp, ix->cent.as<float>(), ix->first_child.as<int32_t>(),
                     ix->n_children.as<int32_t>(), ix->leaf_of_node.as<int32_t>(), ix->tree.n_nodes(), leaf);
      int max_tiles = 0;
      const int chunk = leaf_scan_f32_chunk(ix->dp);
      BucketBufs b = bucket_buffers(c, nq, ix->tree.n_leaves(), chunk, &max_tiles);
      b.tile_order = ix->leaf_by_rows.as<int32_t>();
      launch_bucket(c, leaf, nq, ix->tree.n_leaves(), chunk, b);
      launch_leaf_scan_f32(c, qp, ix->dp, ix->zproj.as<float>(), ix->perm.as<int32_t>(), ix->leaf_off.as<int32_t>(),
                           b, max_tiles, 1, p.residual ? ix->zres.as<float>() : nullptr, nn, nullptr);
      break;
    }
    case PTS_MODE_BRUTE_BF16: {
      require_index(c, ix, w);
      PTS_REQUIRE(ix->has_bf16, PTS_ERR_STATE, "BRUTE_BF16 needs an index built with make_bf16");
      float* qp = c->buf<float>("qproj", (size_t)nq * ix->dp);
      uint16_t* qb = c->buf<uint16_t>("qbf16", (size_t)nq * ix->dk);
      project_on(c, *ix, x, H, W, p.stride, qp, qb);
      int32_t* novf = nullptr;
      int64_t work[2] = {0, 0};
      dist_done = search_brute_bf16(c, ex, *ix, x, H, W, p, qp, qb, nq, nn, dist, &novf, count_work ? work : nullptr);
      st.scan_rows = work[0];
      st.collect_rows = work[1];
      if (timing && novf) {
        int32_t h = 0;
        PTS_HIP(hipMemcpyAsync(&h, novf, 4, hipMemcpyDeviceToHost, c->stream));
        PTS_HIP(hipStreamSynchronize(c->stream));
        st.scan_overflows = h;
      }
      break;
    }
    case PTS_MODE_LEARNED:
    case PTS_MODE_LEARNED_BF16:
    case PTS_MODE_LEARNED_BF16_CLASS: {
      require_index(c, ix, w);
      PTS_REQUIRE(c->mlp.valid, PTS_ERR_STATE, "learned modes need an MLP (pts_mlp_init / set_weights)");
      PTS_REQUIRE(c->mlp.n_in == ix->d && c->mlp.n_out == ix->tree.n_leaves(), PTS_ERR_STATE,
                  "MLP shape does not match the index (n_in = d, n_out = leaves)");
      float* qp = c->buf<float>("qproj", (size_t)nq * ix->dp);
      const bool bf = p.mode != PTS_MODE_LEARNED;
      PTS_REQUIRE(!bf || ix->has_bf16, PTS_ERR_STATE, "LEARNED_BF16 needs an index built with make_bf16");
      uint16_t* qb = bf ? c->buf<uint16_t>("qbf16", (size_t)nq * ix->dk) : nullptr;
      project_on(c, *ix, x, H, W, p.stride, qp, qb);
      int32_t* novf = nullptr;
      int64_t work[2] = {0, 0};
      st.fallbacks =
          search_learned(c, ex, *ix, x, H, W, p, qp, qb, nq, nn, dist, &dist_done, bf,
                         p.mode == PTS_MODE_LEARNED_BF16_CLASS, timing, &novf,
                         count_work ? work : nullptr);
      st.scan_rows = work[0];
      st.collect_rows = work[1];
      if (timing && novf) {
        int32_t h = 0;
        PTS_HIP(hipMemcpyAsync(&h, novf, 4, hipMemcpyDeviceToHost, c->stream));
        PTS_HIP(hipStreamSynchronize(c->stream));
        st.scan_overflows = h;
      }
      break;
    }
    default:
      fail(PTS_ERR_ARG, "unknown search mode");
  }
  if (!dist_done) launch_winner_dist(c, x, H, W, w, p.stride, ex.img, ex.Hz, ex.Wz, nn, dist);
  if (timing) {
    PTS_HIP(hipEventRecord(e1, c->stream));
    PTS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PTS_HIP(hipEventElapsedTime(&ms, e0, e1));
    st.ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return st;
}

EstepStats run_estep(Ctx* c, const float* x, int H, int W, const pts_estep_params& p, int32_t* nn, float* dist,
                     bool timing) {
  ExView ex = ctx_exemplar(c);
  Index* ix = c->index.valid ? &c->index : nullptr;
  return estep_on(c, ex, ix, x, H, W, p, nn, dist, timing, timing);
}

void project_queries(Ctx* c, const float* x, int H, int W, int stride, float* qproj, bool padded_out) {
  PTS_REQUIRE(c->index.valid, PTS_ERR_STATE, "project: no index");
  const Index& ix = c->index;
  validate_grid(H, W, ix.w, stride);
  const int64_t nq = Grid{H, W, ix.w, stride}.nq();
  if (padded_out || ix.dp == ix.d) {
    project_on(c, ix, x, H, W, stride, qproj);
    return;
  }
  float* qp = c->buf<float>("qproj_tmp", (size_t)nq * ix.dp);
  project_on(c, ix, x, H, W, stride, qp);
  PTS_HIP(hipMemcpy2DAsync(qproj, (size_t)ix.d * 4, qp, (size_t)ix.dp * 4, (size_t)ix.d * 4, (size_t)nq,
                           hipMemcpyDeviceToDevice, c->stream));
}

void exemplar_projection(Ctx* c, float* zproj) {
  PTS_REQUIRE(c->index.valid, PTS_ERR_STATE, "exemplar_projection: no index");
  const Index& ix = c->index;
  ExView ex = ctx_exemplar(c);
  float* zo = c->buf<float>("ix_zorig", (size_t)ix.N * ix.dp);
  launch_project_image(c, ex.img, ex.Hz, ex.Wz, ix.w, 1, false, ix.mu_f.as<float>(), ix.basis_f.as<float>(), ix.dp,
                       zo);
  PTS_HIP(hipMemcpy2DAsync(zproj, (size_t)ix.d * 4, zo, (size_t)ix.dp * 4, (size_t)ix.d * 4, (size_t)ix.N,
                           hipMemcpyDeviceToDevice, c->stream));
}

void descend_unpadded(Ctx* c, const float* qproj, int64_t n, int32_t* leaf) {
  const Index& ix = c->index;
  if (n == 0) return;
  float* qp = c->buf<float>("qdesc_tmp", (size_t)n * ix.dp);
  launch_zero_i32(c, reinterpret_cast<int32_t*>(qp), n * ix.dp);
  PTS_HIP(hipMemcpy2DAsync(qp, (size_t)ix.dp * 4, qproj, (size_t)ix.d * 4, (size_t)ix.d * 4, (size_t)n,
                           hipMemcpyDeviceToDevice, c->stream));
  launch_descend(c, qp, n, ix.dp, ix.cent.as<float>(), ix.first_child.as<int32_t>(), ix.n_children.as<int32_t>(),
                 ix.leaf_of_node.as<int32_t>(), ix.tree.n_nodes(), leaf);
}

}  // namespace pts
