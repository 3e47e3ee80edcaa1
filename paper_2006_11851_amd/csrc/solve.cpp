// Coarse-to-fine solve (Methodology 2.1): at every level the search phase
// and the optimisation phase alternate for a fixed number of iterations; the
// result is upsampled by bilinear interpolation to start the next level.
// Every level has its own exemplar (a Gaussian pyramid level) and its own
// PCA basis and tree.
#include <chrono>
#include <cstring>

#include "api_internal.hpp"

namespace pts {

// writes level l's guidance (gw >= 0): the row guidance, or the scale map
static void level_guidance(Ctx* c, float* img, int h, int w, float gw, const ScaleSpec& sc) {
  if (sc.on)
    launch_scale_guidance(c, img, h, w, scale_geom(sc.slant, sc.tilt, h, w), gw);
  else
    launch_fill_guidance(c, img, h, w, gw);
}

const float* pyramid_level(Ctx* c, int levels, int level, float gw, int* h, int* w, const ScaleSpec& scale) {
  if (c->pyr_version != c->ex_version || c->pyr_levels != levels || c->pyr_gw != gw || c->pyr_scale != scale) {
    c->pyr_version = ~0ull;  // invalid until complete
    PTS_REQUIRE((c->Hz >> (levels - 1)) >= 4 && (c->Wz >> (levels - 1)) >= 4, PTS_ERR_ARG,
                "pyramid: exemplar too small for that many levels");
    PTS_REQUIRE(levels == 1 || ((c->Hz % (1 << (levels - 1))) == 0 && (c->Wz % (1 << (levels - 1))) == 0),
                PTS_ERR_ARG, "pyramid: exemplar sides must be divisible by 2^(levels-1)");
    c->pyr_img.clear();
    c->pyr_h.assign(levels, 0);
    c->pyr_w.assign(levels, 0);
    for (int l = 0; l < levels; ++l) c->pyr_img.emplace_back(new DevMem());
    // finest = the exemplar itself, its guidance rewritten with this weight
    // (gw < 0: its own guidance channel kept, and blurred for the coarser levels)
    const int L = levels - 1;
    c->pyr_h[L] = c->Hz;
    c->pyr_w[L] = c->Wz;
    float* fin = static_cast<float*>(c->pyr_img[L]->ensure(c, (size_t)c->Hz * c->Wz * 16));
    PTS_HIP(hipMemcpyAsync(fin, c->ex.ptr, (size_t)c->Hz * c->Wz * 16, hipMemcpyDeviceToDevice, c->stream));
    if (gw >= 0.f) level_guidance(c, fin, c->Hz, c->Wz, gw, scale);
    for (int l = L - 1; l >= 0; --l) {
      c->pyr_h[l] = c->pyr_h[l + 1] / 2;
      c->pyr_w[l] = c->pyr_w[l + 1] / 2;
      float* dst = static_cast<float*>(c->pyr_img[l]->ensure(c, (size_t)c->pyr_h[l] * c->pyr_w[l] * 16));
      launch_blur_decimate(c, c->pyr_img[l + 1]->as<float>(), c->pyr_h[l + 1], c->pyr_w[l + 1], gw, dst);
      if (gw >= 0.f && scale.on) level_guidance(c, dst, c->pyr_h[l], c->pyr_w[l], gw, scale);
    }
    c->pyr_version = c->ex_version;
    c->pyr_levels = levels;
    c->pyr_gw = gw;
    c->pyr_scale = scale;
  }
  *h = c->pyr_h[level];
  *w = c->pyr_w[level];
  return c->pyr_img[level]->as<float>();
}

void run_solve(Ctx* c, const pts_solve_params& p, const float* x0, int H0, int W0, float* x, int H, int W,
               pts_solve_trace* tr) {
  PTS_REQUIRE(c->Hz > 0, PTS_ERR_STATE, "solve: no exemplar");
  PTS_REQUIRE(p.levels >= 1 && p.levels <= 8 && p.level, PTS_ERR_ARG, "solve: levels must be 1..8");
  const int L = p.levels;
  PTS_REQUIRE(H == (H0 << (L - 1)) && W == (W0 << (L - 1)), PTS_ERR_ARG, "solve: H, W must be H0, W0 << (levels-1)");
  PTS_REQUIRE(p.hist_bins == 0 || (p.hist_bins >= 2 && p.hist_bins <= 256), PTS_ERR_ARG,
              "solve: hist_bins must be 0 or 2..256");
  for (int l = 0; l < L; ++l) {
    const pts_level_params& lp = p.level[l];
    validate_grid(H0 << l, W0 << l, lp.w, lp.stride);
    PTS_REQUIRE(lp.iters >= 0, PTS_ERR_ARG, "solve: iters must be >= 0");
  }
  if (tr) tr->count = 0;
  const float gw = p.guidance_weight;
  ScaleSpec scale;
  if (p.scale_map) {
    PTS_REQUIRE(gw >= 0.f, PTS_ERR_ARG, "solve: the scale map needs guidance_weight >= 0");
    scale.on = true;
    scale.slant = p.slant;
    scale.tilt = p.tilt;
    // checks the angles and every level's size before any work
    for (int l = 0; l < L; ++l) scale_geom(scale.slant, scale.tilt, c->Hz >> (L - 1 - l), c->Wz >> (L - 1 - l));
  }
  // working image of the current level (two buffers for the upsampling)
  DevMem buf_a, buf_b;
  float* cur = static_cast<float*>(buf_a.ensure(c, (size_t)H0 * W0 * 16));
  PTS_HIP(hipMemcpyAsync(cur, x0, (size_t)H0 * W0 * 16, hipMemcpyDeviceToDevice, c->stream));
  DevMem nn_a, nn_b, dist_m, e_out, diff_m;
  Index level_index;
  for (int l = 0; l < L; ++l) {
    const pts_level_params& lp = p.level[l];
    const int h = H0 << l, w = W0 << l;
    int hz = 0, wz = 0;
    const float* zimg = pyramid_level(c, L, l, gw, &hz, &wz, scale);
    ExView ex{zimg, hz, wz};
    const bool finest = (l == L - 1);
    const int mode = finest ? p.mode : p.coarse_mode;
    Index* ix = nullptr;
    if (mode != PTS_MODE_EXACT_FULL) {
      if (finest && p.reuse_finest_index) {
        PTS_REQUIRE(c->index.valid && c->index.w == lp.w && c->index.N == (int64_t)(hz - lp.w + 1) * (wz - lp.w + 1),
                    PTS_ERR_STATE, "solve: context index does not match the finest level");
        ix = &c->index;
      } else {
        pts_index_params ip{};
        ip.w = lp.w;
        ip.pca_dims = lp.pca_dims;
        ip.variance_target = 0.95;
        ip.branching = lp.branching;
        ip.depth = lp.depth;
        ip.kmeans_max_iter = p.kmeans_max_iter;
        ip.seed = p.seed;
        ip.make_bf16 = (mode == PTS_MODE_BRUTE_BF16 || mode == PTS_MODE_LEARNED_BF16 ||
                        mode == PTS_MODE_LEARNED_BF16_CLASS) ? 1 : 0;
        build_index_on(c, ex, ip, level_index, nullptr);
        ix = &level_index;
      }
    }
    pts_estep_params ep{};
    ep.mode = mode;
    ep.w = lp.w;
    ep.stride = lp.stride;
    ep.topk = p.topk;
    ep.rerank_full = p.rerank_full;
    ep.n_proposals = p.n_proposals;
    ep.margin = p.margin;
    ep.residual = p.residual;
    const Grid g{h, w, lp.w, lp.stride};
    const int64_t nq = g.nq();
    int32_t* nn_cur = static_cast<int32_t*>(nn_a.ensure(c, (size_t)nq * 4));
    int32_t* nn_prev = static_cast<int32_t*>(nn_b.ensure(c, (size_t)nq * 4));
    float* dist = static_cast<float*>(dist_m.ensure(c, (size_t)nq * 4));
    float* eo = static_cast<float*>(e_out.ensure(c, 8));
    int32_t* dcount = static_cast<int32_t*>(diff_m.ensure(c, 4));
    for (int t = 0; t < lp.iters; ++t) {
      const auto t0 = std::chrono::steady_clock::now();
      EstepStats st = estep_on(c, ex, ix, cur, h, w, ep, nn_cur, dist, tr != nullptr && mode >= PTS_MODE_LEARNED);
      launch_energy(c, dist, nq, p.r, p.delta, eo);
      launch_zero_i32(c, dcount, 1);
      if (t > 0) launch_count_diff(c, nn_cur, nn_prev, nq, dcount);
      const float* factor =
          p.hist_bins ? hist_weight_factors(c, nn_cur, nq, cur, h, w, zimg, hz, wz, lp.w, p.hist_bins) : nullptr;
      launch_mstep(c, nn_cur, dist, cur, h, w, lp.w, lp.stride, zimg, nullptr, hz, wz, p.r, p.delta, p.patch_offset,
                   factor);
      if (tr) {
        float eh[2];
        int32_t ch = 0;
        PTS_HIP(hipMemcpyAsync(eh, eo, 8, hipMemcpyDeviceToHost, c->stream));
        PTS_HIP(hipMemcpyAsync(&ch, dcount, 4, hipMemcpyDeviceToHost, c->stream));
        PTS_HIP(hipStreamSynchronize(c->stream));
        if (tr->count < tr->capacity) {
          const int k = tr->count++;
          if (tr->level) tr->level[k] = l;
          if (tr->E) tr->E[k] = eh[0];
          if (tr->E2) tr->E2[k] = eh[1];
          if (tr->ms)
            tr->ms[k] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          if (tr->nq) tr->nq[k] = nq;
          if (tr->changes) tr->changes[k] = (t == 0) ? nq : ch;
          if (tr->fallbacks) tr->fallbacks[k] = st.fallbacks;
        }
      }
      std::swap(nn_cur, nn_prev);
    }
    if (!finest) {
      float* nxt = static_cast<float*>((l % 2 == 0 ? buf_b : buf_a).ensure(c, (size_t)(2 * h) * (2 * w) * 16));
      launch_upsample2(c, cur, h, w, gw, nxt);
      if (scale.on)  // the next exemplar level's map resampled to the output
        launch_scale_guidance(c, nxt, 2 * h, 2 * w,
                              scale_geom(scale.slant, scale.tilt, c->Hz >> (L - 2 - l), c->Wz >> (L - 2 - l)), gw);
      cur = nxt;
    }
  }
  PTS_HIP(hipMemcpyAsync(x, cur, (size_t)H * W * 16, hipMemcpyDeviceToDevice, c->stream));
  // Section 4, step 4: the result's histograms matched to the exemplar's
  if (p.final_hist_match) histogram_match(c, x, H, W, c->ex.as<float>(), c->Hz, c->Wz);
  PTS_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace pts
