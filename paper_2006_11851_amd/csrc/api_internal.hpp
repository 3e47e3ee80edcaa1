// Host orchestration shared by the C ABI functions (internal).
#pragma once

#include "kernels.hpp"

namespace pts {

struct EstepStats {
  int64_t nq = 0;
  int64_t fallbacks = 0;
  int64_t scan_overflows = 0;
  int64_t scan_rows = 0, collect_rows = 0;
  double ms = 0.0;
};

// An exemplar image the search and blend run against; pk / srow: its 8-bit
// form (Ctx::ex_pk) when it has one, else null.
struct ExView {
  const float* img;
  int Hz, Wz;
  const uint32_t* pk = nullptr;
  const float* srow = nullptr;
};

inline ExView ctx_exemplar(Ctx* c) {
  PTS_REQUIRE(c->Hz > 0, PTS_ERR_STATE, "no exemplar set");
  ExView v{c->ex.as<float>(), c->Hz, c->Wz};
  if (c->ex_packed) {
    v.pk = c->ex_pk.as<uint32_t>();
    v.srow = c->ex_srow.as<float>();
  }
  return v;
}

// padded PCA width: the smallest of 16, 24, 32, 48, 64, 96, 128 >= d
int padded_dims(int d);

// index.cpp
void build_index_on(Ctx* c, ExView ex, const pts_index_params& p, Index& ix, pts_index_info* info);
void export_index(Ctx* c, const Index& ix, pts_index_host* out);
void import_index(Ctx* c, ExView ex, const pts_index_host& in, int make_bf16, Index& ix);

// estep.cpp
// timing: record the call's time, fallbacks and per-query passes; count_work:
// also the scan counts (extra synchronisations)
EstepStats estep_on(Ctx* c, ExView ex, Index* ix, const float* x, int H, int W, const pts_estep_params& p,
                    int32_t* nn, float* dist, bool timing, bool count_work = false);
EstepStats run_estep(Ctx* c, const float* x, int H, int W, const pts_estep_params& p, int32_t* nn, float* dist,
                     bool timing);
// projected queries; padded_out: rows of ix.dp floats, else rows of ix.d
void project_queries(Ctx* c, const float* x, int H, int W, int stride, float* qproj, bool padded_out);
void exemplar_projection(Ctx* c, float* zproj);
void descend_unpadded(Ctx* c, const float* qproj, int64_t n, int32_t* leaf);

BucketBufs bucket_buffers(Ctx* c, int64_t n, int n_leaves, int chunk, int* max_tiles, const char* tag = "bk");

// solve.cpp
const float* pyramid_level(Ctx* c, int levels, int level, float gw, int* h, int* w,
                           const ScaleSpec& scale = ScaleSpec());
void run_solve(Ctx* c, const pts_solve_params& p, const float* x0, int H0, int W0, float* x, int H, int W,
               pts_solve_trace* tr);

}  // namespace pts

// the opaque handle of the C ABI is the context itself
struct pts_ctx : public pts::Ctx {};
