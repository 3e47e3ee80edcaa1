// C ABI of libpts (declarations and contracts in include/pts.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "api_internal.hpp"
#include "eig.hpp"

using namespace pts;

static thread_local std::string g_create_error;

template <class F>
static int guard(pts_ctx* c, F&& f) {
  try {
    if (c) PTS_HIP(hipSetDevice(c->device));
    f();
    if (c) c->last_error.clear();
    return PTS_OK;
  } catch (const pts::Error& e) {
    if (c) c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed";
    return PTS_ERR_OOM;
  } catch (const std::exception& e) {
    if (c) c->last_error = e.what();
    return PTS_ERR_ARG;
  }
}

#define CTX_REQUIRED(c)                                                                            \
  do {                                                                                             \
    if (!(c)) return PTS_ERR_ARG;                                                                  \
  } while (0)

extern "C" {

int pts_create(pts_ctx** out, int device, void* hip_stream, const pts_alloc* alloc_or_null) {
  if (!out) return PTS_ERR_ARG;
  *out = nullptr;
  try {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
      g_create_error = "no HIP device";
      return PTS_ERR_UNSUPPORTED;
    }
    if (device < 0 || device >= n) {
      g_create_error = "device index out of range";
      return PTS_ERR_ARG;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
      g_create_error = "hipGetDeviceProperties failed";
      return PTS_ERR_HIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      g_create_error = std::string("device is ") + prop.gcnArchName + ", libpts is built for gfx950";
      return PTS_ERR_UNSUPPORTED;
    }
    if (alloc_or_null && (!alloc_or_null->alloc || !alloc_or_null->release)) {
      g_create_error = "allocator needs both alloc and release";
      return PTS_ERR_ARG;
    }
    // the fixed scratch of the allocation-free entry points, once per device
    float* escratch = nullptr;
    try {
      if (hipSetDevice(device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        return PTS_ERR_HIP;
      }
      escratch = pts::energy_scratch_init(device);
    } catch (const pts::Error& e) {
      g_create_error = e.msg;
      return e.code;
    }
    pts_ctx* c = new pts_ctx();
    c->device = device;
    c->energy_scratch = escratch;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (alloc_or_null) {
      c->alloc = *alloc_or_null;
      c->has_alloc = true;
    }
    *out = c;
    g_create_error.clear();
    return PTS_OK;
  } catch (...) {
    g_create_error = "context creation failed";
    return PTS_ERR_OOM;
  }
}

void pts_destroy(pts_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  delete c;
}

const char* pts_last_error(const pts_ctx* c) { return c ? c->last_error.c_str() : g_create_error.c_str(); }

int pts_set_stream(pts_ctx* c, void* hip_stream) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    c->prof_drain();
    c->stream = static_cast<hipStream_t>(hip_stream);
  });
}

// ---------------------------------------------------------------- exemplar

int pts_set_exemplar(pts_ctx* c, const float* rgbs, int Hz, int Wz) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(rgbs && Hz >= 2 && Wz >= 2, PTS_ERR_ARG, "set_exemplar: bad image");
    PTS_REQUIRE((int64_t)Hz * Wz <= ((int64_t)1 << 26), PTS_ERR_UNSUPPORTED, "exemplar larger than 2^26 pixels");
    PTS_REQUIRE(count_nonfinite(c, rgbs, (int64_t)Hz * Wz * 4) == 0, PTS_ERR_ARG,
                "set_exemplar: the image holds non-finite values");
    float* dst = static_cast<float*>(c->ex.ensure(c, (size_t)Hz * Wz * 16));
    PTS_HIP(hipMemcpyAsync(dst, rgbs, (size_t)Hz * Wz * 16, hipMemcpyDeviceToDevice, c->stream));
    c->Hz = Hz;
    c->Wz = Wz;
    c->ex_packed = false;
    c->ex_version++;
    c->index.valid = false;
    c->mlp.valid = false;
  });
}

int pts_set_exemplar_u8(pts_ctx* c, const uint8_t* rgb_host, int Hz, int Wz, float gw) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(rgb_host && Hz >= 2 && Wz >= 2, PTS_ERR_ARG, "set_exemplar_u8: bad image");
    PTS_REQUIRE(std::isfinite(gw), PTS_ERR_ARG, "set_exemplar_u8: guidance weight must be finite");
    PTS_REQUIRE((int64_t)Hz * Wz <= ((int64_t)1 << 26), PTS_ERR_UNSUPPORTED, "exemplar larger than 2^26 pixels");
    uint8_t* tmp = c->buf<uint8_t>("u8_upload", (size_t)Hz * Wz * 3);
    PTS_HIP(hipMemcpyAsync(tmp, rgb_host, (size_t)Hz * Wz * 3, hipMemcpyHostToDevice, c->stream));
    float* dst = static_cast<float*>(c->ex.ensure(c, (size_t)Hz * Wz * 16));
    launch_rgbs_from_u8(c, tmp, Hz, Wz, gw, dst);
    uint32_t* pk = static_cast<uint32_t*>(c->ex_pk.ensure(c, (size_t)Hz * Wz * 4));
    float* srow = static_cast<float*>(c->ex_srow.ensure(c, (size_t)Hz * 4));
    launch_pack_exemplar(c, tmp, Hz, Wz, dst, pk, srow);
    PTS_HIP(hipStreamSynchronize(c->stream));  // host buffer may be released by the caller
    c->Hz = Hz;
    c->Wz = Wz;
    c->ex_packed = true;
    c->ex_version++;
    c->index.valid = false;
    c->mlp.valid = false;
  });
}

int pts_fill_guidance(pts_ctx* c, float* x, int H, int W, float gw) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(x && H > 0 && W > 0, PTS_ERR_ARG, "fill_guidance: bad image");
    launch_fill_guidance(c, x, H, W, gw);
  });
}

int pts_scale_guidance(pts_ctx* c, float* x, int H, int W, int ref_h, int ref_w, double slant, double tilt,
                       float weight) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(x && H > 0 && W > 0, PTS_ERR_ARG, "scale_guidance: bad image");
    PTS_REQUIRE(std::isfinite(weight), PTS_ERR_ARG, "scale_guidance: weight must be finite");
    launch_scale_guidance(c, x, H, W, scale_geom(slant, tilt, ref_h, ref_w), weight);
  });
}

int pts_scale_init(pts_ctx* c, const float* ex, int Hz, int Wz, float* x, int H, int W, int tile,
                   const uint32_t* rnd, double slant, double tilt, float weight) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(ex && x && rnd && H > 0 && W > 0, PTS_ERR_ARG, "scale_init: bad image");
    PTS_REQUIRE(std::isfinite(weight), PTS_ERR_ARG, "scale_init: weight must be finite");
    launch_scale_init(c, ex, Hz, Wz, x, H, W, tile, rnd, scale_geom(slant, tilt, Hz, Wz), weight);
  });
}

int pts_rgbs_from_u8(pts_ctx* c, const uint8_t* rgb_host, int H, int W, float gw, float* x) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(rgb_host && x && H > 0 && W > 0, PTS_ERR_ARG, "rgbs_from_u8: bad image");
    uint8_t* tmp = c->buf<uint8_t>("u8_upload", (size_t)H * W * 3);
    PTS_HIP(hipMemcpyAsync(tmp, rgb_host, (size_t)H * W * 3, hipMemcpyHostToDevice, c->stream));
    launch_rgbs_from_u8(c, tmp, H, W, gw, x);
    PTS_HIP(hipStreamSynchronize(c->stream));
  });
}

// ---------------------------------------------------------------- index

int pts_build_index(pts_ctx* c, const pts_index_params* p, pts_index_info* info) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(p, PTS_ERR_ARG, "build_index: null params");
    ExView ex = ctx_exemplar(c);
    c->mlp.valid = false;  // leaf ids change with a new tree
    build_index_on(c, ex, *p, c->index, info);
  });
}

int pts_export_index(pts_ctx* c, pts_index_host* ix) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(ix, PTS_ERR_ARG, "export_index: null");
    export_index(c, c->index, ix);
  });
}

int pts_import_index(pts_ctx* c, const pts_index_host* ix, int make_bf16) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(ix, PTS_ERR_ARG, "import_index: null");
    ExView ex = ctx_exemplar(c);
    c->mlp.valid = false;
    import_index(c, ex, *ix, make_bf16, c->index);
  });
}

// ---------------------------------------------------------------- E-step

int pts_estep(pts_ctx* c, const float* x, int H, int W, const pts_estep_params* p, int32_t* nn, float* dist,
              pts_estep_stats* st) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(p && x && nn && dist, PTS_ERR_ARG, "estep: null argument");
    if (st) {  // the statistics call waits anyway: the image is checked too
      PTS_REQUIRE(H > 0 && W > 0, PTS_ERR_ARG, "estep: bad image size");
      PTS_REQUIRE(count_nonfinite(c, x, (int64_t)H * W * 4) == 0, PTS_ERR_ARG, "estep: the image holds non-finite values");
    }
    EstepStats s = run_estep(c, x, H, W, *p, nn, dist, st != nullptr);
    if (st) {
      st->nq = s.nq;
      st->fallbacks = s.fallbacks;
      st->scan_overflows = s.scan_overflows;
      st->scan_rows = s.scan_rows;
      st->collect_rows = s.collect_rows;
      st->ms = s.ms;
    }
  });
}

int pts_exact_search(pts_ctx* c, const float* x, int H, int W, int w, int stride, const int32_t* qids, int64_t n,
                     int32_t* nn, float* dist) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(x && n >= 0 && (n == 0 || (qids && nn && dist)), PTS_ERR_ARG, "exact_search: bad arguments");
    ExView ex = ctx_exemplar(c);
    validate_grid(H, W, w, stride);
    PTS_REQUIRE(w <= ex.Hz && w <= ex.Wz, PTS_ERR_ARG, "exact_search: window larger than the exemplar");
    launch_exact_subset(c, x, H, W, w, stride, ex.img, ex.Hz, ex.Wz, qids, n, nn, dist);
  });
}

int pts_project(pts_ctx* c, const float* x, int H, int W, int stride, float* qproj) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(x && qproj, PTS_ERR_ARG, "project: null argument");
    project_queries(c, x, H, W, stride, qproj, /*padded_out=*/false);
  });
}

int pts_exemplar_projection(pts_ctx* c, float* zproj) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(zproj, PTS_ERR_ARG, "exemplar_projection: null argument");
    exemplar_projection(c, zproj);
  });
}

int pts_leaf_of(pts_ctx* c, const int32_t* nn, int64_t n, int32_t* leaf) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(c->index.valid, PTS_ERR_STATE, "leaf_of: no index");
    PTS_REQUIRE(n >= 0 && (n == 0 || (nn && leaf)), PTS_ERR_ARG, "leaf_of: bad arguments");
    if (n) launch_leaf_of_ids(c, c->index.leaf_of_ex.as<int32_t>(), nn, n, leaf, c->index.N);
  });
}

int pts_descend(pts_ctx* c, const float* qproj, int64_t n, int32_t* leaf) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(c->index.valid, PTS_ERR_STATE, "descend: no index");
    PTS_REQUIRE(n >= 0 && (n == 0 || (qproj && leaf)), PTS_ERR_ARG, "descend: bad arguments");
    descend_unpadded(c, qproj, n, leaf);
  });
}

// ---------------------------------------------------------------- M-step / energy

int pts_mstep(pts_ctx* c, const int32_t* nn, const float* dist, float* x, int H, int W, const pts_mstep_params* p) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(p && nn && dist && x, PTS_ERR_ARG, "mstep: null argument");
    PTS_REQUIRE(c->Hz > 0, PTS_ERR_STATE, "mstep: no exemplar");
    validate_grid(H, W, p->w, p->stride);
    PTS_REQUIRE(p->w <= c->Hz && p->w <= c->Wz, PTS_ERR_ARG, "mstep: window larger than exemplar");
    PTS_REQUIRE(p->r > 0.f && p->r <= 2.f && p->delta > 0.f, PTS_ERR_ARG, "mstep: need 0 < r <= 2, delta > 0");
    PTS_REQUIRE(p->hist_bins == 0 || (p->hist_bins >= 2 && p->hist_bins <= 256), PTS_ERR_ARG,
                "mstep: hist_bins must be 0 or 2..256");
    const float* factor =
        p->hist_bins ? hist_weight_factors(c, nn, Grid{H, W, p->w, p->stride}.nq(), x, H, W, c->ex.as<float>(), c->Hz,
                                           c->Wz, p->w, p->hist_bins)
                     : nullptr;
    launch_mstep(c, nn, dist, x, H, W, p->w, p->stride, c->ex.as<float>(),
                 c->ex_packed ? c->ex_pk.as<uint32_t>() : nullptr, c->Hz, c->Wz, p->r, p->delta,
                 p->patch_offset, factor);
  });
}

int pts_irls_weights(pts_ctx* c, const int32_t* nn, const float* dist, const float* x, int H, int W,
                     const pts_mstep_params* p, float* weights) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(p && nn && dist && x && weights, PTS_ERR_ARG, "irls_weights: null argument");
    PTS_REQUIRE(c->Hz > 0, PTS_ERR_STATE, "irls_weights: no exemplar");
    validate_grid(H, W, p->w, p->stride);
    PTS_REQUIRE(p->w <= c->Hz && p->w <= c->Wz, PTS_ERR_ARG, "irls_weights: window larger than exemplar");
    PTS_REQUIRE(p->r > 0.f && p->r <= 2.f && p->delta > 0.f, PTS_ERR_ARG, "irls_weights: need 0 < r <= 2, delta > 0");
    PTS_REQUIRE(p->hist_bins == 0 || (p->hist_bins >= 2 && p->hist_bins <= 256), PTS_ERR_ARG,
                "irls_weights: hist_bins must be 0 or 2..256");
    const int64_t nq = Grid{H, W, p->w, p->stride}.nq();
    const float* factor =
        p->hist_bins ? hist_weight_factors(c, nn, nq, x, H, W, c->ex.as<float>(), c->Hz, c->Wz, p->w, p->hist_bins)
                     : nullptr;
    launch_irls_weights(c, dist, factor, nq, p->r, p->delta, weights);
  });
}

int pts_histogram_match(pts_ctx* c, float* x, int H, int W) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(x && H > 0 && W > 0, PTS_ERR_ARG, "histogram_match: bad image");
    PTS_REQUIRE(c->Hz > 0, PTS_ERR_STATE, "histogram_match: no exemplar");
    histogram_match(c, x, H, W, c->ex.as<float>(), c->Hz, c->Wz);
  });
}

int pts_energy(pts_ctx* c, const float* dist, int64_t nq, float r, float delta, double* E, double* E2) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(nq >= 0 && (nq == 0 || dist) && E && E2, PTS_ERR_ARG, "energy: bad arguments");
    PTS_REQUIRE(r > 0.f && r <= 2.f && delta > 0.f, PTS_ERR_ARG, "energy: need 0 < r <= 2, delta > 0");
    float* out = c->buf<float>("energy_out", 2);
    float host[2] = {0.f, 0.f};
    if (nq > 0) {
      launch_energy(c, dist, nq, r, delta, out);
      PTS_HIP(hipMemcpyAsync(host, out, 8, hipMemcpyDeviceToHost, c->stream));
      PTS_HIP(hipStreamSynchronize(c->stream));
    }
    *E = host[0];
    *E2 = host[1];
  });
}

int pts_energy_device(pts_ctx* c, const float* dist, int64_t nq, float r, float delta, float* out) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(nq >= 0 && (nq == 0 || dist) && out, PTS_ERR_ARG, "energy_device: bad arguments");
    PTS_REQUIRE(r > 0.f && r <= 2.f && delta > 0.f, PTS_ERR_ARG, "energy_device: need 0 < r <= 2, delta > 0");
    // a fill kernel, not a memset node, so that a caller may capture the call
    if (nq > 0) launch_energy(c, dist, nq, r, delta, out);
    else launch_zero_i32(c, reinterpret_cast<int32_t*>(out), 2);
  });
}

int pts_energy_device_noalloc(pts_ctx* c, const float* dist, int64_t nq, float r, float delta, float* out) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(nq >= 0 && (nq == 0 || dist) && out, PTS_ERR_ARG, "energy_device_noalloc: bad arguments");
    PTS_REQUIRE(r > 0.f && r <= 2.f && delta > 0.f, PTS_ERR_ARG,
                "energy_device_noalloc: need 0 < r <= 2, delta > 0");
    if (nq > 0) launch_energy_scratch(c, dist, nq, r, delta, out, c->energy_scratch);
    else launch_zero_i32(c, reinterpret_cast<int32_t*>(out), 2);
  });
}

// ---------------------------------------------------------------- multiscale helpers

int pts_exemplar_pyramid_level(pts_ctx* c, int levels, int level, float gw, float* out) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(out, PTS_ERR_ARG, "pyramid: null output");
    PTS_REQUIRE(c->Hz > 0, PTS_ERR_STATE, "pyramid: no exemplar");
    PTS_REQUIRE(levels >= 1 && levels <= 8 && level >= 0 && level < levels, PTS_ERR_ARG, "pyramid: bad level");
    int h = 0, w = 0;
    const float* src = pyramid_level(c, levels, level, gw, &h, &w);
    PTS_HIP(hipMemcpyAsync(out, src, (size_t)h * w * 16, hipMemcpyDeviceToDevice, c->stream));
  });
}

int pts_upsample2(pts_ctx* c, const float* x, int H, int W, float gw, float* out) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(x && out && H > 0 && W > 0, PTS_ERR_ARG, "upsample2: bad arguments");
    launch_upsample2(c, x, H, W, gw, out);
  });
}

int pts_solve(pts_ctx* c, const pts_solve_params* p, const float* x0, int H0, int W0, float* x, int H, int W,
              pts_solve_trace* tr) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(p && x0 && x, PTS_ERR_ARG, "solve: null argument");
    PTS_REQUIRE(H0 > 0 && W0 > 0, PTS_ERR_ARG, "solve: bad image size");
    PTS_REQUIRE(count_nonfinite(c, x0, (int64_t)H0 * W0 * 4) == 0, PTS_ERR_ARG,
                "solve: the initial output holds non-finite values");
    run_solve(c, *p, x0, H0, W0, x, H, W, tr);
  });
}

// ---------------------------------------------------------------- host utilities

int pts_eig_sym_top(const double* C, int n, int d, double* evals, double* evecs, int nthreads) {
  if (!C || !evals || !evecs || n <= 0 || d <= 0 || d > n) return PTS_ERR_ARG;
  try {
    return pts::eig_sym_top(C, n, d, evals, evecs, nthreads) == 0 ? PTS_OK : PTS_ERR_ARG;
  } catch (...) {
    return PTS_ERR_OOM;
  }
}

// ---------------------------------------------------------------- profiling

int pts_profile_enable(pts_ctx* c, int on) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    c->prof_drain();
    c->prof_table.clear();
    c->prof_order.clear();
    c->prof_on = on != 0;
  });
}

int pts_profile_count(pts_ctx* c, int* count) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    PTS_REQUIRE(count, PTS_ERR_ARG, "profile_count: null");
    c->prof_drain();
    *count = (int)c->prof_order.size();
  });
}

int pts_profile_read(pts_ctx* c, int i, char* name, int cap, double* total_ms, int64_t* launches) {
  CTX_REQUIRED(c);
  return guard(c, [&] {
    c->prof_drain();
    PTS_REQUIRE(i >= 0 && i < (int)c->prof_order.size(), PTS_ERR_ARG, "profile_read: index out of range");
    const std::string& nm = c->prof_order[i];
    const ProfEntry& e = c->prof_table[nm];
    if (name && cap > 0) {
      std::strncpy(name, nm.c_str(), (size_t)cap - 1);
      name[cap - 1] = 0;
    }
    if (total_ms) *total_ms = e.total_ms;
    if (launches) *launches = e.launches;
  });
}

}  // extern "C"
