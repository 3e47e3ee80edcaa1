// Internal runtime of libpts: error handling, device memory, the context,
// kernel-launch profiling.  Not part of the ABI (see include/pts.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pts.h"

namespace pts {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

#define PTS_HIP(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      ::pts::fail(e_ == hipErrorOutOfMemory ? PTS_ERR_OOM : PTS_ERR_HIP,                           \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                              \
  } while (0)

#define PTS_REQUIRE(cond, code, msg)                                                               \
  do {                                                                                             \
    if (!(cond)) ::pts::fail(code, msg);                                                           \
  } while (0)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

struct Ctx;

// A device allocation owned by the context (freed through the context's
// allocator).  Grows on demand; contents are not preserved across growth.
struct DevMem {
  Ctx* ctx = nullptr;
  void* ptr = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem();
  void reset();
  void* ensure(Ctx* c, size_t nbytes);  // returns ptr with at least nbytes
  template <class T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

// Tree arrays of the host index (breadth-first nodes, see include/pts.h).
struct HostTree {
  int d = 0;
  std::vector<double> centroids;  // [n_nodes][d]
  std::vector<int32_t> first_child, n_children, leaf_of_node;
  std::vector<int64_t> leaf_off;  // [n_leaves + 1]
  std::vector<int32_t> perm;      // [N]
  int n_nodes() const { return (int)first_child.size(); }
  int n_leaves() const { return (int)leaf_off.size() - 1; }
};

struct Index {
  bool valid = false;
  int w = 0, D = 0, d = 0, dp = 0, dk = 0;  // dp: d padded to 4; dk: padded to 32 (bf16 K)
  int64_t N = 0;
  std::vector<double> mu, basis, eig;  // host FP64: [D], [D][d], [d]
  double trace = 0.0;
  HostTree tree;
  int max_depth = 0;
  bool has_bf16 = false;
  // device
  DevMem mu_f, basis_f;        // f32 [D], [D][dp] (zero padded columns)
  DevMem zproj;                // f32 [N][dp], leaf order
  DevMem znorm;                // f32 [N] ||z'||^2 (leaf order)
  DevMem zbf;                  // bf16 [N][dk], leaf order
  DevMem zbnorm;               // f32 [N] ||bf16(z')||^2
  DevMem zres;                 // f32 [N] ||z - mu||^2 - ||z'||^2: energy outside the PCA subspace
  DevMem zbnorm_res;           // f32 [N] zbnorm + zres
  DevMem perm;                 // i32 [N] leaf position -> exemplar id
  DevMem leaf_of_ex;           // i32 [N] exemplar id -> leaf
  DevMem leaf_off;             // i32 [n_leaves + 1]
  DevMem leaf_by_rows;         // i32 [n_leaves] leaves by member count, largest first (ties: lower id)
  DevMem cent;                 // f32 [n_nodes][dp]
  DevMem first_child, n_children, leaf_of_node;  // i32 [n_nodes]
};

struct Mlp {
  bool valid = false;
  int n_in = 0, h = 0, n_out = 0;
  int64_t n_params = 0;
  DevMem params;      // f32 packed W1, b1, W2, b2, W3, b3
  DevMem in_scale;    // f32 [n_in]
  DevMem adam_m, adam_v;
  int64_t adam_t = 0;
  uint64_t version = 0;               // bumped on every weight change
  DevMem w1b, w2b, w3b;               // bf16 copies for inference
  DevMem b3p;                         // output bias padded to 32 rows (-FLT_MAX)
  uint64_t bf_version = ~0ull;
};

struct ProfEntry {
  double total_ms = 0.0;
  int64_t launches = 0;
};

// the guidance a solve writes at every level: the row guidance, or (on) the
// perspective scale map of a slant and a tilt (radians)
struct ScaleSpec {
  bool on = false;
  double slant = 0.0, tilt = 0.0;
  bool operator==(const ScaleSpec& o) const { return on == o.on && slant == o.slant && tilt == o.tilt; }
  bool operator!=(const ScaleSpec& o) const { return !(*this == o); }
};

struct Ctx {
  int device = 0;
  int n_cu = 256;  // compute units of the device
  float* energy_scratch = nullptr;  // the device's fixed energy scratch (set at creation)
  hipStream_t stream = nullptr;
  pts_alloc alloc{};
  bool has_alloc = false;
  std::string last_error;

  // exemplar
  DevMem ex;  // f32 [Hz][Wz][4]
  int Hz = 0, Wz = 0;
  uint64_t ex_version = 0;
  // an exemplar set from 8-bit RGB also keeps that form: ex_pk [Hz][Wz] =
  // R | G << 8 | B << 16 and ex_srow [Hz] = its guidance value per row, from
  // which the gathers rebuild exactly the floats of ex at a quarter of the bytes
  DevMem ex_pk, ex_srow;
  bool ex_packed = false;

  Index index;
  Mlp mlp;

  // materialised exemplar windows cache (for the exact full-D search)
  DevMem exwin;
  int exwin_w = 0;
  uint64_t exwin_version = ~0ull;

  // exemplar pyramid (coarse to fine), rebuilt when the exemplar changes
  uint64_t pyr_version = ~0ull;
  int pyr_levels = 0;
  float pyr_gw = -1.f;
  ScaleSpec pyr_scale;
  std::vector<std::unique_ptr<DevMem>> pyr_img;
  std::vector<int> pyr_h, pyr_w;

  // named scratch
  std::map<std::string, std::unique_ptr<DevMem>> scratch;
  template <class T>
  T* buf(const char* name, size_t count) {
    auto& p = scratch[name];
    if (!p) p.reset(new DevMem());
    return static_cast<T*>(p->ensure(this, count * sizeof(T) + 256));
  }

  // profiling
  bool prof_on = false;
  std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
  std::vector<hipEvent_t> prof_free;
  std::map<std::string, ProfEntry> prof_table;
  std::vector<std::string> prof_order;
  void prof_begin(const char* name);
  void prof_end();
  void prof_drain();

  void* dalloc(size_t bytes);
  void dfree(void* p, size_t bytes);
  ~Ctx();
};

// Scoped launch bracket: records events around the kernels launched inside.
struct ProfScope {
  Ctx* c;
  ProfScope(Ctx* ctx, const char* name) : c(ctx) {
    if (c->prof_on) c->prof_begin(name);
  }
  ~ProfScope() {
    if (c->prof_on) c->prof_end();
  }
};

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(PTS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// geometry of the two window grids
struct Grid {
  int H, W, w, s;
  int rows() const { return (H - w) / s + 1; }
  int cols() const { return W / s; }
  int64_t nq() const { return (int64_t)rows() * cols(); }
};

void validate_grid(int H, int W, int w, int s);

}  // namespace pts
