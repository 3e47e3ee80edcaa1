// Index build: PCA basis + hierarchical k-means tree (Methodology 2.2).
//
// The covariance of all exemplar windows is accumulated on the GPU in FP64
// and eigen-decomposed on the host in FP64; the exemplar windows are then
// projected (FP32) and a k-means tree is grown breadth first.  Every tree
// level runs its splits together: k-means++ seeding (the seeding draws are
// made on the host from the GPU's running minimum distances), then Lloyd
// iterations whose assignment and centroid sums run on the GPU, until no
// assignment changes or the iteration limit is reached.  A node becomes a
// leaf at the depth limit (none with depth -1: the paper's own rule) or when
// it holds fewer members than the branching factor (the paper stops below k
// members).  Empty clusters are dropped; a node whose split leaves a single
// cluster (its points cannot be told apart) stays a leaf, so that the
// uncapped growth ends.
// Children are kept in cluster order and a node's members in ascending id.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "api_internal.hpp"
#include "eig.hpp"

namespace pts {

int padded_dims(int d) {
  static const int opts[] = {16, 24, 32, 48, 64, 96, 128};
  for (int o : opts)
    if (d <= o) return o;
  fail(PTS_ERR_UNSUPPORTED, "PCA dims above 128");
}

namespace {

struct Rng {  // xoshiro256** seeded through splitmix64
  uint64_t s[4];
  explicit Rng(uint64_t seed) {
    uint64_t z = seed;
    for (auto& v : s) {
      z += 0x9E3779B97F4A7C15ull;
      uint64_t t = z;
      t = (t ^ (t >> 30)) * 0xBF58476D1CE4E5B9ull;
      t = (t ^ (t >> 27)) * 0x94D049BB133111EBull;
      v = t ^ (t >> 31);
    }
  }
  static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  uint64_t next() {
    const uint64_t r = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return r;
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  int64_t below(int64_t n) { return (int64_t)(uniform() * (double)n) % n; }
};

template <class T>
T* upload(Ctx* c, DevMem& m, const std::vector<T>& v) {
  T* p = static_cast<T*>(m.ensure(c, std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) {
    PTS_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    PTS_HIP(hipStreamSynchronize(c->stream));  // the host vector may be a temporary
  }
  return p;
}

template <class T>
void download(Ctx* c, std::vector<T>& v, const T* p, size_t n) {
  v.resize(n);
  if (n) PTS_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  PTS_HIP(hipStreamSynchronize(c->stream));
}

struct Node {
  int64_t begin, count;  // range in the member array
  int depth;
  int first_child = 0, n_children = 0;
  std::vector<double> centroid;
};

// Grows the tree over the projected points P (device, [N][dp], original id
// order).  Returns host tree arrays; `members` ends up in leaf order.
void grow_tree(Ctx* c, const float* P, int64_t N, int d, int dp, int branching, int depth, int max_iter,
               uint64_t seed, HostTree& out) {
  std::vector<Node> nodes;
  nodes.push_back(Node{0, N, 0, 0, 0, std::vector<double>(d, 0.0)});
  std::vector<int32_t> members(N);
  std::iota(members.begin(), members.end(), 0);
  Rng rng(seed);
  if (max_iter <= 0) max_iter = 50;

  DevMem d_members, d_seg_of, d_cent_off, d_k, d_cents, d_assign, d_mind, d_ids, d_cand, d_sums, d_counts, d_changed;

  for (int level = 0; depth < 0 || level < depth; ++level) {
    std::vector<int> segs;
    for (int i = 0; i < (int)nodes.size(); ++i)
      if (nodes[i].depth == level && nodes[i].n_children == 0 && nodes[i].count >= branching) segs.push_back(i);
    if (segs.empty()) break;
    const int ns = (int)segs.size();
    // active members, back to back per segment
    std::vector<int32_t> act, seg_of;
    std::vector<int64_t> seg_begin(ns), seg_cnt(ns);
    for (int s = 0; s < ns; ++s) {
      const Node& nd = nodes[segs[s]];
      seg_begin[s] = (int64_t)act.size();
      seg_cnt[s] = nd.count;
      for (int64_t i = 0; i < nd.count; ++i) {
        act.push_back(members[nd.begin + i]);
        seg_of.push_back(s);
      }
    }
    const int64_t m = (int64_t)act.size();
    const int32_t* dm = upload(c, d_members, act);
    const int32_t* dso = upload(c, d_seg_of, seg_of);
    float* mind = static_cast<float*>(d_mind.ensure(c, (size_t)m * 4));
    float* cand = static_cast<float*>(d_cand.ensure(c, (size_t)ns * dp * 4));
    int32_t* ids_dev = static_cast<int32_t*>(d_ids.ensure(c, (size_t)ns * 4));

    // ---- k-means++ seeding
    std::vector<std::vector<int32_t>> chosen(ns);
    std::vector<int32_t> pick(ns);
    std::vector<float> mind_h;
    for (int j = 0; j < branching; ++j) {
      if (j == 0) {
        for (int s = 0; s < ns; ++s) pick[s] = act[seg_begin[s] + rng.below(seg_cnt[s])];
      } else {
        download(c, mind_h, mind, (size_t)m);
        for (int s = 0; s < ns; ++s) {
          double tot = 0.0;
          for (int64_t i = 0; i < seg_cnt[s]; ++i) tot += (double)mind_h[seg_begin[s] + i];
          int64_t sel = seg_cnt[s] - 1;
          if (tot > 0.0) {
            const double u = rng.uniform() * tot;
            double run = 0.0;
            for (int64_t i = 0; i < seg_cnt[s]; ++i) {
              run += (double)mind_h[seg_begin[s] + i];
              if (run > u) {
                sel = i;
                break;
              }
            }
          } else {
            sel = rng.below(seg_cnt[s]);
          }
          pick[s] = act[seg_begin[s] + sel];
        }
      }
      for (int s = 0; s < ns; ++s) chosen[s].push_back(pick[s]);
      PTS_HIP(hipMemcpyAsync(ids_dev, pick.data(), (size_t)ns * 4, hipMemcpyHostToDevice, c->stream));
      PTS_HIP(hipStreamSynchronize(c->stream));
      launch_permute_rows(c, P, ids_dev, ns, dp, cand, nullptr);
      if (j + 1 < branching) launch_kmeans_mindist(c, P, dp, dm, m, dso, cand, mind, j == 0 ? 1 : 0);
    }

    // ---- Lloyd
    std::vector<int32_t> cent_off(ns), kk(ns, branching);
    std::vector<int32_t> all_ids;
    for (int s = 0; s < ns; ++s) {
      cent_off[s] = s * branching;
      for (int j = 0; j < branching; ++j) all_ids.push_back(chosen[s][j]);
    }
    int ncent = ns * branching;
    float* cents = static_cast<float*>(d_cents.ensure(c, (size_t)ncent * dp * 4));
    upload(c, d_ids, all_ids);
    launch_permute_rows(c, P, d_ids.as<int32_t>(), ncent, dp, cents, nullptr);
    std::vector<std::vector<double>> cent_h(ncent);  // FP64 centroids of the current list
    int32_t* assign = static_cast<int32_t*>(d_assign.ensure(c, (size_t)m * 4));
    {
      std::vector<int32_t> neg(m, -1);
      PTS_HIP(hipMemcpyAsync(assign, neg.data(), (size_t)m * 4, hipMemcpyHostToDevice, c->stream));
      PTS_HIP(hipStreamSynchronize(c->stream));
    }
    int32_t* changed = static_cast<int32_t*>(d_changed.ensure(c, 4));
    std::vector<unsigned long long> sums_h;
    std::vector<int32_t> counts_h;
    // Runs until an iteration drops no cluster (every drop removes a centroid,
    // so this ends): the final assignment must use the final numbering.
    for (int it = 0;; ++it) {
      upload(c, d_cent_off, cent_off);
      upload(c, d_k, kk);
      launch_zero_i32(c, changed, 1);
      launch_kmeans_assign(c, P, dp, dm, m, dso, d_cent_off.as<int32_t>(), d_k.as<int32_t>(), cents, assign, changed);
      unsigned long long* sums =
          static_cast<unsigned long long*>(d_sums.ensure(c, (size_t)ncent * dp * sizeof(unsigned long long)));
      int32_t* counts = static_cast<int32_t*>(d_counts.ensure(c, (size_t)ncent * 4));
      launch_zero_i32(c, reinterpret_cast<int32_t*>(sums), (int64_t)ncent * dp * 2);
      launch_zero_i32(c, counts, ncent);
      launch_kmeans_accumulate(c, P, dp, dm, m, dso, d_cent_off.as<int32_t>(), assign, sums, counts, ncent);
      int32_t changed_h = 0;
      PTS_HIP(hipMemcpyAsync(&changed_h, changed, 4, hipMemcpyDeviceToHost, c->stream));
      download(c, sums_h, sums, (size_t)ncent * dp);
      download(c, counts_h, counts, (size_t)ncent);
      // new centroids; drop empty clusters
      bool dropped = false;
      std::vector<int32_t> new_off(ns), new_k(ns);
      std::vector<std::vector<double>> new_cent;
      for (int s = 0; s < ns; ++s) {
        new_off[s] = (int32_t)new_cent.size();
        int k2 = 0;
        for (int j = 0; j < kk[s]; ++j) {
          const int ci = cent_off[s] + j;
          if (counts_h[ci] == 0) {
            dropped = true;
            continue;
          }
          std::vector<double> cc(d);
          for (int k = 0; k < d; ++k)
            cc[k] = (double)(long long)sums_h[(size_t)ci * dp + k] / (1073741824.0 * (double)counts_h[ci]);
          new_cent.push_back(std::move(cc));
          ++k2;
        }
        new_k[s] = k2;
      }
      ncent = (int)new_cent.size();
      cent_off = new_off;
      kk = new_k;
      cent_h = new_cent;
      std::vector<float> cf((size_t)ncent * dp, 0.f);
      for (int ci = 0; ci < ncent; ++ci)
        for (int k = 0; k < d; ++k) cf[(size_t)ci * dp + k] = (float)cent_h[ci][k];
      cents = upload(c, d_cents, cf);
      const bool converged = (it > 0 && changed_h == 0 && !dropped);
      if (converged || (it + 1 >= max_iter && !dropped)) break;
    }
    // final assignment against the final centroids was the last assign pass
    std::vector<int32_t> assign_h;
    download(c, assign_h, assign, (size_t)m);
    // partition every segment into its children (stable: ascending ids kept)
    for (int s = 0; s < ns; ++s) {
      Node& nd = nodes[segs[s]];
      const int k = kk[s];
      if (k < 2) continue;  // k-means left one cluster (identical points): the node stays a leaf
      nd.first_child = (int)nodes.size();
      nd.n_children = k;
      std::vector<std::vector<int32_t>> parts(k);
      for (int64_t i = 0; i < seg_cnt[s]; ++i) {
        const int a = assign_h[seg_begin[s] + i];
        parts[a].push_back(act[seg_begin[s] + i]);
      }
      int64_t pos = nd.begin;
      const int64_t nd_begin = nd.begin;
      (void)nd_begin;
      for (int j = 0; j < k; ++j) {
        Node ch{pos, (int64_t)parts[j].size(), level + 1, 0, 0, cent_h[cent_off[s] + j]};
        std::copy(parts[j].begin(), parts[j].end(), members.begin() + pos);
        pos += (int64_t)parts[j].size();
        nodes.push_back(std::move(ch));
      }
    }
  }

  // flatten
  const int nn = (int)nodes.size();
  out.d = d;
  out.centroids.assign((size_t)nn * d, 0.0);
  out.first_child.assign(nn, 0);
  out.n_children.assign(nn, 0);
  out.leaf_of_node.assign(nn, -1);
  out.leaf_off.assign(1, 0);
  out.perm.clear();
  out.perm.reserve(N);
  for (int i = 0; i < nn; ++i) {
    const Node& nd = nodes[i];
    for (int k = 0; k < d; ++k) out.centroids[(size_t)i * d + k] = nd.centroid[k];
    out.first_child[i] = nd.first_child;
    out.n_children[i] = nd.n_children;
    if (nd.n_children == 0) {
      out.leaf_of_node[i] = out.n_leaves();
      for (int64_t j = 0; j < nd.count; ++j) out.perm.push_back(members[nd.begin + j]);
      out.leaf_off.push_back((int64_t)out.perm.size());
    }
  }
}

int tree_depth(const HostTree& t) {
  std::vector<int> dep(t.n_nodes(), 0);
  int mx = 0;
  for (int i = 0; i < t.n_nodes(); ++i)
    for (int j = 0; j < t.n_children[i]; ++j) {
      dep[t.first_child[i] + j] = dep[i] + 1;
      mx = std::max(mx, dep[i] + 1);
    }
  return mx;
}

// Device copies of everything the search needs, from the host basis/tree and
// the exemplar projected in original order (zorig, [N][dp]).
void finalize_device(Ctx* c, Index& ix, ExView ex, const float* zorig, bool make_bf16) {
  const int64_t N = ix.N;
  const HostTree& t = ix.tree;
  std::vector<float> cf((size_t)t.n_nodes() * ix.dp, 0.f);
  for (int i = 0; i < t.n_nodes(); ++i)
    for (int k = 0; k < ix.d; ++k) cf[(size_t)i * ix.dp + k] = (float)t.centroids[(size_t)i * ix.d + k];
  upload(c, ix.cent, cf);
  upload(c, ix.first_child, t.first_child);
  upload(c, ix.n_children, t.n_children);
  upload(c, ix.leaf_of_node, t.leaf_of_node);
  std::vector<int32_t> lo32(t.leaf_off.begin(), t.leaf_off.end());
  upload(c, ix.leaf_off, lo32);
  std::vector<int32_t> by_rows(t.n_leaves());
  for (int l = 0; l < t.n_leaves(); ++l) by_rows[l] = l;
  std::stable_sort(by_rows.begin(), by_rows.end(), [&](int a, int b) {
    return t.leaf_off[a + 1] - t.leaf_off[a] > t.leaf_off[b + 1] - t.leaf_off[b];
  });
  upload(c, ix.leaf_by_rows, by_rows);
  upload(c, ix.perm, t.perm);
  std::vector<int32_t> leaf_of(N, -1);
  for (int l = 0; l < t.n_leaves(); ++l)
    for (int64_t j = t.leaf_off[l]; j < t.leaf_off[l + 1]; ++j) leaf_of[t.perm[j]] = l;
  upload(c, ix.leaf_of_ex, leaf_of);
  float* zl = static_cast<float*>(ix.zproj.ensure(c, (size_t)N * ix.dp * 4));
  float* zn = static_cast<float*>(ix.znorm.ensure(c, (size_t)N * 4));
  launch_permute_rows(c, zorig, ix.perm.as<int32_t>(), N, ix.dp, zl, zn);
  ix.has_bf16 = make_bf16;
  float* cn = c->buf<float>("ix_cnorm", (size_t)N);
  launch_centered_norm(c, ex.img, ex.Hz, ex.Wz, ix.w, ix.mu_f.as<float>(), cn);
  float* zr = static_cast<float*>(ix.zres.ensure(c, (size_t)N * 4));
  if (make_bf16) {
    ix.dk = (int)round_up(ix.d, 32);
    uint16_t* zb = static_cast<uint16_t*>(ix.zbf.ensure(c, (size_t)N * ix.dk * 2));
    float* zbn = static_cast<float*>(ix.zbnorm.ensure(c, (size_t)N * 4));
    launch_to_bf16_rows(c, zl, N, ix.dp, ix.dk, zb, zbn);
    float* zbr = static_cast<float*>(ix.zbnorm_res.ensure(c, (size_t)N * 4));
    launch_residual(c, cn, ix.perm.as<int32_t>(), zn, zbn, N, zr, zbr);
  } else {
    launch_residual(c, cn, ix.perm.as<int32_t>(), zn, nullptr, N, zr, nullptr);
  }
  ix.max_depth = tree_depth(t);
  PTS_HIP(hipStreamSynchronize(c->stream));
  ix.valid = true;
}

void upload_basis(Ctx* c, Index& ix) {
  std::vector<float> muf(ix.D), bf((size_t)ix.D * ix.dp, 0.f);
  for (int j = 0; j < ix.D; ++j) muf[j] = (float)ix.mu[j];
  for (int j = 0; j < ix.D; ++j)
    for (int k = 0; k < ix.d; ++k) bf[(size_t)j * ix.dp + k] = (float)ix.basis[(size_t)j * ix.d + k];
  upload(c, ix.mu_f, muf);
  upload(c, ix.basis_f, bf);
}

}  // namespace

void build_index_on(Ctx* c, ExView ex, const pts_index_params& p, Index& ix, pts_index_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  PTS_REQUIRE(p.w >= 2 && p.w <= 32 && p.w % 2 == 0, PTS_ERR_UNSUPPORTED, "index: w must be even, 2..32");
  PTS_REQUIRE(p.w <= ex.Hz && p.w <= ex.Wz, PTS_ERR_ARG, "index: window larger than the exemplar");
  PTS_REQUIRE(p.pca_dims >= 0 && p.pca_dims <= 128, PTS_ERR_UNSUPPORTED, "index: pca_dims must be 0..128");
  PTS_REQUIRE(p.pca_dims > 0 || (p.variance_target > 0.0 && p.variance_target <= 1.0), PTS_ERR_ARG,
              "index: variance_target must be in (0, 1]");
  PTS_REQUIRE(p.branching >= 2 && p.branching <= 64, PTS_ERR_UNSUPPORTED, "index: branching must be 2..64");
  PTS_REQUIRE(p.depth >= -1 && p.depth <= 8, PTS_ERR_UNSUPPORTED, "index: depth must be -1 (no cap) or 0..8");
  const int w = p.w, D = 4 * w * w;
  const int64_t N = (int64_t)(ex.Hz - w + 1) * (ex.Wz - w + 1);
  PTS_REQUIRE(N < ((int64_t)1 << 31) - 1, PTS_ERR_UNSUPPORTED, "index: too many exemplar windows");
  ix.valid = false;

  // ---- PCA: FP64 covariance on the GPU, FP64 eigensolve on the host
  double* dmean = c->buf<double>("ix_mean", D);
  double* dcov = c->buf<double>("ix_cov", (size_t)D * D);
  launch_mean_cov_image(c, ex.img, ex.Hz, ex.Wz, w, dmean, dcov);
  std::vector<double> mean, cov;
  download(c, mean, dmean, D);
  download(c, cov, dcov, (size_t)D * D);
  double tr = 0.0;
  for (int j = 0; j < D; ++j) tr += cov[(size_t)j * D + j];
  const int dmax = std::min(D, 128);
  int d = p.pca_dims > 0 ? std::min(p.pca_dims, D) : dmax;
  std::vector<double> ev(d), vec((size_t)D * d);
  PTS_REQUIRE(eig_sym_top(cov.data(), D, d, ev.data(), vec.data(), 0) == 0, PTS_ERR_ARG, "eigensolve failed");
  if (p.pca_dims == 0) {  // smallest d reaching the variance target
    double run = 0.0;
    int dd = d;
    for (int k = 0; k < d; ++k) {
      run += ev[k];
      if (tr <= 0.0 || run / tr >= p.variance_target - 1e-12) {
        dd = k + 1;
        break;
      }
    }
    std::vector<double> v2((size_t)D * dd);
    for (int j = 0; j < D; ++j)
      for (int k = 0; k < dd; ++k) v2[(size_t)j * dd + k] = vec[(size_t)j * d + k];
    vec.swap(v2);
    ev.resize(dd);
    d = dd;
  }
  ix.w = w;
  ix.D = D;
  ix.d = d;
  ix.dp = padded_dims(d);
  ix.N = N;
  ix.mu = mean;
  ix.basis = vec;
  ix.eig = ev;
  ix.trace = tr;
  upload_basis(c, ix);

  // ---- projection of every exemplar window (original id order)
  float* zorig = c->buf<float>("ix_zorig", (size_t)N * ix.dp);
  launch_project_image(c, ex.img, ex.Hz, ex.Wz, w, 1, false, ix.mu_f.as<float>(), ix.basis_f.as<float>(), ix.dp,
                       zorig);

  // ---- tree
  grow_tree(c, zorig, N, d, ix.dp, p.branching, p.depth, p.kmeans_max_iter, p.seed, ix.tree);
  finalize_device(c, ix, ex, zorig, p.make_bf16 != 0);

  if (info) {
    info->N = N;
    info->D = D;
    info->d = d;
    double s = 0.0;
    for (double v : ev) s += v;
    info->retained_variance = tr > 0.0 ? s / tr : 1.0;
    info->n_nodes = ix.tree.n_nodes();
    info->n_leaves = ix.tree.n_leaves();
    int64_t mn = N, mx = 0;
    for (int l = 0; l < ix.tree.n_leaves(); ++l) {
      const int64_t sz = ix.tree.leaf_off[l + 1] - ix.tree.leaf_off[l];
      mn = std::min(mn, sz);
      mx = std::max(mx, sz);
    }
    info->leaf_min = mn;
    info->leaf_max = mx;
    info->leaf_mean = (double)N / std::max(1, ix.tree.n_leaves());
    info->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
}

void export_index(Ctx* c, const Index& ix, pts_index_host* o) {
  (void)c;
  PTS_REQUIRE(ix.valid, PTS_ERR_STATE, "export_index: no index");
  const HostTree& t = ix.tree;
  o->w = ix.w;
  o->D = ix.D;
  o->d = ix.d;
  o->N = ix.N;
  o->n_nodes = t.n_nodes();
  o->n_leaves = t.n_leaves();
  if (!o->mu || !o->basis || !o->centroids || !o->first_child || !o->n_children || !o->leaf_of_node || !o->leaf_off ||
      !o->perm)
    return;  // sizes only
  std::copy(ix.mu.begin(), ix.mu.end(), o->mu);
  std::copy(ix.basis.begin(), ix.basis.end(), o->basis);
  if (o->eigenvalues) std::copy(ix.eig.begin(), ix.eig.end(), o->eigenvalues);
  std::copy(t.centroids.begin(), t.centroids.end(), o->centroids);
  std::copy(t.first_child.begin(), t.first_child.end(), o->first_child);
  std::copy(t.n_children.begin(), t.n_children.end(), o->n_children);
  std::copy(t.leaf_of_node.begin(), t.leaf_of_node.end(), o->leaf_of_node);
  std::copy(t.leaf_off.begin(), t.leaf_off.end(), o->leaf_off);
  std::copy(t.perm.begin(), t.perm.end(), o->perm);
}

void import_index(Ctx* c, ExView ex, const pts_index_host& in, int make_bf16, Index& ix) {
  PTS_REQUIRE(in.w >= 2 && in.w <= 32 && in.w % 2 == 0, PTS_ERR_ARG, "import: bad w");
  const int D = 4 * in.w * in.w;
  const int64_t N = (int64_t)(ex.Hz - in.w + 1) * (ex.Wz - in.w + 1);
  PTS_REQUIRE(in.w <= ex.Hz && in.w <= ex.Wz && in.N == N && in.D == D, PTS_ERR_ARG,
              "import: w/N/D do not match the exemplar");
  PTS_REQUIRE(in.d >= 1 && in.d <= 128 && in.d <= D, PTS_ERR_ARG, "import: d must be 1..128");
  PTS_REQUIRE(in.n_nodes >= 1 && in.n_leaves >= 1 && in.n_leaves <= in.n_nodes, PTS_ERR_ARG, "import: bad node counts");
  PTS_REQUIRE(in.mu && in.basis && in.centroids && in.first_child && in.n_children && in.leaf_of_node && in.leaf_off &&
                  in.perm,
              PTS_ERR_ARG, "import: null array");
  const int nn = in.n_nodes, nl = in.n_leaves;
  // structure checks: children after their parent, within range; leaves
  // numbered 0..nl-1 once each; offsets monotone; perm a permutation
  std::vector<char> leaf_seen(nl, 0);
  for (int i = 0; i < nn; ++i) {
    const int f = in.first_child[i], k = in.n_children[i], l = in.leaf_of_node[i];
    if (k == 0) {
      PTS_REQUIRE(l >= 0 && l < nl && !leaf_seen[l], PTS_ERR_ARG, "import: bad leaf numbering");
      leaf_seen[l] = 1;
    } else {
      PTS_REQUIRE(k > 0 && f > i && (int64_t)f + k <= nn && l == -1, PTS_ERR_ARG, "import: bad child range");
    }
  }
  PTS_REQUIRE(in.leaf_off[0] == 0 && in.leaf_off[nl] == N, PTS_ERR_ARG, "import: leaf offsets must span [0, N)");
  for (int l = 0; l < nl; ++l)
    PTS_REQUIRE(in.leaf_off[l + 1] > in.leaf_off[l], PTS_ERR_ARG, "import: empty or decreasing leaf");
  std::vector<char> seen(N, 0);
  for (int64_t i = 0; i < N; ++i) {
    const int32_t e = in.perm[i];
    PTS_REQUIRE(e >= 0 && e < N && !seen[e], PTS_ERR_ARG, "import: perm is not a permutation");
    seen[e] = 1;
  }
  ix.valid = false;
  ix.w = in.w;
  ix.D = D;
  ix.d = in.d;
  ix.dp = padded_dims(in.d);
  ix.N = N;
  ix.mu.assign(in.mu, in.mu + D);
  ix.basis.assign(in.basis, in.basis + (size_t)D * in.d);
  ix.eig.assign(in.d, 0.0);
  if (in.eigenvalues) ix.eig.assign(in.eigenvalues, in.eigenvalues + in.d);
  HostTree& t = ix.tree;
  t.d = in.d;
  t.centroids.assign(in.centroids, in.centroids + (size_t)nn * in.d);
  t.first_child.assign(in.first_child, in.first_child + nn);
  t.n_children.assign(in.n_children, in.n_children + nn);
  t.leaf_of_node.assign(in.leaf_of_node, in.leaf_of_node + nn);
  t.leaf_off.assign(in.leaf_off, in.leaf_off + nl + 1);
  t.perm.assign(in.perm, in.perm + N);
  upload_basis(c, ix);
  float* zorig = c->buf<float>("ix_zorig", (size_t)N * ix.dp);
  launch_project_image(c, ex.img, ex.Hz, ex.Wz, ix.w, 1, false, ix.mu_f.as<float>(), ix.basis_f.as<float>(), ix.dp,
                       zorig);
  finalize_device(c, ix, ex, zorig, make_bf16 != 0);
}

}  // namespace pts
