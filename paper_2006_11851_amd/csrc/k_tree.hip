// Tree search kernels (Methodology 2.2: k-means search tree over the PCA-
// reduced neighbourhoods).
//
//  * descent: greedy, nearest child centroid at every level (ties to the
//    lowest child): the first level per query, then per bucket of queries
//    that share their level-1 node (that node's rows read once per wave);
//  * bucketing: counting sort of the queries by leaf, then a work list of
//    (leaf, 64-query chunk) tiles, so a leaf's members are streamed once per
//    64 queries instead of once per query;
//  * leaf scan (FP32): per tile, the 64 queries sit in registers (one per
//    lane, replicated in the block's 4 waves), the leaf's member rows stream
//    through LDS in chunks of 64, each wave takes every fourth member, and
//    the 4 partial winners are merged in LDS.  Direct form sum (q - z)^2;
//    ties go to the lowest exemplar id.
#include <cfloat>
#include <climits>

#include "kernels_bf16.hpp"
#include "device_util.hpp"

namespace pts {

// nearest child of `node` (ties to the lowest child); the centroid rows are
// read with the addresses the lanes hold (uniform for the root, so the
// compiler reads them through the scalar cache)
template <int DP>
__device__ __forceinline__ int nearest_child(const float (&qv)[DP], int f, int nc, const float* __restrict__ cent) {
  float best = FLT_MAX;
  int bj = 0;
  for (int j = 0; j < nc; ++j) {
    const float* cr = cent + (int64_t)(f + j) * DP;
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < DP; k += 4) {
      const float4 cv = *reinterpret_cast<const float4*>(cr + k);
      const float t0 = qv[k] - cv.x, t1 = qv[k + 1] - cv.y, t2 = qv[k + 2] - cv.z, t3 = qv[k + 3] - cv.w;
      acc = fmaf(t0, t0, acc);
      acc = fmaf(t1, t1, acc);
      acc = fmaf(t2, t2, acc);
      acc = fmaf(t3, t3, acc);
    }
    if (acc < best) {
      best = acc;
      bj = j;
    }
  }
  return f + bj;
}

// Descent in two kernels.  Level 1 (the root's children, the same rows for
// every lane) per entry; entries are then bucketed by the level-1 node they
// reached, and the rest runs per (node, 64 entries) tile with one wave per
// tile: the node is the same for the whole wave, so its children's rows are
// read once for all lanes through the scalar cache instead of by every lane
// from its own node.  Levels below the second follow each lane.  The
// arithmetic and tie rule are those of a plain per-query descent.
//
// Entry i is query list ? list[i] : i; with n_list, entries at or past
// *n_list are empty.  node1[i] = the level-1 node to continue from, or -1
// (empty entry, or the level-1 child is a leaf: its leaf is written here).
template <int DP>
__global__ __launch_bounds__(256) void k_descend_root(const float* __restrict__ Qp, const int32_t* __restrict__ list,
                                                      const int32_t* __restrict__ n_list, int64_t n,
                                                      const float* __restrict__ cent,
                                                      const int32_t* __restrict__ first_child,
                                                      const int32_t* __restrict__ n_children,
                                                      const int32_t* __restrict__ leaf_of_node,
                                                      int32_t* __restrict__ node1, int32_t* __restrict__ leaf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (n_list && i >= *n_list) {
    node1[i] = -1;
    return;
  }
  const int64_t q = list ? list[i] : i;
  float qv[DP];
#pragma unroll
  for (int k = 0; k < DP; k += 4) {
    const float4 v = *reinterpret_cast<const float4*>(Qp + q * DP + k);
    qv[k] = v.x;
    qv[k + 1] = v.y;
    qv[k + 2] = v.z;
    qv[k + 3] = v.w;
  }
  const int nc0 = n_children[0];
  const int node = nc0 > 0 ? nearest_child<DP>(qv, first_child[0], nc0, cent) : 0;
  const bool inner = n_children[node] > 0;
  node1[i] = inner ? node : -1;
  if (!inner) leaf[q] = leaf_of_node[node];
}

constexpr int DS_CHUNK = 64;  // entries per tile: one wave

template <int DP>
__global__ __launch_bounds__(256) void k_descend_tiles(const float* __restrict__ Qp, const int32_t* __restrict__ list,
                                                       const float* __restrict__ cent,
                                                       const int32_t* __restrict__ first_child,
                                                       const int32_t* __restrict__ n_children,
                                                       const int32_t* __restrict__ leaf_of_node,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ order,
                                                       const int2* __restrict__ tiles,
                                                       const int32_t* __restrict__ ntiles, int n_nodes,
                                                       int32_t* __restrict__ leaf) {
  const int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  if (t >= *ntiles) return;  // uniform per wave
  const int2 tile = tiles[t];
  const int node = tile.x;
  const int pos = tile.y + (int)(threadIdx.x & 63);
  if (pos >= min(off[node + 1], tile.y + DS_CHUNK)) return;
  const int i = order[pos];
  const int64_t q = list ? list[i] : i;
  float qv[DP];
#pragma unroll
  for (int k = 0; k < DP; k += 4) {
    const float4 v = *reinterpret_cast<const float4*>(Qp + q * DP + k);
    qv[k] = v.x;
    qv[k + 1] = v.y;
    qv[k + 2] = v.z;
    qv[k + 3] = v.w;
  }
  int nd = nearest_child<DP>(qv, first_child[node], n_children[node], cent);
  for (int step = 0; step < n_nodes; ++step) {  // bounded: no path is longer than the node count
    const int nc = n_children[nd];
    if (nc == 0) break;
    nd = nearest_child<DP>(qv, first_child[nd], nc, cent);
  }
  leaf[q] = leaf_of_node[nd];
}

// Descent restricted to queries whose margin is below thr: a compaction
// pass lists them, the descent runs over the list (its length read on the
// device), and every other query gets leaf -1.
__global__ __launch_bounds__(256) void k_compact_low(const float* __restrict__ margin, int64_t nq, float thr,
                                                     int32_t* __restrict__ list, int32_t* __restrict__ n,
                                                     int32_t* __restrict__ leaf) {
  // block-aggregated append: the block's count from the four wave ballots,
  // one atomic per block reserves its slots
  __shared__ int wcount[4];
  __shared__ int base;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool in = q < nq;
  if (in) leaf[q] = -1;
  const bool low = in && !(margin[q] >= thr);
  const uint64_t m = __ballot(low);
  if (lane == 0) wcount[wave] = (int)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    base = tot ? atomicAdd(n, tot) : 0;
  }
  __syncthreads();
  int off = base;
  for (int w = 0; w < wave; ++w) off += wcount[w];
  if (low) list[off + (int)__popcll(m & ((1ull << lane) - 1ull))] = (int32_t)q;
}

static void bucket_core(Ctx* c, const int32_t* leaf, int64_t n, int n_leaves, int chunk, const BucketBufs& b);

// entries of (list, n_list) or 0 .. n-1
static void descend_entries(Ctx* c, const float* Qp, const int32_t* list, const int32_t* n_list, int64_t n, int dp,
                            const float* cent, const int32_t* first_child, const int32_t* n_children,
                            const int32_t* leaf_of_node, int n_nodes, int32_t* leaf) {
  int32_t* node1 = c->buf<int32_t>("ds_node1", (size_t)n);
  PTS_DP_SWITCH(dp, hipLaunchKernelGGL(k_descend_root<DPC>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream,
                                       Qp, list, n_list, n, cent, first_child, n_children, leaf_of_node, node1, leaf));
  check_launch("k_descend_root");
  BucketBufs b;
  b.counts = c->buf<int32_t>("ds_counts", (size_t)n_nodes);
  b.off = c->buf<int32_t>("ds_off", (size_t)n_nodes + 1);
  b.cursor = c->buf<int32_t>("ds_cursor", (size_t)n_nodes);
  b.tile_off = c->buf<int32_t>("ds_tile_off", (size_t)n_nodes + 1);
  b.ntiles = c->buf<int32_t>("ds_ntiles", 1);
  b.order = c->buf<int32_t>("ds_order", (size_t)n);
  const int64_t max_tiles = ceil_div(n, DS_CHUNK) + n_nodes;
  b.tiles = c->buf<int2>("ds_tiles", (size_t)max_tiles);
  bucket_core(c, node1, n, n_nodes, DS_CHUNK, b);
  PTS_DP_SWITCH(dp, hipLaunchKernelGGL(k_descend_tiles<DPC>, dim3((unsigned)ceil_div(max_tiles, 4)), dim3(256), 0,
                                       c->stream, Qp, list, cent, first_child, n_children, leaf_of_node, b.off,
                                       b.order, b.tiles, b.ntiles, n_nodes, leaf));
  check_launch("k_descend_tiles");
}

void launch_descend_low_margin(Ctx* c, const float* Qp, int64_t nq, int dp, const float* margin, float thr,
                               const float* cent, const int32_t* first_child, const int32_t* n_children,
                               const int32_t* leaf_of_node, int n_nodes, int32_t* list, int32_t* n, int32_t* leaf) {
  ProfScope ps(c, "tree_descend_low");
  if (nq == 0) return;
  hipLaunchKernelGGL(k_compact_low, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, margin, nq, thr, list, n,
                     leaf);
  check_launch("k_compact_low");
  descend_entries(c, Qp, list, n, nq, dp, cent, first_child, n_children, leaf_of_node, n_nodes, leaf);
}

void launch_descend(Ctx* c, const float* Qp, int64_t nq, int dp, const float* cent, const int32_t* first_child,
                    const int32_t* n_children, const int32_t* leaf_of_node, int n_nodes, int32_t* leaf) {
  ProfScope ps(c, "tree_descend");
  if (nq == 0) return;
  descend_entries(c, Qp, nullptr, nullptr, nq, dp, cent, first_child, n_children, leaf_of_node, n_nodes, leaf);
}

// ---------------------------------------------------------------------------
// bucketing

__global__ __launch_bounds__(256) void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_leaf_hist(const int32_t* __restrict__ leaf, int64_t n, int n_leaves,
                                                   int32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int l = leaf[i];
  if (l >= 0 && l < n_leaves) atomicAdd(counts + l, 1);
}

// one block of 1024 threads: exclusive scans of the counts and of the tile
// counts; cursor = off for the scatter; writes the tile count.
__global__ __launch_bounds__(1024) void k_leaf_scan_offsets(const int32_t* __restrict__ counts, int n_leaves,
                                                            int chunk, int32_t* __restrict__ off,
                                                            int32_t* __restrict__ cursor,
                                                            int32_t* __restrict__ tile_off,
                                                            int32_t* __restrict__ ntiles,
                                                            const int32_t* __restrict__ tile_order) {
  __shared__ int s_a[1024], s_b[1024];
  __shared__ int carry_a, carry_b;
  if (threadIdx.x == 0) {
    carry_a = 0;
    carry_b = 0;
  }
  __syncthreads();
  for (int base = 0; base < n_leaves; base += 1024) {
    const int l = base + threadIdx.x;
    const int ca = (l < n_leaves) ? counts[l] : 0;
    const int cb = (ca + chunk - 1) / chunk;
    s_a[threadIdx.x] = ca;
    s_b[threadIdx.x] = cb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
      int va = 0, vb = 0;
      if (threadIdx.x >= o) {
        va = s_a[threadIdx.x - o];
        vb = s_b[threadIdx.x - o];
      }
      __syncthreads();
      s_a[threadIdx.x] += va;
      s_b[threadIdx.x] += vb;
      __syncthreads();
    }
    if (l < n_leaves) {
      const int ea = carry_a + s_a[threadIdx.x] - ca;
      const int eb = carry_b + s_b[threadIdx.x] - cb;
      off[l] = ea;
      cursor[l] = ea;
      tile_off[l] = eb;
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      carry_a += s_a[1023];
      carry_b += s_b[1023];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    off[n_leaves] = carry_a;
    tile_off[n_leaves] = carry_b;
    *ntiles = carry_b;
  }
  if (!tile_order) return;  // uniform
  // tile offsets again, the leaves taken in tile_order (same total)
  __syncthreads();
  if (threadIdx.x == 0) carry_b = 0;
  __syncthreads();
  for (int base = 0; base < n_leaves; base += 1024) {
    const int i = base + threadIdx.x;
    const int l = (i < n_leaves) ? tile_order[i] : -1;
    const int cb = (l >= 0) ? (counts[l] + chunk - 1) / chunk : 0;
    s_b[threadIdx.x] = cb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int vb = (threadIdx.x >= o) ? s_b[threadIdx.x - o] : 0;
      __syncthreads();
      s_b[threadIdx.x] += vb;
      __syncthreads();
    }
    if (l >= 0) tile_off[l] = carry_b + s_b[threadIdx.x] - cb;
    __syncthreads();
    if (threadIdx.x == 1023) carry_b += s_b[1023];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_leaf_scatter(const int32_t* __restrict__ leaf, int64_t n, int n_leaves,
                                                      int32_t* __restrict__ cursor, int32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int l = leaf[i];
  if (l < 0 || l >= n_leaves) return;
  const int pos = atomicAdd(cursor + l, 1);
  order[pos] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_leaf_tiles(const int32_t* __restrict__ off, const int32_t* __restrict__ tile_off,
                                                    int n_leaves, int chunk, int2* __restrict__ tiles) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_leaves) return;
  // the leaf's tiles: tile_off[l] .. + its tile count (tile_off need not follow leaf order)
  const int t0 = tile_off[l], t1 = t0 + (off[l + 1] - off[l] + chunk - 1) / chunk;
  for (int t = t0; t < t1; ++t) tiles[t] = make_int2(l, off[l] + (t - t0) * chunk);
}

// LDS-privatised histogram: per block, count its chunk in LDS, then one
// global atomic per (block, leaf) with a non-zero count.
constexpr int BK_LDS_LEAVES = 8192;
constexpr int BK_PER_BLOCK = 4096;

__global__ __launch_bounds__(256) void k_leaf_hist_lds(const int32_t* __restrict__ leaf, int64_t n, int n_leaves,
                                                       int32_t* __restrict__ counts) {
  __shared__ int sc[BK_LDS_LEAVES];
  for (int i = threadIdx.x; i < n_leaves; i += 256) sc[i] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * BK_PER_BLOCK;
  const int64_t e1 = min(n, e0 + BK_PER_BLOCK);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int l = leaf[e];
    if (l >= 0 && l < n_leaves) atomicAdd(sc + l, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_leaves; i += 256)
    if (sc[i]) atomicAdd(counts + i, sc[i]);
}

// scatter: ranks within the block from LDS atomics, one global reservation
// per (block, leaf)
__global__ __launch_bounds__(256) void k_leaf_scatter_lds(const int32_t* __restrict__ leaf, int64_t n, int n_leaves,
                                                          int32_t* __restrict__ cursor, int32_t* __restrict__ order) {
  __shared__ int sc[BK_LDS_LEAVES];
  for (int i = threadIdx.x; i < n_leaves; i += 256) sc[i] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * BK_PER_BLOCK;
  const int64_t e1 = min(n, e0 + BK_PER_BLOCK);
  int rank[BK_PER_BLOCK / 256];
#pragma unroll
  for (int u = 0; u < BK_PER_BLOCK / 256; ++u) {
    const int64_t e = e0 + threadIdx.x + u * 256;
    rank[u] = -1;
    if (e < e1) {
      const int l = leaf[e];
      if (l >= 0 && l < n_leaves) rank[u] = atomicAdd(sc + l, 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_leaves; i += 256)
    if (sc[i]) sc[i] = atomicAdd(cursor + i, sc[i]);  // base of this block's run
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BK_PER_BLOCK / 256; ++u) {
    const int64_t e = e0 + threadIdx.x + u * 256;
    if (rank[u] >= 0) order[sc[leaf[e]] + rank[u]] = (int32_t)e;
  }
}

static void bucket_core(Ctx* c, const int32_t* leaf, int64_t n, int n_leaves, int chunk, const BucketBufs& b) {
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)ceil_div(n_leaves, 256)), dim3(256), 0, c->stream, b.counts,
                     (int64_t)n_leaves);
  check_launch("k_zero_i32");
  const bool lds = n_leaves <= BK_LDS_LEAVES;
  if (n > 0 && lds) {
    hipLaunchKernelGGL(k_leaf_hist_lds, dim3((unsigned)ceil_div(n, BK_PER_BLOCK)), dim3(256), 0, c->stream, leaf, n,
                       n_leaves, b.counts);
    check_launch("k_leaf_hist_lds");
  } else if (n > 0) {
    hipLaunchKernelGGL(k_leaf_hist, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, leaf, n, n_leaves,
                       b.counts);
    check_launch("k_leaf_hist");
  }
  hipLaunchKernelGGL(k_leaf_scan_offsets, dim3(1), dim3(1024), 0, c->stream, b.counts, n_leaves, chunk, b.off,
                     b.cursor, b.tile_off, b.ntiles, b.tile_order);
  check_launch("k_leaf_scan_offsets");
  if (n > 0 && lds) {
    hipLaunchKernelGGL(k_leaf_scatter_lds, dim3((unsigned)ceil_div(n, BK_PER_BLOCK)), dim3(256), 0, c->stream, leaf, n,
                       n_leaves, b.cursor, b.order);
    check_launch("k_leaf_scatter_lds");
  } else if (n > 0) {
    hipLaunchKernelGGL(k_leaf_scatter, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, leaf, n, n_leaves,
                       b.cursor, b.order);
    check_launch("k_leaf_scatter");
  }
  hipLaunchKernelGGL(k_leaf_tiles, dim3((unsigned)ceil_div(n_leaves, 256)), dim3(256), 0, c->stream, b.off, b.tile_off,
                     n_leaves, chunk, b.tiles);
  check_launch("k_leaf_tiles");
}

void launch_bucket(Ctx* c, const int32_t* leaf, int64_t n, int n_leaves, int chunk, BucketBufs b) {
  ProfScope ps(c, "leaf_bucket");
  bucket_core(c, leaf, n, n_leaves, chunk, b);
}

// ---------------------------------------------------------------------------
// leaf scan, FP32 direct form

constexpr int LS_Q = 64, LS_M = 64;

// Workgroup barrier for LDS buffers: this wave's LDS reads and writes
// complete, then s_barrier; unlike __syncthreads() it leaves the wave's
// global loads in flight.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

int leaf_scan_f32_chunk(int dp) {
  (void)dp;
  return LS_Q;
}

__device__ __forceinline__ bool better_id(float d, int id, float bd, int bid) {
  return d < bd || (d == bd && id < bid);
}

// TOPK: each pair keeps its 8 best (distance, leaf position) instead of the
// single best id, written sorted to top_d / top_i [pair][8] (with the
// optional offset added, as the ranking uses it).
template <int DP, bool TOPK>
__global__ __launch_bounds__(256) void k_leaf_scan_f32(const float* __restrict__ Qp, const float* __restrict__ Zp,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ leaf_off,
                                                       const int32_t* __restrict__ qoff,
                                                       const int32_t* __restrict__ order,
                                                       const int2* __restrict__ tiles,
                                                       const int32_t* __restrict__ ntiles, int P,
                                                       const float* __restrict__ zres,
                                                       int32_t* __restrict__ nn, float* __restrict__ best_d2,
                                                       float* __restrict__ top_d, int32_t* __restrict__ top_i) {
  // member rows stream through two LDS buffers: chunk c + 1 is stored while
  // chunk c is scanned, and chunk c + 2 is loaded into registers meanwhile
  constexpr int NF4 = LS_M * (DP / 4);          // float4 per chunk
  constexpr int PERT = (NF4 + 255) / 256;        // per thread
  __shared__ float4 Zs[2][LS_M][DP / 4];
  __shared__ int Zid[2][LS_M];
  __shared__ float Zr[2][LS_M];
  __shared__ float rd[4][LS_Q];
  __shared__ int ri[4][LS_Q];
  // plain hardware order: the tile costs vary with the leaf size and cluster
  // along the list, so a contiguous range per XCD would be unbalanced
  const int t = blockIdx.x;
  if (t >= *ntiles) return;  // uniform per block
  const int2 tile = tiles[t];
  const int l = tile.x;
  const int qend = qoff[l + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pos = tile.y + lane;
  const bool active = pos < qend && pos < tile.y + LS_Q;
  const int pair = active ? order[pos] : -1;  // query * P + slot
  const int q = active ? pair / P : -1;
  float qv[DP];
#pragma unroll
  for (int k = 0; k < DP; k += 4) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) v = *reinterpret_cast<const float4*>(Qp + (int64_t)q * DP + k);
    qv[k] = v.x;
    qv[k + 1] = v.y;
    qv[k + 2] = v.z;
    qv[k + 3] = v.w;
  }
  float bd = FLT_MAX;
  int bi = INT_MAX;
  Top8Lex top;
  if constexpr (TOPK) top.init();
  const int m0 = leaf_off[l], m1 = leaf_off[l + 1];
  const int nchunks = (m1 - m0 + LS_M - 1) / LS_M;
  // chunk loads carry no condition (rows past the leaf re-read its last row
  // and are replaced when stored), so the barriers leave them in flight
  float4 zreg[PERT];
  int idreg = 0;
  float rreg = 0.f;
  auto load_chunk = [&](int c) {
    const int mb = m0 + c * LS_M;
#pragma unroll
    for (int u = 0; u < PERT; ++u) {
      const int idx = min(tid + u * 256, NF4 - 1);
      const int r = idx / (DP / 4), k4 = idx - r * (DP / 4);
      zreg[u] = reinterpret_cast<const float4*>(Zp + (int64_t)min(mb + r, m1 - 1) * DP)[k4];
    }
    const int rr = min(mb + (tid & (LS_M - 1)), m1 - 1);
    idreg = perm[rr];
    rreg = zres ? zres[rr] : 0.f;
  };
  auto store_chunk = [&](int c) {
    const int mb = m0 + c * LS_M, b = c & 1;
#pragma unroll
    for (int u = 0; u < PERT; ++u) {
      const int idx = tid + u * 256;
      if (idx < NF4) {
        const int r = idx / (DP / 4), k4 = idx - r * (DP / 4);
        Zs[b][r][k4] = (mb + r < m1) ? zreg[u] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    if (tid < LS_M) {
      Zid[b][tid] = (mb + tid < m1) ? idreg : INT_MAX;
      Zr[b][tid] = (mb + tid < m1) ? rreg : 0.f;
    }
  };
  if (nchunks > 0) {
    load_chunk(0);
    store_chunk(0);
    load_chunk(min(1, nchunks - 1));
    lds_barrier();
  }
  for (int c = 0; c < nchunks; ++c) {
    const int b = c & 1;
    if (c + 1 < nchunks) store_chunk(c + 1);  // into the buffer chunk c - 1 used
    load_chunk(min(c + 2, nchunks - 1));       // past the end: the last chunk again, never stored
    const int mcount = min(LS_M, m1 - (m0 + c * LS_M));
    for (int r = wave; r < mcount; r += 4) {
      float acc = 0.f;
#pragma unroll
      for (int k4 = 0; k4 < DP / 4; ++k4) {
        const float4 z = Zs[b][r][k4];
        const float t0 = qv[4 * k4] - z.x, t1 = qv[4 * k4 + 1] - z.y;
        const float t2 = qv[4 * k4 + 2] - z.z, t3 = qv[4 * k4 + 3] - z.w;
        acc = fmaf(t0, t0, acc);
        acc = fmaf(t1, t1, acc);
        acc = fmaf(t2, t2, acc);
        acc = fmaf(t3, t3, acc);
      }
      acc += Zr[b][r];
      if constexpr (TOPK) {
        const int mp = m0 + c * LS_M + r;  // the member's leaf position
        if (lex_lt(acc, mp, top.d[7], top.i[7])) top.insert(acc, mp);
      } else {
        const int id = Zid[b][r];
        if (better_id(acc, id, bd, bi)) {
          bd = acc;
          bi = id;
        }
      }
    }
    lds_barrier();
  }
  if constexpr (TOPK) {
    // the 4 waves' lists through LDS
    __shared__ float ld[4 * 8 * LS_Q];
    __shared__ int li[4 * 8 * LS_Q];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      ld[(wave * 8 + t) * LS_Q + lane] = top.d[t];
      li[(wave * 8 + t) * LS_Q + lane] = top.i[t];
    }
    __syncthreads();
    if (wave == 0 && active) {
      for (int w = 1; w < 4; ++w)
        for (int t = 0; t < 8; ++t) {
          const float v = ld[(w * 8 + t) * LS_Q + lane];
          const int i = li[(w * 8 + t) * LS_Q + lane];
          if (lex_lt(v, i, top.d[7], top.i[7])) top.insert(v, i);
        }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        top_d[(int64_t)pair * 8 + t] = top.d[t];
        top_i[(int64_t)pair * 8 + t] = top.i[t];
      }
    }
    return;
  }
  rd[wave][lane] = bd;
  ri[wave][lane] = bi;
  __syncthreads();
  if (wave == 0 && active) {
    for (int w = 1; w < 4; ++w)
      if (better_id(rd[w][lane], ri[w][lane], bd, bi)) {
        bd = rd[w][lane];
        bi = ri[w][lane];
      }
    nn[pair] = (bi == INT_MAX) ? -1 : bi;
    if (best_d2) best_d2[pair] = bd;
  }
}

void launch_leaf_scan_f32(Ctx* c, const float* Qp, int dp, const float* Zp, const int32_t* perm,
                          const int32_t* leaf_off, const BucketBufs& b, int max_tiles, int P, const float* zres,
                          int32_t* nn, float* best_d2, float* top_d, int32_t* top_i) {
  ProfScope ps(c, "leaf_scan_f32");
  if (max_tiles == 0) return;
  if (top_d) {
    PTS_DP_SWITCH(dp, hipLaunchKernelGGL((k_leaf_scan_f32<DPC, true>), dim3(max_tiles), dim3(256), 0, c->stream, Qp,
                                         Zp, perm, leaf_off, b.off, b.order, b.tiles, b.ntiles, P, zres, nn, best_d2,
                                         top_d, top_i));
  } else {
    PTS_DP_SWITCH(dp, hipLaunchKernelGGL((k_leaf_scan_f32<DPC, false>), dim3(max_tiles), dim3(256), 0, c->stream, Qp,
                                         Zp, perm, leaf_off, b.off, b.order, b.tiles, b.ntiles, P, zres, nn, best_d2,
                                         nullptr, nullptr));
  }
  check_launch("k_leaf_scan_f32");
}

}  // namespace pts

namespace pts {

void launch_zero_i32(Ctx* c, int32_t* p, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, p, n);
  check_launch("k_zero_i32");
}

}  // namespace pts

namespace pts {

// pair lists of the learned search: slot s of query q scans leaf
// pair_leaf[q * (P + 1) + s] (-1 = unused): slots 0..P-1 the P proposed
// leaves; slot P the tree's own leaf when the margin is below thr (the
// fallback) and that leaf is not already proposed.
__global__ __launch_bounds__(256) void k_learned_pairs(const int32_t* __restrict__ prop, const float* __restrict__ margin,
                                                       const int32_t* __restrict__ dleaf, int64_t nq, int P, float thr,
                                                       int n_leaves, int32_t* __restrict__ pair_leaf,
                                                       int32_t* __restrict__ fallbacks) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const bool fb = !(margin[q] >= thr);
  const int dl = dleaf[q];
  bool dup = false;
  for (int s = 0; s < P; ++s) {
    int l = prop[q * P + s];
    if (l < 0 || l >= n_leaves) l = -1;
    dup = dup || (l == dl);
    pair_leaf[q * (P + 1) + s] = l;
  }
  pair_leaf[q * (P + 1) + P] = (fb && !dup && dl >= 0 && dl < n_leaves) ? dl : -1;
  // one atomic per wave: the wave's count of fallbacks (when counted)
  if (fallbacks) {
    const uint64_t m = __ballot(fb);
    if ((threadIdx.x & 63) == (uint32_t)(__ffsll((unsigned long long)__ballot(1)) - 1) && m)
      atomicAdd(fallbacks, (int)__popcll(m));
  }
}

void launch_learned_pairs(Ctx* c, const int32_t* prop, const float* margin, const int32_t* dleaf, int64_t nq, int P,
                          float thr, int n_leaves, int32_t* pair_leaf, int32_t* fallbacks) {
  ProfScope ps(c, "learned_pairs");
  if (nq == 0) return;
  hipLaunchKernelGGL(k_learned_pairs, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, prop, margin, dleaf,
                     nq, P, thr, n_leaves, pair_leaf, fallbacks);
  check_launch("k_learned_pairs");
}

// nn[q] = the best of the query's P pair winners (ties to the lowest id)
__global__ __launch_bounds__(256) void k_merge_pairs_f32(const int32_t* __restrict__ pair_leaf,
                                                         const int32_t* __restrict__ pair_id,
                                                         const float* __restrict__ pair_d, int64_t nq, int P,
                                                         int32_t* __restrict__ nn) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  float bd = FLT_MAX;
  int bi = INT_MAX;
  for (int s = 0; s < P; ++s) {
    const int64_t p = q * P + s;
    if (pair_leaf[p] < 0) continue;
    const int id = pair_id[p];
    const float d = pair_d[p];
    if (id >= 0 && better_id(d, id, bd, bi)) {
      bd = d;
      bi = id;
    }
  }
  nn[q] = (bi == INT_MAX) ? -1 : bi;
}

void launch_merge_pairs_f32(Ctx* c, const int32_t* pair_leaf, const int32_t* pair_id, const float* pair_d, int64_t nq,
                            int P, int32_t* nn) {
  ProfScope ps(c, "merge_pairs");
  if (nq == 0) return;
  hipLaunchKernelGGL(k_merge_pairs_f32, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, pair_leaf, pair_id,
                     pair_d, nq, P, nn);
  check_launch("k_merge_pairs_f32");
}

}  // namespace pts
