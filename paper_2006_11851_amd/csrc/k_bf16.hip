// BF16 distance form of the search: every projected query against every
// projected exemplar window on the matrix cores, keeping the k best per
// query, then an FP32 re-rank of those k.
//
// Distances use ||q - z||^2 = ||q||^2 - 2 q.z + ||z||^2.  ||q||^2 does not
// change a query's ranking and is dropped; the MFMA accumulator starts at
// ||z||^2 (FP32 norm of the bf16-rounded z) and the query operand is stored
// as bf16(-2 q) (exact: a power-of-two scale), so the accumulator ends at
// ||z||^2 - 2 q.z with no epilogue arithmetic.  bf16 products are exact in
// FP32; accumulation is FP32.
//
// Tiling (v_mfma_f32_32x32x16_bf16, wave64): A = 32 exemplar rows x 16 of
// K, B = 16 of K x 32 queries; lane l owns query column l % 32 and 16
// exemplar rows, so each lane keeps a sorted top-k of its own query in
// registers and the two lanes sharing a query merge at the end.  A block of
// 8 waves holds 512 queries (64 per wave, two B tiles kept in registers);
// exemplar rows stream through LDS in stages of 128 rows, double buffered,
// pre-swizzled into MFMA fragment order (conflict-free 16-byte reads).  The
// exemplar is split into S contiguous ranges; block b takes range b % S, so
// with the round-robin placement of blocks over the 8 XCDs every XCD streams
// one range through its own L2.  A per-query merge of the S partial lists
// and the FP32 re-rank follow.
#include <algorithm>
#include <cfloat>
#include <type_traits>
#include <utility>
#include <climits>

#include "kernels_bf16.hpp"
#include "device_util.hpp"

namespace pts {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// sorted top-K (ascending) in registers

template <int K>
struct TopK {
  float d[K];
  int i[K];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      d[t] = FLT_MAX;
      i[t] = INT_MAX;
    }
  }
  // insert (v, id); a no-op unless v < d[K-1]
  __device__ __forceinline__ void insert(float v, int id) {
#pragma unroll
    for (int t = K - 1; t > 0; --t) {
      const bool s = v < d[t - 1];
      const bool n = v < d[t];
      d[t] = s ? d[t - 1] : (n ? v : d[t]);
      i[t] = s ? i[t - 1] : (n ? id : i[t]);
    }
    if (v < d[0]) {
      d[0] = v;
      i[0] = id;
    }
  }
};

constexpr int BB_WAVES = 8;
constexpr int BB_QPB = BB_WAVES * 64;  // queries per block
constexpr int BB_STAGE = 128;          // exemplar rows per LDS stage
constexpr int BB_TOPK = 8;

// Workgroup barrier for the LDS stage buffers: this wave's LDS reads and
// writes complete, then s_barrier.  Unlike __syncthreads() it does not wait
// for the wave's global loads, so the next stages stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Fragment layout of a stage, in 16-byte units: 32-row tile t, k-chunk kk,
// half hh (k-values 16 kk + 8 hh .. + 7), row i at t TS + kk KKS + hh HS + i.
// The MFMA read (lane l: half l / 32, row l % 32) is contiguous for every 16
// lanes.  A store cycle of 16 lanes covers 16 / (2 KS) rows and all their
// chunks (2 KS per row); with HS = 32 + SP and KKS = 64 + 2 SP, SP = 16 / (2
// KS), chunk c of row i lands in bank group (SP c + i) mod 16: distinct over
// the cycle, where unpadded strides would put a row's chunks in one group.
template <int KS>
struct StageLayout {
  static constexpr int SP = 2 * KS >= 16 ? 1 : 16 / (2 * KS);
  static constexpr int HS = 32 + SP, KKS = 64 + 2 * SP, TS = KS * KKS;
};

template <int KS>
struct BruteSmem {
  uint4 frag[2][BB_STAGE / 32 * StageLayout<KS>::TS];  // [buffer][fragment layout above]
  float zn[2][BB_STAGE];
};

// the lane's 16-byte fragment of tile t, k-chunk kk
template <int KS>
__device__ __forceinline__ uint4 stage_frag(const BruteSmem<KS>& S, int buf, int t, int kk, int lane) {
  using L = StageLayout<KS>;
  return S.frag[buf][t * L::TS + kk * L::KKS + (lane >> 5) * L::HS + (lane & 31)];
}

// A tile's operands from a stage: the lane's row fragments and the row
// norms that start its accumulator (rows 8 (r / 4) + 4 (lane / 32) + r % 4)
template <int KS>
__device__ __forceinline__ void tile_operands(const BruteSmem<KS>& S, int buf, int t, int lane, bf16x8 (&A)[KS],
                                              floatx16& cz) {
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const uint4 u = stage_frag<KS>(S, buf, t, kk, lane);
    A[kk] = *reinterpret_cast<const bf16x8*>(&u);
  }
  const float* zr = &S.zn[buf][t * 32 + 4 * (lane >> 5)];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 z4 = *reinterpret_cast<const float4*>(zr + 8 * g);
    cz[4 * g + 0] = z4.x;
    cz[4 * g + 1] = z4.y;
    cz[4 * g + 2] = z4.z;
    cz[4 * g + 3] = z4.w;
  }
}

// Loads one stage (rows r0 .. r0+127 of [row_begin, row_end)) from global
// into registers: each thread owns up to 2 chunks of 16 B plus zn entries.
template <int KS, int NTH = BB_QPB>
struct StageRegs {
  uint4 v[(BB_STAGE * KS * 2 + NTH - 1) / NTH];
  float zn;
};

// The loads carry no lane-dependent condition (rows past the range read the
// last row; stage_store replaces them by zero rows with norm FLT_MAX), so
// the compiler waits for them only right before the store.
template <int KS, int NTH = BB_QPB>
__device__ __forceinline__ void stage_load(StageRegs<KS, NTH>& R, const uint16_t* __restrict__ Zb,
                                           const float* __restrict__ zbn, int64_t r0, int64_t row_end, int tid) {
  constexpr int CH = KS * 2;  // 16-byte chunks per row
  constexpr int NCH = BB_STAGE * CH;
  constexpr int PER = (NCH + NTH - 1) / NTH;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int c = tid + u * NTH;
    if (c < NCH) {  // uniform per wave
      const int row = c / CH, ch = c - row * CH;
      const int64_t gr = min(r0 + row, row_end - 1);
      R.v[u] = reinterpret_cast<const uint4*>(Zb + gr * (KS * 16))[ch];
    }
  }
  R.zn = zbn[min(r0 + (tid & (BB_STAGE - 1)), row_end - 1)];
}

template <int KS, int NTH = BB_QPB>
__device__ __forceinline__ void stage_store(const StageRegs<KS, NTH>& R, BruteSmem<KS>& S, int buf, int tid,
                                            int64_t r0, int64_t row_end) {
  static_assert(NTH >= BB_STAGE, "one thread per row norm");
  constexpr int CH = KS * 2;
  constexpr int NCH = BB_STAGE * CH;
  constexpr int PER = (NCH + NTH - 1) / NTH;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int c = tid + u * NTH;
    if (c < NCH) {
      const int row = c / CH, ch = c - row * CH;
      const int tile = row >> 5, i = row & 31;
      const int kk = ch >> 1, half = ch & 1;
      S.frag[buf][tile * StageLayout<KS>::TS + kk * StageLayout<KS>::KKS + half * StageLayout<KS>::HS + i] =
          (r0 + row < row_end) ? R.v[u] : make_uint4(0, 0, 0, 0);
    }
  }
  if (tid < BB_STAGE) S.zn[buf][tid] = (r0 + tid < row_end) ? R.zn : FLT_MAX;
}

// Class minima of a scan: a sorted per-lane top-k would insert on a large
// share of rows (and under SIMT every value slot would pay for it), so each
// lane keeps instead, for each of its 8 classes (value slots r and r + 8 of
// the 32x32 output, i.e. rows i and i + 16 of every 32-row tile, i < 16 fixed
// per class and half-wave), the minimum score over the scan and the 32-row
// tile holding it: v_min3 + compare + select per class and tile.  The bound
// pass takes the K-th smallest class minimum of a query as its bound; the
// class-candidate pass hands the class minima themselves to the re-rank.
// FULL: all 128 rows of the stage are valid (no per-tile exit, so the whole
// stage is one straight-line block the scheduler can interleave).
// ROW: ct records the row of the minimum's first occurrence (its tile's
// first row, plus 16 if it is the class's second row of that tile)
template <int KS, bool FULL, bool ROW = false>
__device__ __forceinline__ void stage_compute_cls(const BruteSmem<KS>& S, int buf, const bf16x8 (&B)[2][KS],
                                                  float (&cm)[2][8], int (&ct)[2][8], int pos0, int lane,
                                                  int nvalid) {
#pragma unroll
  for (int t = 0; t < BB_STAGE / 32; ++t) {
    if (!FULL && t * 32 >= nvalid) break;
    bf16x8 A[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const uint4 u = stage_frag<KS>(S, buf, t, kk, lane);
      A[kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
    floatx16 cinit;
    const float* zr = &S.zn[buf][t * 32 + 4 * (lane >> 5)];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 z4 = *reinterpret_cast<const float4*>(zr + 8 * g);
      cinit[4 * g + 0] = z4.x;
      cinit[4 * g + 1] = z4.y;
      cinit[4 * g + 2] = z4.z;
      cinit[4 * g + 3] = z4.w;
    }
    const int tbase = pos0 + t * 32;
#pragma unroll
    for (int qt = 0; qt < 2; ++qt) {
      floatx16 acc = cinit;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[qt][kk], acc, 0, 0, 0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float m3 = __builtin_fminf(cm[qt][c], __builtin_fminf(acc[c], acc[c + 8]));
        const int tb = ROW ? (acc[c + 8] < acc[c] ? tbase + 16 : tbase) : tbase;
        ct[qt][c] = (m3 < cm[qt][c]) ? tb : ct[qt][c];
        cm[qt][c] = m3;
      }
    }
  }
}

// pairs per leaf-scan tile (one block of 8 waves, 64 pairs each; blocks of
// 4 waves, two per CU, were slower)
constexpr int LS_QPB = 512;
constexpr int LS_HC_MAX = 14;  // collect slots per (pair, half-lane): all of them held in LDS
int leaf_scan_bf16_chunk() { return LS_QPB; }
// collect slots that fit in LDS beside the stage buffers (at most LS_HC_MAX)
template <int KS>
constexpr int ls_hc_cap() {
  constexpr int avail = (160 * 1024 - (int)sizeof(BruteSmem<KS>) - 256) / (2 * LS_QPB * (int)sizeof(int2));
  return avail < LS_HC_MAX ? avail : LS_HC_MAX;
}

// The full-stage form of stage_compute_cls, software pipelined: the products
// of tile t (two independent chains, one per query tile) are woven with the
// class updates of tile t - 1, so that the accumulators are read long after
// their last product; only the last tile's updates follow the products.
template <int KS, int kk>
__device__ __forceinline__ void cls_order_step() {
  __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
  __builtin_amdgcn_sched_group_barrier(0x002, 24 / KS, 0);
  __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
  __builtin_amdgcn_sched_group_barrier(0x002, 24 / KS, 0);
}
template <int KS, int... KK>
__device__ __forceinline__ void cls_order(std::integer_sequence<int, KK...>) {
  (cls_order_step<KS, KK>(), ...);
}

template <int KS, bool ROW = false>
__device__ __forceinline__ void stage_compute_cls_full(const BruteSmem<KS>& S, int buf, const bf16x8 (&B)[2][KS],
                                                       float (&cm)[2][8], int (&ct)[2][8], int pos0, int lane) {
  auto update = [&](const floatx16& acc, int qt, int c, int tbase) {
    const float m3 = __builtin_fminf(cm[qt][c], __builtin_fminf(acc[c], acc[c + 8]));
    const int tb = ROW ? (acc[c + 8] < acc[c] ? tbase + 16 : tbase) : tbase;  // as in stage_compute_cls
    ct[qt][c] = (m3 < cm[qt][c]) ? tb : ct[qt][c];
    cm[qt][c] = m3;
  };
  constexpr int NT = BB_STAGE / 32;
  floatx16 accp[2];
  // tile t + 1's operands are read from LDS while tile t's products run
  // (up to 64 dimensions; wider rows have no registers to spare for it)
  constexpr bool PF = KS <= 4;
  bf16x8 A[KS];
  floatx16 cz;
  if constexpr (PF) tile_operands<KS>(S, buf, 0, lane, A, cz);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    __builtin_amdgcn_sched_barrier(0);  // tile by tile
    bf16x8 An[KS];
    floatx16 czn;
    if constexpr (PF) {
      if (t + 1 < NT) tile_operands<KS>(S, buf, t + 1, lane, An, czn);
    } else {
      tile_operands<KS>(S, buf, t, lane, A, cz);
    }
    floatx16 accn[2] = {cz, cz};
    const int tprev = pos0 + (t - 1) * 32;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
      for (int qt = 0; qt < 2; ++qt) {
        accn[qt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[qt][kk], accn[qt], 0, 0, 0);
        if (t > 0) {
          // the 16 class updates of the previous tile spread over the 2 KS products
#pragma unroll
          for (int j = (16 * (2 * kk + qt)) / (2 * KS); j < (16 * (2 * kk + qt + 1)) / (2 * KS); ++j)
            update(accp[j >> 3], j >> 3, j & 7, tprev);
        }
      }
    }
    if (PF ? t + 1 < NT : t > 0) __builtin_amdgcn_sched_group_barrier(0x100, 2 * KS, 0);
    if (t > 0) cls_order<KS>(std::make_integer_sequence<int, KS>{});
    accp[0] = accn[0];
    accp[1] = accn[1];
    if (PF && t + 1 < NT) {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) A[kk] = An[kk];
      cz = czn;
    }
  }
  const int tlast = pos0 + (NT - 1) * 32;
#pragma unroll
  for (int qt = 0; qt < 2; ++qt)
#pragma unroll
    for (int c = 0; c < 8; ++c) update(accp[qt], qt, c, tlast);
}

// ---------------------------------------------------------------------------
// Exact BF16 top-8 of the learned form's leaf scans, in two passes over the
// bucketed (query, leaf) pairs.  Scores order lexicographically by (score,
// leaf position); the position breaks exact ties (flat texels repeat whole
// windows), and leaves keep their members in ascending exemplar id.
//
// Pass 1 (bound): each pair keeps its 16 class minima (rows i % 16 fixed,
// each with the 32-row tile of its first occurrence).  The classes are
// disjoint, so the 8th smallest class key is an upper bound on the pair's
// 8th smallest key; the query's bound tau is the smallest over its pairs.
// Pass 2 (collect): the same products again; every row whose key is at most
// tau is written to the lane's own slots of its (pair, half) - on average
// about ten rows per query in all.  At least 8 rows qualify, so the 8
// smallest collected keys are the exact top-8 of the scanned members.  A
// (pair, half) with more rows than slots sends its query to a per-query
// pass with the same matrix products (identical scores) and a full sort.

// order-preserving 64-bit key of (score, position): the score's bits mapped
// so that unsigned order is float order, the position below them
__device__ __forceinline__ uint64_t score_key(float v, int pos) {
  uint32_t u = __float_as_uint(v);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)u << 32) | (uint32_t)pos;
}
__device__ __forceinline__ float key_score(uint64_t k) {
  uint32_t u = (uint32_t)(k >> 32);
  u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(u);
}
__device__ __forceinline__ int key_pos(uint64_t k) { return (int)(uint32_t)k; }
__device__ __forceinline__ void cmp_swap(uint64_t& a, uint64_t& b) {
  const bool s = b < a;
  const uint64_t lo = s ? b : a;
  b = s ? a : b;
  a = lo;
}

// One wave: 64 queries (two B tiles) against the staged 128 rows.
template <int KS, int KT>
__device__ __forceinline__ void stage_compute(const BruteSmem<KS>& S, int buf, const bf16x8 (&B)[2][KS],
                                              TopK<KT> (&top)[2], const float (&tv)[2], int64_t pos0, int lane,
                                              int nvalid) {
#pragma unroll
  for (int t = 0; t < BB_STAGE / 32; ++t) {
    if (t * 32 >= nvalid) break;  // rows past the range: padding only
    bf16x8 A[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const uint4 u = stage_frag<KS>(S, buf, t, kk, lane);
      A[kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
    floatx16 cinit;
    const float* zr = &S.zn[buf][t * 32 + 4 * (lane >> 5)];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 z4 = *reinterpret_cast<const float4*>(zr + 8 * g);
      cinit[4 * g + 0] = z4.x;
      cinit[4 * g + 1] = z4.y;
      cinit[4 * g + 2] = z4.z;
      cinit[4 * g + 3] = z4.w;
    }
    const int64_t tpos = pos0 + t * 32 + 4 * (lane >> 5);
#pragma unroll
    for (int qt = 0; qt < 2; ++qt) {
      floatx16 acc = cinit;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[qt][kk], acc, 0, 0, 0);
      float m = acc[0];
#pragma unroll
      for (int r = 1; r < 16; ++r) m = fminf(m, acc[r]);
      // only scores within the query's bound can be among its KT smallest
      const float lim = fminf(top[qt].d[KT - 1], tv[qt]);
      if (__any(m < top[qt].d[KT - 1] && m <= tv[qt])) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float v = acc[r];
          if (v < top[qt].d[KT - 1] && v <= lim) top[qt].insert(v, (int)(tpos + 8 * (r >> 2) + (r & 3)));
        }
      }
    }
  }
}

template <int KS, int KT>
__global__ __launch_bounds__(512) void k_brute_bf16_topk(const uint16_t* __restrict__ Qb, int64_t nq,
                                                         const uint16_t* __restrict__ Zb,
                                                         const float* __restrict__ zbn, int64_t N, int S,
                                                         int64_t rows_per_split,
                                                         const uint64_t* __restrict__ tau_q,
                                                         float* __restrict__ part_d,
                                                         int32_t* __restrict__ part_i) {
  __shared__ BruteSmem<KS> sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int split = blockIdx.x % S;
  const int64_t qb = blockIdx.x / S;
  const int64_t row_begin = (int64_t)split * rows_per_split;
  const int64_t row_end = min(N, row_begin + rows_per_split);
  // query B fragments: lane holds K = 16 kk + 8 (lane / 32) .. + 7 of query lane % 32
  bf16x8 B[2][KS];
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
    const int64_t q = qb * BB_QPB + wave * 64 + qt * 32 + (lane & 31);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      uint4 u = make_uint4(0, 0, 0, 0);
      if (q < nq) u = reinterpret_cast<const uint4*>(Qb + q * (KS * 16))[2 * kk + (lane >> 5)];
      B[qt][kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
  }
  TopK<KT> top[2];
  top[0].init();
  top[1].init();
  // the query's bound (its KT-th smallest key is at most it); none: no filter
  float tv[2];
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
    const int64_t q = qb * BB_QPB + wave * 64 + qt * 32 + (lane & 31);
    tv[qt] = (tau_q && q < nq) ? key_score(tau_q[q]) : INFINITY;
  }
  if (row_begin < row_end) {
    const int nstages = (int)ceil_div(row_end - row_begin, BB_STAGE);
    // stages load two ahead (two register sets): stage st + 2 is issued at
    // step st and stored at step st + 1
    StageRegs<KS> R[2];
    stage_load<KS>(R[0], Zb, zbn, row_begin, row_end, tid);
    stage_load<KS>(R[1], Zb, zbn, row_begin + (int64_t)min(1, nstages - 1) * BB_STAGE, row_end, tid);
    stage_store<KS>(R[0], sm, 0, tid, row_begin, row_end);
    lds_barrier();
    for (int s0 = 0; s0 < nstages; s0 += 2) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int st = s0 + u;
        if (st >= nstages) break;
        // unconditional (past the end: the last rows again, never stored), so
        // the wait before the store covers only the older stage
        stage_load<KS>(R[u], Zb, zbn, row_begin + (int64_t)min(st + 2, nstages - 1) * BB_STAGE, row_end, tid);
        stage_compute<KS, KT>(sm, u, B, top, tv, row_begin + (int64_t)st * BB_STAGE, lane,
                          (int)min((int64_t)BB_STAGE, row_end - row_begin - (int64_t)st * BB_STAGE));
        if (st + 1 < nstages)
          stage_store<KS>(R[u ^ 1], sm, u ^ 1, tid, row_begin + (int64_t)(st + 1) * BB_STAGE, row_end);
        lds_barrier();
      }
    }
  }
  // merge the two lanes that share a query: the k smallest of two sorted
  // lists (in bitonic order; the merge kernels take them in any order)
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
    float od[KT];
    int oi[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      od[t] = __shfl_xor(top[qt].d[t], 32, 64);
      oi[t] = __shfl_xor(top[qt].i[t], 32, 64);
    }
    const int64_t q = qb * BB_QPB + wave * 64 + qt * 32 + (lane & 31);
    if (lane < 32 && q < nq) {
      float* pd = part_d + ((int64_t)split * nq + q) * KT;
      int32_t* pi = part_i + ((int64_t)split * nq + q) * KT;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const float a = top[qt].d[t], b = od[KT - 1 - t];
        const int ia = top[qt].i[t], ib = oi[KT - 1 - t];
        const bool take_a = a < b || (a == b && ia < ib);
        pd[t] = take_a ? a : b;
        pi[t] = take_a ? ia : ib;
      }
    }
  }
}

// the 19-comparator sorting network for 8 keys (ascending)
__device__ __forceinline__ void sort8(uint64_t (&k)[8]) {
  cmp_swap(k[0], k[2]); cmp_swap(k[1], k[3]); cmp_swap(k[4], k[6]); cmp_swap(k[5], k[7]);
  cmp_swap(k[0], k[4]); cmp_swap(k[1], k[5]); cmp_swap(k[2], k[6]); cmp_swap(k[3], k[7]);
  cmp_swap(k[0], k[1]); cmp_swap(k[2], k[3]); cmp_swap(k[4], k[5]); cmp_swap(k[6], k[7]);
  cmp_swap(k[2], k[4]); cmp_swap(k[3], k[5]);
  cmp_swap(k[1], k[4]); cmp_swap(k[3], k[6]);
  cmp_swap(k[1], k[2]); cmp_swap(k[3], k[4]); cmp_swap(k[5], k[6]);
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const int lo = __shfl_xor((int)(uint32_t)v, m, 64);
  const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}


struct LeafScanOut {
  // pass 1
  uint64_t* pair_keys;  // [pairs][16] the pair's class keys (two sorted runs of 8)
  // class-minimum candidates (pass 3): [pairs][8] (score, leaf position)
  float* part_d;
  int32_t* part_i;
  // pass 2
  const uint64_t* tau_q;  // [nq] smallest bound over the query's pairs
  int2* hits;             // [pairs][2][hs] (score bits, leaf position)
  int32_t* hit_cnt;       // [pairs][2] rows collected (may exceed hc: overflow)
  int hc;                 // slots the pass may fill per (pair, half), <= hs
  int hs;                 // slot stride (the per-query pass needs P * 2 * hs >= K * FB_CHUNKS)
};

// The collected rows of a query, as the re-rank kernels read them.
struct HitLists {
  const int2* hits;         // null: the kernels read sorted part lists instead
  const int32_t* hit_cnt;
  const int32_t* pair_leaf; // [nq * P]; pairs with a negative leaf were not scanned
  int P, hs;
};

// top <- the 8 smallest (score, position) keys among the query's collected
// rows (the pair leaves and counts are loaded together, then the rows)
constexpr int HL_PMAX = 16;  // pairs per query: up to 8 proposals + the tree's leaf, or 16 exemplar splits
template <int K>
__device__ __forceinline__ void top8_from_hits(TopLex<K>& top, const HitLists& L, int64_t q) {
  int n[2 * HL_PMAX];
#pragma unroll
  for (int j = 0; j < HL_PMAX; ++j) {
    const bool ok = j < L.P && L.pair_leaf[q * L.P + j] >= 0;
    const int64_t p = q * L.P + j;
    n[2 * j] = ok ? L.hit_cnt[2 * p] : 0;
    n[2 * j + 1] = ok ? L.hit_cnt[2 * p + 1] : 0;
  }
#pragma unroll
  for (int j = 0; j < 2 * HL_PMAX; ++j) {
    const int2* hp = L.hits + (2 * (q * L.P) + j) * L.hs;
    for (int e = 0; e < n[j]; ++e) {
      const int2 v = hp[e];
      const float sv = __int_as_float(v.x);
      if (lex_lt(sv, v.y, top.d[K - 1], top.i[K - 1])) top.insert(sv, v.y);
    }
  }
}

// Collected rows of a lane for one query tile: slot cnt is the next free
// one.  The rows stay in LDS (slot k of lane-set j at k * 2 LS_QPB + j) until
// the tile's stages are done, and only then go to their global slots: a
// global store pending in the stage loop would make every wait for the row
// loads a full drain (loads and stores share one completion counter and may
// complete out of order), undoing the two-stage prefetch.
struct HitLane {
  float tv;    // the query's bound: score
  int tp;      // and position
  int2* dst;   // the (pair, half) slots
  int cnt;
  int lds;     // the lane-set's first LDS slot
};

__device__ __forceinline__ void hit_push(HitLane& L, int2* lbuf, int hc, int2 e) {
  if (L.cnt < hc) lbuf[L.lds + L.cnt * (2 * LS_QPB)] = e;
  ++L.cnt;
}

__device__ __forceinline__ void hit_write(const HitLane& L, const int2* lbuf, int hc) {
  const int n = min(L.cnt, hc);
  for (int k = 0; k < n; ++k) L.dst[k] = lbuf[L.lds + k * (2 * LS_QPB)];
}

// rows of a tile (accumulator acc, first row tpos) at or below the query's
// bound, tested four values at a time (rows i, i + 8, i + 16, i + 24 of the
// lane's half) so that a tile takes 4 tests.  Rows past the leaf score
// FLT_MAX and the bound's score is held below FLT_MAX, so they never pass.
__device__ __forceinline__ void collect_rows(const floatx16& acc, HitLane& L, int2* lbuf, int hc, int tpos) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float m = __builtin_fminf(__builtin_fminf(acc[c], acc[c + 4]), __builtin_fminf(acc[c + 8], acc[c + 12]));
    if (m <= L.tv) {
#pragma unroll
      for (int r = c; r < 16; r += 4) {
        const float v = acc[r];
        const int pos = tpos + 8 * (r >> 2) + (r & 3);
        if (v <= L.tv && (v < L.tv || pos <= L.tp)) hit_push(L, lbuf, hc, make_int2(__float_as_int(v), pos));
      }
    }
  }
}

// Pass 2 over one stage, software pipelined: tile t + 1's operands are read
// from LDS (up to 64 dimensions) and tile t's products issued, then tile
// t - 1's rows are collected while they run.  Every stage takes all 4 tiles: rows past the
// leaf are zero rows with norm FLT_MAX in LDS, so they score FLT_MAX and are
// never collected (one code path keeps the kernel small).
template <int KS>
__device__ __forceinline__ void stage_collect(const BruteSmem<KS>& S, int buf, const bf16x8 (&B)[2][KS],
                                              HitLane& L0, HitLane& L1, int2* lbuf, int hc, int pos0, int lane,
                                              int row_end) {
  constexpr int NT = BB_STAGE / 32;
  floatx16 accp[2];
  const int hofs = 4 * (lane >> 5);
  constexpr bool PF = KS <= 4;  // as in the bound pass
  bf16x8 A[KS];
  floatx16 cz;
  if constexpr (PF) tile_operands<KS>(S, buf, 0, lane, A, cz);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    bf16x8 An[KS];
    floatx16 czn;
    if constexpr (PF) {
      if (t + 1 < NT) tile_operands<KS>(S, buf, t + 1, lane, An, czn);
    } else {
      tile_operands<KS>(S, buf, t, lane, A, cz);
    }
    floatx16 accn[2] = {cz, cz};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
      for (int qt = 0; qt < 2; ++qt)
        accn[qt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[qt][kk], accn[qt], 0, 0, 0);
    if (t > 0) {
      collect_rows(accp[0], L0, lbuf, hc, pos0 + (t - 1) * 32 + hofs);
      collect_rows(accp[1], L1, lbuf, hc, pos0 + (t - 1) * 32 + hofs);
    }
    accp[0] = accn[0];
    accp[1] = accn[1];
    if (PF && t + 1 < NT) {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) A[kk] = An[kk];
      cz = czn;
    }
  }
  collect_rows(accp[0], L0, lbuf, hc, pos0 + (NT - 1) * 32 + hofs);
  collect_rows(accp[1], L1, lbuf, hc, pos0 + (NT - 1) * 32 + hofs);
}

// One tile = (leaf, LS_QPB pairs of the bucketed order); rows = the leaf's
// members (contiguous in leaf order).  Waves without pairs skip the matrix
// work but still help stage the rows.
template <int KS, int PASS>
__device__ __forceinline__ void leaf_scan_tile(int t, BruteSmem<KS>& sm, const uint16_t* __restrict__ Qb, int P,
                                               const uint16_t* __restrict__ Zb, const float* __restrict__ zbn,
                                               const int32_t* __restrict__ leaf_off,
                                               const int32_t* __restrict__ qoff, const int32_t* __restrict__ order,
                                               const int2* __restrict__ tiles, const LeafScanOut& o, int2* lbuf) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5;
  const int2 tile = tiles[t];
  const int row_begin = leaf_off[tile.x], row_end = leaf_off[tile.x + 1];
  const int nstages = (int)ceil_div(row_end - row_begin, BB_STAGE);
  // the first two stages' rows are requested before the pairs' query
  // operands (a chain of two dependent loads), so that both are in flight
  StageRegs<KS, LS_QPB> R0, R1;
  if (row_begin < row_end) {
    stage_load<KS, LS_QPB>(R0, Zb, zbn, row_begin, row_end, tid);
    stage_load<KS, LS_QPB>(R1, Zb, zbn, row_begin + (int64_t)min(1, nstages - 1) * BB_STAGE, row_end, tid);
  }
  const int pend = min(qoff[tile.x + 1], tile.y + LS_QPB);
  const bool wave_active = tile.y + wave * 64 < pend;
  bf16x8 B[2][KS];
  int pr[2];
  int64_t qid[2];
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
    const int pos = tile.y + wave * 64 + qt * 32 + (lane & 31);
    pr[qt] = pos < pend ? order[pos] : -1;
    // a lane without a pair reads query 0: its results are never written
    qid[qt] = pr[qt] >= 0 ? pr[qt] / P : 0;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const uint4 u = reinterpret_cast<const uint4*>(Qb + qid[qt] * (KS * 16))[2 * kk + (lane >> 5)];
      B[qt][kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
  }
  float cm[2][8];
  int ct[2][8];
  HitLane L0, L1;
  if constexpr (PASS != 2) {
#pragma unroll
    for (int qt = 0; qt < 2; ++qt)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        cm[qt][c] = FLT_MAX;
        ct[qt][c] = -1;
      }
  } else {
    auto init_lane = [&](HitLane& L, int qt) {
      L.cnt = 0;
      L.lds = tid * 2 + qt;
      if (pr[qt] >= 0) {
        const uint64_t k = o.tau_q[qid[qt]];
        // a bound of FLT_MAX (fewer than 8 rows in all of the query's
        // leaves: every row qualifies) is held just below it, so that the
        // padding rows, which score FLT_MAX, never qualify
        L.tv = fminf(key_score(k), 0x1.fffffcp127f);
        L.tp = key_pos(k);
        L.dst = o.hits + ((int64_t)pr[qt] * 2 + h) * o.hs;
      } else {  // nothing is ever collected for a lane without a pair
        L.tv = -INFINITY;
        L.tp = -1;
        L.dst = o.hits;
      }
    };
    init_lane(L0, 0);
    init_lane(L1, 1);
  }
  if (row_begin < row_end) {
    // stages load two ahead: step st loads
    // stage st + 2 into the registers it frees, computes on LDS buffer st % 2
    // and stores stage st + 1 (loaded two steps earlier) into the other
    // buffer.  The two register sets are named, not indexed, so that they
    // stay in registers.
    auto step = [&](StageRegs<KS, LS_QPB>& Rcur, StageRegs<KS, LS_QPB>& Rnext, int st,
                    int buf) __attribute__((always_inline)) {
      // unconditional (past the end: the last rows again, never stored), so
      // the wait before the store covers only the older stage
      stage_load<KS, LS_QPB>(Rcur, Zb, zbn, row_begin + (int64_t)min(st + 2, nstages - 1) * BB_STAGE, row_end, tid);
      if (wave_active) {
        const int nvalid = min(BB_STAGE, row_end - row_begin - st * BB_STAGE);
        const int p0 = row_begin + st * BB_STAGE;
        if constexpr (PASS != 2) {
          if (nvalid == BB_STAGE) stage_compute_cls_full<KS, PASS == 3>(sm, buf, B, cm, ct, p0, lane);
          else stage_compute_cls<KS, false, PASS == 3>(sm, buf, B, cm, ct, p0, lane, nvalid);
        } else {
          stage_collect<KS>(sm, buf, B, L0, L1, lbuf, o.hc, p0, lane, row_end);
        }
      }
      if (st + 1 < nstages)
        stage_store<KS, LS_QPB>(Rnext, sm, buf ^ 1, tid, row_begin + (int64_t)(st + 1) * BB_STAGE, row_end);
      lds_barrier();
    };
    // every load issued so far (the query operands, the first two stages) is
    // complete before the loop: the wait tracking cannot follow the query
    // operands around the loop and would otherwise wait for them in every
    // stage, draining the row loads issued two stages ahead each time
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    stage_store<KS, LS_QPB>(R0, sm, 0, tid, row_begin, row_end);
    lds_barrier();
    // two steps per trip, the register sets trading roles, so that no copy
    // of a set (which would wait for its loads in flight) is needed
    for (int st = 0; st < nstages; st += 2) {
      step(R0, R1, st, 0);
      if (st + 1 < nstages) step(R1, R0, st + 1, 1);
    }
  }
  if constexpr (PASS == 1) {
    // rows of class c in half h of a tile: i = 8 (c / 4) + 4 h + (c % 4) and
    // i + 16; a class's key takes the later of the two rows of its recorded
    // tile (an upper bound on the position of its minimum) unless that row
    // is past the leaf.  Each half writes its 8 keys, sorted; the classes are
    // disjoint, so the k-th smallest of a query's class keys (over all its
    // pairs) bounds its k-th smallest key from above.
#pragma unroll
    for (int qt = 0; qt < 2; ++qt) {
      uint64_t k[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int ra = ct[qt][c] + 8 * (c >> 2) + 4 * h + (c & 3);
        const int rk = ra + 16 < row_end ? ra + 16 : ra;
        k[c] = ct[qt][c] < 0 ? score_key(FLT_MAX, INT_MAX) : score_key(cm[qt][c], rk);
      }
      sort8(k);
      if (pr[qt] >= 0) {
        uint64_t* dk = o.pair_keys + (int64_t)pr[qt] * 16 + 8 * h;
#pragma unroll
        for (int c = 0; c < 8; ++c) dk[c] = k[c];
      }
    }
  } else if constexpr (PASS == 3) {
    // class-minimum candidates: the pair's 16 class minima (each with the row
    // of its first occurrence), half h's 8 at entries 8 h .. 8 h + 7
#pragma unroll
    for (int qt = 0; qt < 2; ++qt) {
      if (pr[qt] < 0) continue;
      float* dd = o.part_d + (int64_t)pr[qt] * 16 + 8 * h;
      int32_t* di = o.part_i + (int64_t)pr[qt] * 16 + 8 * h;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const bool ok = ct[qt][c] >= 0;
        dd[c] = ok ? cm[qt][c] : FLT_MAX;
        di[c] = ok ? ct[qt][c] + 8 * (c >> 2) + 4 * h + (c & 3) : INT_MAX;
      }
    }
  } else {
    hit_write(L0, lbuf, o.hc);
    hit_write(L1, lbuf, o.hc);
    if (pr[0] >= 0) o.hit_cnt[(int64_t)pr[0] * 2 + h] = L0.cnt;
    if (pr[1] >= 0) o.hit_cnt[(int64_t)pr[1] * 2 + h] = L1.cnt;
  }
}

// Persistent form: one block per compute unit takes tiles from a counter
// (zeroed before the launch) until the list is done, so no block waits for
// the dispatcher between tiles of very different cost.
template <int KS, int PASS>
__global__ __launch_bounds__(LS_QPB) void k_leaf_scan_bf16(const uint16_t* __restrict__ Qb, int P,
                                                        const uint16_t* __restrict__ Zb,
                                                        const float* __restrict__ zbn,
                                                        const int32_t* __restrict__ leaf_off,
                                                        const int32_t* __restrict__ qoff,
                                                        const int32_t* __restrict__ order,
                                                        const int2* __restrict__ tiles,
                                                        const int32_t* __restrict__ ntiles,
                                                        int32_t* __restrict__ next, LeafScanOut o) {
  __shared__ BruteSmem<KS> sm;
  __shared__ int2 s_hits[PASS == 2 ? LS_QPB * 2 * ls_hc_cap<KS>() : 1];
  __shared__ int s_t;
  const int nt = *ntiles;
  for (;;) {
    if (threadIdx.x == 0) s_t = atomicAdd(next, 1);
    __syncthreads();
    const int t = s_t;
    if (t >= nt) break;  // uniform per block; the counter only grows, so every block gets here
    leaf_scan_tile<KS, PASS>(t, sm, Qb, P, Zb, zbn, leaf_off, qoff, order, tiles, o, s_hits);
    __syncthreads();  // LDS buffers and s_t free for the next tile
  }
}

// tau[q] = the K-th smallest class key over the query's scanned pairs (an
// upper bound on its K-th smallest key: the classes hold disjoint rows); a
// pair whose smallest score exceeds the bound's score holds no row within it
// and is left out of the collect pass (pair_leaf2 = -1), the others keep
// their leaf.  Each pair's keys come as two sorted runs of 8, so a run is
// left as soon as one of its keys cannot enter the K smallest.
template <int K>
__global__ __launch_bounds__(256) void k_pair_tau_pool(const int32_t* __restrict__ pair_leaf,
                                                       const uint64_t* __restrict__ pair_keys, int64_t nq, int P,
                                                       uint64_t* __restrict__ tau, int32_t* __restrict__ pair_leaf2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  // (an empty class's key, FLT_MAX: with fewer than K rows in all the
  // query's leaves every row is within the bound)
  uint64_t top[K];
#pragma unroll
  for (int t = 0; t < K; ++t) top[t] = score_key(FLT_MAX, INT_MAX);
  for (int j = 0; j < P; ++j) {
    const int64_t p = q * P + j;
    if (pair_leaf[p] < 0) continue;
    // the pair's 16 keys in eight independent 16-byte loads
    uint64_t kv[16];
    const ulonglong2* kp = reinterpret_cast<const ulonglong2*>(pair_keys + p * 16);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const ulonglong2 u = kp[c];
      kv[2 * c] = u.x;
      kv[2 * c + 1] = u.y;
    }
#pragma unroll
    for (int run = 0; run < 2; ++run) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        uint64_t v = kv[8 * run + c];
        if (v >= top[K - 1]) break;  // the run is sorted: nothing later enters
        // insertion into the sorted list
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const uint64_t lo = v < top[t] ? v : top[t];
          v = v < top[t] ? top[t] : v;
          top[t] = lo;
        }
      }
    }
  }
  const uint64_t b = top[K - 1];
  tau[q] = b;
  const float bv = key_score(b);
  for (int j = 0; j < P; ++j) {
    const int64_t p = q * P + j;
    const int l = pair_leaf[p];
    bool keep = false;
    if (l >= 0) {
      const uint64_t m0 = pair_keys[p * 16], m1 = pair_keys[p * 16 + 8];
      keep = key_score(m0 < m1 ? m0 : m1) <= bv;
    }
    pair_leaf2[p] = keep ? l : -1;
  }
}

// queries with a (pair, half) that collected more rows than it has slots
__global__ __launch_bounds__(256) void k_hit_overflow(const int32_t* __restrict__ pair_leaf,
                                                      const int32_t* __restrict__ hit_cnt, int64_t nq, int P, int hc,
                                                      int32_t* __restrict__ list, int32_t* __restrict__ n) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  bool over = false;
  for (int j = 0; j < P; ++j) {
    const int64_t p = q * P + j;
    if (pair_leaf[p] < 0) continue;
    over = over || hit_cnt[2 * p] > hc || hit_cnt[2 * p + 1] > hc;
  }
  if (over) list[atomicAdd(n, 1)] = (int32_t)q;
}

// The per-query exact top-K (K = 8 or 16) for the overflowed queries, in two kernels.
// Chunks: the query's 32-row tiles (its collect pairs' leaves, pair after
// pair) are dealt to FB_CHUNKS waves in turn; each wave runs the same matrix
// products as the tile kernels (the query in all 32 columns, so each half of
// the wave holds the same 16 rows of a tile: identical scores, the products
// seeing the same operands in the same order), keeps a sorted top-K of
// (score, position) per lane over the rows within the query's bound (only
// those can be among its K smallest keys), merges its two halves and writes
// the K into the query's own slots (chunk c at K c: the query owns P * 2 * hs
// >= K * FB_CHUNKS slots).  Merge: one thread per query takes the K best of
// the chunk lists and leaves them in the slots of its first collect pair
// (count K, contiguous from there; the other counts 0).  Waves and threads loop over the list, whose length
// is read on the device.
constexpr int FB_CHUNKS = 16;
template <int KS, int K>
__global__ __launch_bounds__(256) void k_scan_topk_chunks(const uint16_t* __restrict__ Qb, int P,
                                                          const uint16_t* __restrict__ Zb,
                                                          const float* __restrict__ zbn,
                                                          const int32_t* __restrict__ leaf_off,
                                                          const int32_t* __restrict__ pair_leaf,
                                                          const int32_t* __restrict__ list,
                                                          const int32_t* __restrict__ n,
                                                          const uint64_t* __restrict__ tau_q,
                                                          int2* __restrict__ hits, int hs) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nw = gridDim.x * (blockDim.x >> 6);
  const int64_t items = (int64_t)(*n) * FB_CHUNKS;
  for (int64_t it = gw; it < items; it += nw) {
    const int64_t q = list[it / FB_CHUNKS];
    const int c = (int)(it % FB_CHUNKS);
    // the query's bound from the first pass: only rows at or below it can be
    // among its 8 smallest keys, so the rest skip the insertion
    const uint64_t tk = tau_q[q];
    const float tv = key_score(tk);
    const int tp = key_pos(tk);
    bf16x8 B[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const uint4 u = reinterpret_cast<const uint4*>(Qb + q * (KS * 16))[2 * kk + h];
      B[kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
    TopLex<K> top;
    top.init();
    int g0 = 0;  // tiles of the earlier pairs
    for (int j = 0; j < P; ++j) {
      const int l = pair_leaf[q * P + j];
      if (l < 0) continue;
      const int rb = leaf_off[l], re = leaf_off[l + 1];
      const int nt = (int)ceil_div(re - rb, 32);
      for (int t = (c - g0 % FB_CHUNKS + FB_CHUNKS) % FB_CHUNKS; t < nt; t += FB_CHUNKS) {
        const int t0 = rb + 32 * t;
        const int64_t row = min(t0 + (lane & 31), re - 1);
        bf16x8 A[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
          const uint4 u = reinterpret_cast<const uint4*>(Zb + row * (KS * 16))[2 * kk + h];
          A[kk] = *reinterpret_cast<const bf16x8*>(&u);
        }
        floatx16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = zbn[min(t0 + 8 * (r >> 2) + 4 * h + (r & 3), re - 1)];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[kk], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int pr = t0 + 8 * (r >> 2) + 4 * h + (r & 3);
          const float v = acc[r];
          if (pr < re && (v < tv || (v == tv && pr <= tp)) && lex_lt(v, pr, top.d[K - 1], top.i[K - 1]))
            top.insert(v, pr);
        }
      }
      g0 += nt;
    }
    float od[K];
    int oi[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      od[t] = __shfl_xor(top.d[t], 32, 64);
      oi[t] = __shfl_xor(top.i[t], 32, 64);
    }
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < K; ++t)
        if (lex_lt(od[t], oi[t], top.d[K - 1], top.i[K - 1])) top.insert(od[t], oi[t]);
      int2* dst = hits + (q * P) * 2 * hs + K * c;
#pragma unroll
      for (int t = 0; t < K; ++t) dst[t] = make_int2(__float_as_int(top.d[t]), top.i[t]);
    }
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_scan_topk_merge(int P, const int32_t* __restrict__ pair_leaf,
                                                         const int32_t* __restrict__ list,
                                                         const int32_t* __restrict__ n, int2* __restrict__ hits,
                                                         int32_t* __restrict__ hit_cnt, int hs) {
  const int cnt = *n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const int64_t q = list[i];
    const int2* src = hits + (q * P) * 2 * hs;
    TopLex<K> top;
    top.init();
    // 32 entries loaded together, then inserted in the same order (one
    // memory latency per 32 entries instead of one per entry)
    constexpr int NB = 32;
    static_assert((K * FB_CHUNKS) % NB == 0, "whole batches");
    for (int e0 = 0; e0 < K * FB_CHUNKS; e0 += NB) {
      int2 v[NB];
#pragma unroll
      for (int e = 0; e < NB; ++e) v[e] = src[e0 + e];
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const float sv = __int_as_float(v[e].x);
        if (lex_lt(sv, v[e].y, top.d[K - 1], top.i[K - 1])) top.insert(sv, v[e].y);
      }
    }
    int j0 = 0;  // the first pair the query scans (it has at least one)
    while (j0 + 1 < P && pair_leaf[q * P + j0] < 0) ++j0;
    int2* dst = hits + (q * P + j0) * 2 * hs;
    int m = 0;
    for (int t = 0; t < K; ++t)
      if (top.i[t] != INT_MAX) dst[m++] = make_int2(__float_as_int(top.d[t]), top.i[t]);
    for (int jj = 0; jj < P; ++jj) {
      hit_cnt[(q * P + jj) * 2] = jj == j0 ? m : 0;
      hit_cnt[(q * P + jj) * 2 + 1] = 0;
    }
  }
}

#define PTS_KS_SWITCH(dk, ...)                                                                     \
  switch (dk) {                                                                                    \
    case 32: { constexpr int KSC = 2; __VA_ARGS__; } break;                                        \
    case 64: { constexpr int KSC = 4; __VA_ARGS__; } break;                                        \
    case 96: { constexpr int KSC = 6; __VA_ARGS__; } break;                                        \
    case 128: { constexpr int KSC = 8; __VA_ARGS__; } break;                                       \
    default: ::pts::fail(PTS_ERR_UNSUPPORTED, "bf16 width must be 32/64/96/128");                  \
  }

int brute_splits(int64_t nq) {
  // at least ~4 blocks per CU over 256 CUs; a multiple of the 8 XCDs
  const int64_t qblocks = ceil_div(nq, BB_QPB);
  int S = 8;
  while (qblocks * S < 1024 && S < 64) S *= 2;
  return S;
}

void launch_brute_bf16_topk(Ctx* c, const uint16_t* Qb, int64_t nq, const uint16_t* Zb, const float* zbn, int64_t N,
                            int dk, int S, int kt, const uint64_t* tau_q, float* part_d, int32_t* part_i) {
  ProfScope ps(c, "brute_bf16_topk");
  if (nq == 0) return;
  PTS_REQUIRE(N > 0 && N < INT_MAX, PTS_ERR_ARG, "brute: bad N");
  const int64_t qblocks = ceil_div(nq, BB_QPB);
  const int64_t rows = round_up(ceil_div(N, S), BB_STAGE);
  PTS_REQUIRE(qblocks * S < (int64_t)1 << 31, PTS_ERR_UNSUPPORTED, "brute: grid too large");
  PTS_REQUIRE(kt == 8 || kt == 16, PTS_ERR_ARG, "brute: list length must be 8 or 16");
  if (kt == 8) {
    PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_brute_bf16_topk<KSC, 8>), dim3((unsigned)(qblocks * S)), dim3(BB_QPB), 0,
                                         c->stream, Qb, nq, Zb, zbn, N, S, rows, tau_q, part_d, part_i));
  } else {
    PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_brute_bf16_topk<KSC, 16>), dim3((unsigned)(qblocks * S)), dim3(BB_QPB),
                                         0, c->stream, Qb, nq, Zb, zbn, N, S, rows, tau_q, part_d, part_i));
  }
  check_launch("k_brute_bf16_topk");
}

// pair_leaf[i] = i % S: every query scans every split of the exemplar set
__global__ __launch_bounds__(256) void k_fill_splits(int32_t* __restrict__ pair_leaf, int64_t n, int S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pair_leaf[i] = (int32_t)(i % S);
}

// off[j] = min(N, j * ceil(N / S)), j = 0..S: the row ranges of the splits
__global__ void k_split_offsets(int32_t* __restrict__ off, int S, int64_t N) {
  const int j = threadIdx.x;
  const int64_t per = (N + S - 1) / S;
  if (j <= S) off[j] = (int32_t)min(N, (int64_t)j * per);
}

void launch_split_offsets(Ctx* c, int32_t* off, int S, int64_t N) {
  PTS_REQUIRE(S >= 1 && S <= 255, PTS_ERR_ARG, "split count");
  hipLaunchKernelGGL(k_split_offsets, dim3(1), dim3(256), 0, c->stream, off, S, N);
  check_launch("k_split_offsets");
}

void launch_fill_splits(Ctx* c, int32_t* pair_leaf, int64_t n, int S) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_splits, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, pair_leaf, n, S);
  check_launch("k_fill_splits");
}

static HitLists hit_lists(const ScanHits* sh) {
  HitLists h{};
  if (sh) {
    h.hits = sh->hits;
    h.hit_cnt = sh->hit_cnt;
    h.pair_leaf = sh->pair_leaf;
    h.P = sh->P;
    h.hs = sh->hs;
  }
  return h;
}

// rows[0] += the leaf sizes of the scanned pairs (pair_leaf >= 0): the
// (query, exemplar) score count of a scan over them
__global__ __launch_bounds__(256) void k_scan_rows(const int32_t* __restrict__ pair_leaf, int64_t n,
                                                   const int32_t* __restrict__ leaf_off,
                                                   unsigned long long* __restrict__ rows) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = 0;
  if (p < n) {
    const int l = pair_leaf[p];
    if (l >= 0) v = (unsigned long long)(leaf_off[l + 1] - leaf_off[l]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(rows, v);
}

int64_t count_scan_rows(Ctx* c, const int32_t* pair_leaf, int64_t n, const int32_t* leaf_off) {
  if (n == 0) return 0;
  unsigned long long* d = c->buf<unsigned long long>("ls_rows_count", 1);
  launch_zero_i32(c, reinterpret_cast<int32_t*>(d), 2);
  hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, pair_leaf, n, leaf_off,
                     d);
  check_launch("k_scan_rows");
  unsigned long long h = 0;
  PTS_HIP(hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, c->stream));
  PTS_HIP(hipStreamSynchronize(c->stream));
  return (int64_t)h;
}

void launch_leaf_scan_bf16_bound(Ctx* c, const uint16_t* Qb, int64_t nq, int P, const uint16_t* Zb, const float* zbn,
                                 int dk, const int32_t* leaf_off, const BucketBufs& b, int max_tiles,
                                 const int32_t* pair_leaf, int32_t* pair_leaf2, int K) {
  PTS_REQUIRE(K == 8 || K == 16, PTS_ERR_ARG, "the scan keeps 8 or 16 candidates");
  PTS_REQUIRE(P >= 1 && P <= HL_PMAX, PTS_ERR_ARG, "at most 16 scanned leaves per query");
  const int64_t npairs = nq * P;
  LeafScanOut o{};
  o.pair_keys = c->buf<uint64_t>("ls_pair_keys", (size_t)std::max<int64_t>(1, npairs * 16));
  uint64_t* tau_q = c->buf<uint64_t>("ls_tau_q", (size_t)std::max<int64_t>(1, nq));
  if (nq == 0) return;
  if (max_tiles > 0) {
    ProfScope ps(c, "leaf_scan_bf16");
    int32_t* next = c->buf<int32_t>("ls_next_tile", 1);
    launch_zero_i32(c, next, 1);
    const int grid = std::min(max_tiles, c->n_cu);
    PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_leaf_scan_bf16<KSC, 1>), dim3(grid), dim3(LS_QPB), 0, c->stream, Qb, P,
                                         Zb, zbn, leaf_off, b.off, b.order, b.tiles, b.ntiles, next, o));
    check_launch("k_leaf_scan_bf16 (bound)");
  }
  ProfScope ps(c, "scan_tau_min");
  if (K == 8)
    hipLaunchKernelGGL(k_pair_tau_pool<8>, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, pair_leaf,
                       o.pair_keys, nq, P, tau_q, pair_leaf2);
  else
    hipLaunchKernelGGL(k_pair_tau_pool<16>, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, pair_leaf,
                       o.pair_keys, nq, P, tau_q, pair_leaf2);
  check_launch("k_pair_tau_pool");
}

void launch_leaf_scan_bf16_class(Ctx* c, const uint16_t* Qb, int64_t nq, int P, const uint16_t* Zb, const float* zbn,
                                 int dk, const int32_t* leaf_off, const BucketBufs& b, int max_tiles, float* part_d,
                                 int32_t* part_i) {
  LeafScanOut o{};
  o.part_d = part_d;
  o.part_i = part_i;
  if (nq == 0 || max_tiles <= 0) return;
  ProfScope ps(c, "leaf_scan_bf16_class");
  int32_t* next = c->buf<int32_t>("ls_next_tile", 1);
  launch_zero_i32(c, next, 1);
  const int grid = std::min(max_tiles, c->n_cu);
  PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_leaf_scan_bf16<KSC, 3>), dim3(grid), dim3(LS_QPB), 0, c->stream, Qb, P, Zb,
                                       zbn, leaf_off, b.off, b.order, b.tiles, b.ntiles, next, o));
  check_launch("k_leaf_scan_bf16 (class candidates)");
}

void launch_leaf_scan_bf16_collect(Ctx* c, const uint16_t* Qb, int64_t nq, int P, const uint16_t* Zb,
                                   const float* zbn, int dk, const int32_t* leaf_off, const BucketBufs& b,
                                   int max_tiles, const int32_t* pair_leaf2, int hc, ScanHits* sh,
                                   int32_t* n_overflow, int K) {
  PTS_REQUIRE(K == 8 || K == 16, PTS_ERR_ARG, "the scan keeps 8 or 16 candidates");
  PTS_REQUIRE(hc >= 0 && hc <= LS_HC_MAX, PTS_ERR_ARG, "collect slots must be 0..14");
  int cap = 0;  // fewer fit beside the wider stage buffers of 96 and 128 dimensions
  PTS_KS_SWITCH(dk, cap = ls_hc_cap<KSC>());
  hc = std::min(hc, cap);
  PTS_REQUIRE(P >= 1 && P <= HL_PMAX, PTS_ERR_ARG, "at most 16 scanned leaves per query");
  // slot stride: hc, but room for the per-query pass's chunk lists (and for
  // the K merged entries in the last pair's two halves) too
  const int hs = std::max({hc, (int)ceil_div(K * FB_CHUNKS, 2 * P), (int)ceil_div(K, 2)});
  const int64_t npairs = nq * P;
  LeafScanOut o{};
  o.tau_q = c->buf<uint64_t>("ls_tau_q", (size_t)std::max<int64_t>(1, nq));
  o.hits = c->buf<int2>("ls_hits", (size_t)std::max<int64_t>(1, npairs * 2 * hs));
  o.hit_cnt = c->buf<int32_t>("ls_hit_cnt", (size_t)std::max<int64_t>(1, npairs * 2));
  o.hc = hc;
  o.hs = hs;
  sh->hits = o.hits;
  sh->hit_cnt = o.hit_cnt;
  sh->pair_leaf = pair_leaf2;
  sh->P = P;
  sh->hs = hs;
  if (nq == 0) return;
  if (max_tiles > 0) {
    ProfScope ps(c, "leaf_scan_bf16_collect");
    int32_t* next = c->buf<int32_t>("ls_next_tile", 1);
    launch_zero_i32(c, next, 1);
    const int grid = std::min(max_tiles, c->n_cu);
    PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_leaf_scan_bf16<KSC, 2>), dim3(grid), dim3(LS_QPB), 0, c->stream, Qb, P,
                                         Zb, zbn, leaf_off, b.off, b.order, b.tiles, b.ntiles, next, o));
    check_launch("k_leaf_scan_bf16 (collect)");
  }
  ProfScope ps(c, "scan_overflow");
  int32_t* list = c->buf<int32_t>("ls_ovf_list", (size_t)nq);
  launch_zero_i32(c, n_overflow, 1);
  hipLaunchKernelGGL(k_hit_overflow, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, pair_leaf2,
                     o.hit_cnt, nq, P, hc, list, n_overflow);
  check_launch("k_hit_overflow");
  // waves and threads loop over the list (its length is only known on the device)
  PTS_REQUIRE((int64_t)P * 2 * hs >= K * FB_CHUNKS, PTS_ERR_ARG, "too few collect slots per query");
  if (K == 8) {
    PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_scan_topk_chunks<KSC, 8>), dim3(4 * c->n_cu), dim3(256), 0, c->stream,
                                         Qb, P, Zb, zbn, leaf_off, pair_leaf2, list, n_overflow, o.tau_q, o.hits, hs));
    check_launch("k_scan_topk_chunks");
    hipLaunchKernelGGL(k_scan_topk_merge<8>, dim3(64), dim3(256), 0, c->stream, P, pair_leaf2, list, n_overflow,
                       o.hits, o.hit_cnt, hs);
  } else {
    PTS_KS_SWITCH(dk, hipLaunchKernelGGL((k_scan_topk_chunks<KSC, 16>), dim3(4 * c->n_cu), dim3(256), 0, c->stream,
                                         Qb, P, Zb, zbn, leaf_off, pair_leaf2, list, n_overflow, o.tau_q, o.hits, hs));
    check_launch("k_scan_topk_chunks");
    hipLaunchKernelGGL(k_scan_topk_merge<16>, dim3(64), dim3(256), 0, c->stream, P, pair_leaf2, list, n_overflow,
                       o.hits, o.hit_cnt, hs);
  }
  check_launch("k_scan_topk_merge");
}

// ---------------------------------------------------------------------------
// merge the S partial top-k lists of a query and re-rank the k survivors by
// the FP32 distance in PCA space; nn = original id (ties to the lowest id)

// list s of query q is row (q * qs + s * ss) of part [..][8]; a list whose
// valid[] entry is negative is skipped (valid == NULL: all lists valid).
template <int DP, int KL>
__global__ __launch_bounds__(256) void k_merge_rerank_pca(const float* __restrict__ part_d,
                                                          const int32_t* __restrict__ part_i, int64_t nq, int S,
                                                          int64_t qs, int64_t ss, const int32_t* __restrict__ valid,
                                                          HitLists hl, int k, const float* __restrict__ Qp,
                                                          const float* __restrict__ Zp,
                                                          const float* __restrict__ zres,
                                                          const int32_t* __restrict__ perm, int64_t N,
                                                          int32_t* __restrict__ cand_out,
                                                          int32_t* __restrict__ nn) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  TopLex<KL> top;
  top.init();
  if (hl.hits) {
    top8_from_hits(top, hl, q);
  } else {
    for (int s = 0; s < S; ++s) {
      const int64_t row = q * qs + (int64_t)s * ss;
      if (valid && valid[row] < 0) continue;
      const float* pd = part_d + row * KL;
      const int32_t* pi = part_i + row * KL;
      for (int t = 0; t < KL; ++t)
        if (lex_lt(pd[t], pi[t], top.d[KL - 1], top.i[KL - 1])) top.insert(pd[t], pi[t]);
    }
  }
  if (!nn) {  // candidates only (the first 8; a full-D re-rank follows)
#pragma unroll
    for (int t = 0; t < BB_TOPK; ++t) {
      const int pos = top.i[t];
      cand_out[q * BB_TOPK + t] = (t < k && pos >= 0 && pos < N) ? perm[pos] : -1;
    }
    return;
  }
  float qv[DP];
#pragma unroll
  for (int kq = 0; kq < DP; kq += 4) {
    const float4 v = *reinterpret_cast<const float4*>(Qp + q * DP + kq);
    qv[kq] = v.x;
    qv[kq + 1] = v.y;
    qv[kq + 2] = v.z;
    qv[kq + 3] = v.w;
  }
  float best = FLT_MAX;
  int bid = INT_MAX;
#pragma unroll
  for (int t = 0; t < KL; ++t) {
    const int pos = top.i[t];
    if (cand_out && t < BB_TOPK) cand_out[q * BB_TOPK + t] = (t < k && pos >= 0 && pos < N) ? perm[pos] : -1;
    if (t >= k || pos < 0 || pos >= N) continue;
    const float* zr = Zp + (int64_t)pos * DP;
    float acc = 0.f;
#pragma unroll
    for (int kq = 0; kq < DP; kq += 4) {
      const float4 z = *reinterpret_cast<const float4*>(zr + kq);
      const float t0 = qv[kq] - z.x, t1 = qv[kq + 1] - z.y, t2 = qv[kq + 2] - z.z, t3 = qv[kq + 3] - z.w;
      acc = fmaf(t0, t0, acc);
      acc = fmaf(t1, t1, acc);
      acc = fmaf(t2, t2, acc);
      acc = fmaf(t3, t3, acc);
    }
    if (zres) acc += zres[pos];
    const int id = perm[pos];
    if (acc < best || (acc == best && id < bid)) {
      best = acc;
      bid = id;
    }
  }
  nn[q] = (bid == INT_MAX) ? -1 : bid;
}

void launch_merge_rerank_pca(Ctx* c, const float* part_d, const int32_t* part_i, int64_t nq, int S, int64_t qs,
                             int64_t ss, const int32_t* valid, const ScanHits* sh, int k, const float* Qp, int dp,
                             const float* Zp, const float* zres, const int32_t* perm, int64_t N, int32_t* cand_out,
                             int32_t* nn, int list_len) {
  ProfScope ps(c, "merge_rerank");
  if (nq == 0) return;
  PTS_REQUIRE(k >= 1 && k <= 16, PTS_ERR_ARG, "topk must be 1..16");
  PTS_REQUIRE(list_len == 0 || list_len == 8 || list_len == 16, PTS_ERR_ARG, "candidate lists hold 8 or 16");
  const int kl = list_len ? list_len : (k <= 8 ? 8 : 16);
  PTS_REQUIRE(k <= kl, PTS_ERR_ARG, "more candidates asked for than the lists hold");
  const HitLists hl = hit_lists(sh);
  if (kl == 8) {
    PTS_DP_SWITCH(dp, hipLaunchKernelGGL((k_merge_rerank_pca<DPC, 8>), dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0,
                                         c->stream, part_d, part_i, nq, S, qs, ss, valid, hl, k, Qp, Zp, zres, perm, N,
                                         cand_out, nn));
  } else {
    PTS_DP_SWITCH(dp, hipLaunchKernelGGL((k_merge_rerank_pca<DPC, 16>), dim3((unsigned)ceil_div(nq, 256)), dim3(256),
                                         0, c->stream, part_d, part_i, nq, S, qs, ss, valid, hl, k, Qp, Zp, zres, perm,
                                         N, cand_out, nn));
  }
  check_launch("k_merge_rerank_pca");
}

// Merge of the partial candidate lists of a query followed by the re-rank of
// the best k in full dimension, fused.  Phase 1: one thread per query merges
// its lists (each sorted by (score, position)) into the 8 best by (score,
// position) and maps positions to exemplar ids in LDS.  Phase 2: 16 lanes
// per query (4 queries per wave at a time) gather the query window and the k
// candidate windows pixel by pixel from the two images, reduce the 8
// squared distances with a halving butterfly, and keep the smallest (ties:
// lower exemplar id).  Writes nn and, if dist is given, the full-D distance
// of the winner.

constexpr int SR_QPB = 256;

// PK: the exemplar windows come from its 8-bit form (pk, srow), rebuilt as
// the same floats the RGBS image holds (channel value / 255, the row's
// guidance value), at 4 bytes a pixel instead of 16.  The PK forms run four
// waves per SIMD (at most 128 registers; the gathers are latency bound and
// the fourth wave hides more of it than the registers it costs: 0.53 against
// 0.59 ms for 8 candidates per query, 0.84 against 0.91 for 12).
template <bool PK, int KL>
__global__ __launch_bounds__(SR_QPB) __attribute__((amdgpu_waves_per_eu(PK ? 4 : 1))) void k_select_rerank_full(
    const float* __restrict__ part_d, const int32_t* __restrict__ part_i, int64_t nq, int S, int64_t qs, int64_t ss,
    const int32_t* __restrict__ valid, HitLists hl, int k, const int32_t* __restrict__ perm, int64_t npos,
    const float4* __restrict__ x, int W, int w, int s, int cols, const float4* __restrict__ ex,
    const uint32_t* __restrict__ pk, const float* __restrict__ srow, int Hz, int Wz, int32_t* __restrict__ nn,
    float* __restrict__ dist) {
  // per query of the block (phase 1, one thread each): the candidates' window
  // origins (pixel index, row; row -1 for no candidate) and the query window's
  // row and column, so that the 16 lanes of a query in phase 2 do no index
  // arithmetic of their own beyond the winner's id
  __shared__ int32_t cbase[KL][SR_QPB];
  __shared__ int32_t crow[KL][SR_QPB];
  __shared__ int32_t qvu[2][SR_QPB];
  const int tid = threadIdx.x;
  const int64_t q0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SR_QPB;
  const int nu = Wz - w + 1;
  const int64_t N = (int64_t)(Hz - w + 1) * nu;
  {
    const int64_t q = q0 + tid;
    TopLex<KL> top;
    top.init();
    if (q < nq && hl.hits) {
      top8_from_hits(top, hl, q);
    } else if (q < nq) {
      for (int li = 0; li < S; ++li) {
        const int64_t row = q * qs + (int64_t)li * ss;
        if (valid && valid[row] < 0) continue;
        float dv[KL];
        int iv[KL];
#pragma unroll
        for (int t4 = 0; t4 < KL / 4; ++t4) {
          const float4 da = reinterpret_cast<const float4*>(part_d + row * KL)[t4];
          const int4 ia = reinterpret_cast<const int4*>(part_i + row * KL)[t4];
          dv[4 * t4] = da.x;
          dv[4 * t4 + 1] = da.y;
          dv[4 * t4 + 2] = da.z;
          dv[4 * t4 + 3] = da.w;
          iv[4 * t4] = ia.x;
          iv[4 * t4 + 1] = ia.y;
          iv[4 * t4 + 2] = ia.z;
          iv[4 * t4 + 3] = ia.w;
        }
#pragma unroll
        for (int t = 0; t < KL; ++t) {
          // once nothing in the wave improves on the last kept entry, skip the insertion network
          if (__any(lex_lt(dv[t], iv[t], top.d[KL - 1], top.i[KL - 1]))) top.insert(dv[t], iv[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < KL; ++t) {
      const int pos = top.i[t];
      const int e = (t < k && pos >= 0 && pos < npos) ? perm[pos] : -1;
      const bool ok = e >= 0 && e < N;
      const int ee = ok ? e : 0;  // an in-bounds window, result discarded in phase 2
      const int ey = ee / nu;
      cbase[t][tid] = ey * Wz + (ee - ey * nu);
      crow[t][tid] = ok ? ey : -1;
    }
    const int64_t qc = q < nq ? q : 0;
    const int qi = (int)(qc / cols);
    qvu[0][tid] = qi * s;
    qvu[1][tid] = (int)(qc - (int64_t)qi * cols) * s;
  }
  __syncthreads();
  const int lane = tid & 63, g = lane & 15, grp = lane >> 4;
  const int npx = w * w;
  const int ci = ((g >> 3) & 1) * 4 + ((g >> 2) & 1) * 2 + ((g >> 1) & 1);  // candidate held after the butterfly
  for (int it = 0; it < SR_QPB / 16; ++it) {
    const int ql = (tid >> 6) * 64 + it * 4 + grp;
    const int64_t q = q0 + ql;
    if (q >= nq) continue;  // uniform per 16-lane group; shuffles stay inside the group
    const int v = qvu[0][ql], u = qvu[1][ql];
    float bbd = FLT_MAX;
    int bbi = INT_MAX;
    // the candidates in groups of 8 (one group unless more than 8 are re-ranked; a last
    // group of at most 4 gathers 4 windows)
#pragma unroll
    for (int cg = 0; cg < KL; cg += 8) {
      if (cg >= k) break;  // lists longer than the candidates re-ranked
      // 32-bit byte offsets of the windows' origins in the 8-bit form (pixel
      // indices below 2^26): loads from a scalar base plus a 32-bit offset
      uint32_t eb[8];
      int eyc[8];
      float acc[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = 0.f;
      // NC windows gathered: 4 when the group holds no more candidates than
      // that (the rest keep a zero sum and are masked after the butterfly)
      auto gather = [&](auto ncv) {
        constexpr int NC = decltype(ncv)::value;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          eb[c] = PK ? (uint32_t)cbase[cg + c][ql] * 4u : (uint32_t)cbase[cg + c][ql];
          eyc[c] = max(crow[cg + c][ql], 0);
        }
        int dy = 0, dx = g;
        while (dx >= w) {
          dx -= w;
          ++dy;
        }
#pragma unroll 4
        for (int p = g; p < npx; p += 16) {
          int xx = u + dx;
          if (xx >= W) xx -= W;
          const float4 a = x[(int64_t)(v + dy) * W + xx];
          const uint32_t eo = (uint32_t)(dy * Wz + dx) * (PK ? 4u : 1u);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            float4 b;
            if constexpr (PK) {
              // the rounded products, as stored in the RGBS image (contraction
              // off: not fused into the subtraction below)
#pragma clang fp contract(off)
              const float inv = 1.0f / 255.0f;
              const uint32_t pv = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(pk) + (eb[c] + eo));
              b.x = (float)(pv & 255u) * inv;
              b.y = (float)((pv >> 8) & 255u) * inv;
              b.z = (float)((pv >> 16) & 255u) * inv;
              b.w = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(srow) + (uint32_t)(eyc[c] + dy) * 4u);
            } else {
              b = ex[eb[c] + eo];
            }
            const float t0 = a.x - b.x, t1 = a.y - b.y, t2 = a.z - b.z, t3 = a.w - b.w;
            acc[c] = fmaf(t0, t0, acc[c]);
            acc[c] = fmaf(t1, t1, acc[c]);
            acc[c] = fmaf(t2, t2, acc[c]);
            acc[c] = fmaf(t3, t3, acc[c]);
          }
          dx += 16;
          while (dx >= w) {
            dx -= w;
            ++dy;
          }
        }
      };
      if (k - cg <= 4) gather(std::integral_constant<int, 4>{});
      else gather(std::integral_constant<int, 8>{});
      // halving butterfly over the 16 lanes: after it, lane g holds the full
      // sum of candidate ci(g) (lanes g and g^1 hold the same one)
      float b4[4];
      const bool h8 = g & 8, h4 = g & 4, h2 = g & 2;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float keep = h8 ? acc[t + 4] : acc[t];
        const float send = h8 ? acc[t] : acc[t + 4];
        b4[t] = keep + __shfl_xor(send, 8, 64);
      }
      float b2[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float keep = h4 ? b4[t + 2] : b4[t];
        const float send = h4 ? b4[t] : b4[t + 2];
        b2[t] = keep + __shfl_xor(send, 4, 64);
      }
      float tot;
      {
        const float keep = h2 ? b2[1] : b2[0];
        const float send = h2 ? b2[0] : b2[1];
        tot = keep + __shfl_xor(send, 2, 64);
      }
      tot += __shfl_xor(tot, 1, 64);
      // the candidate's exemplar id from its window origin
      const int ey = crow[cg + ci][ql];
      const int e = ey * nu + (cbase[cg + ci][ql] - ey * Wz);
      float bd = (cg + ci < k && ey >= 0) ? tot : FLT_MAX;
      int bi = (cg + ci < k && ey >= 0) ? e : INT_MAX;
#pragma unroll
      for (int off = 2; off <= 8; off <<= 1) {
        const float od = __shfl_xor(bd, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (lex_lt(od, oi, bd, bi)) {
          bd = od;
          bi = oi;
        }
      }
      if (lex_lt(bd, bi, bbd, bbi)) {
        bbd = bd;
        bbi = bi;
      }
    }
    const float bd = bbd;
    const int bi = bbi;
    if (g == 0) {
      nn[q] = (bi == INT_MAX) ? -1 : bi;
      if (dist) dist[q] = (bi == INT_MAX) ? __int_as_float(0x7fc00000) : sqrtf(bd);
    }
  }
}

void launch_select_rerank_full(Ctx* c, const float* part_d, const int32_t* part_i, int64_t nq, int S, int64_t qs,
                               int64_t ss, const int32_t* valid, const ScanHits* sh, int k, const int32_t* perm,
                               int64_t npos,
                               const float* x, int H, int W, int w, int s, const float* ex, const uint32_t* ex_pk,
                               const float* ex_srow, int Hz, int Wz, int32_t* nn, float* dist, int list_len) {
  ProfScope ps(c, "select_rerank_full");
  if (nq == 0) return;
  PTS_REQUIRE(k >= 1 && k <= 16, PTS_ERR_ARG, "topk must be 1..16");
  PTS_REQUIRE(list_len == 0 || list_len == 8 || list_len == 16, PTS_ERR_ARG, "candidate lists hold 8 or 16");
  const int kl = list_len ? list_len : (k <= 8 ? 8 : 16);
  PTS_REQUIRE(k <= kl, PTS_ERR_ARG, "more candidates asked for than the lists hold");
  PTS_REQUIRE(w >= 1 && w <= Hz && w <= Wz && w <= H && W % s == 0, PTS_ERR_ARG, "select_rerank_full: bad geometry");
  const dim3 grid((unsigned)ceil_div(nq, SR_QPB));
  const HitLists hl = hit_lists(sh);
  auto go = [&](auto PKV, auto KLV) {
    hipLaunchKernelGGL((k_select_rerank_full<decltype(PKV)::value, decltype(KLV)::value>), grid, dim3(SR_QPB), 0,
                       c->stream, part_d, part_i, nq, S, qs, ss, valid, hl, k, perm, npos,
                       reinterpret_cast<const float4*>(x), W, w, s, W / s, reinterpret_cast<const float4*>(ex), ex_pk,
                       ex_srow, Hz, Wz, nn, dist);
  };
  const bool pk = ex_pk && ex_srow;
  using T = std::true_type;
  using F = std::false_type;
  using K8 = std::integral_constant<int, 8>;
  using K16 = std::integral_constant<int, 16>;
  if (kl == 8) {
    if (pk) go(T{}, K8{});
    else go(F{}, K8{});
  } else {
    if (pk) go(T{}, K16{});
    else go(F{}, K16{});
  }
  check_launch("k_select_rerank_full");
}

}  // namespace pts
