// Leaf-proposal MLP kernels: a small network maps a PCA-reduced query to
// scores over the leaves of the k-means search tree, so a query can be sent
// to its most likely leaves directly (the tree of Methodology 2.2 stays the
// fallback).  Layers n_in -> h -> h -> n_out, GELU(x) = x Phi(x) with the
// exact error function.
//
// Training (FP32 master weights): tiled GEMMs on the vector ALU in three
// transpose forms (forward A W^T, input gradient G W, weight gradient
// G^T A), optionally with both operands rounded to bf16 (products exact in
// FP32, FP32 accumulation - the arithmetic of the matrix-core path), plus
// bias/GELU, softmax cross-entropy, GELU backward, column sums and Adam.
// Every reduction has a fixed order, so a training run is reproducible.
//
// Inference (bf16 weights, FP32 accumulation) on the matrix cores
// (v_mfma_f32_32x32x16_bf16): A = 32 weight rows, B = 32 queries, so each
// lane owns half of one query's 32 output features of a tile (16 values);
// weight tiles stream through LDS shared by the block's 8 waves (256
// queries).  Both hidden layers run in one kernel and write GELU(acc + b) of
// the second as bf16; the output layer never writes logits: two passes over
// its weight tiles give the exact top-P leaves (descending, ties to the lower
// leaf) and the softmax margin, the two lanes of a query merging at the end.
#include <algorithm>
#include <cfloat>
#include <utility>
#include <type_traits>
#include <climits>

#include "kernels_mlp.hpp"

namespace pts {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float round_bf16f(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return __uint_as_float(b & 0xFFFF0000u);
}

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

// Inference GELU: Phi(x) = 1/2 + x P(x^2), |x| clamped to c = 4, P of degree
// 7, a near-minimax fit (coefficients from fit_phi_poly.py beside this
// package); |error| <= 5.3e-5 in Phi and <= 4.2e-4 in GELU for |x| <= 8, and
// wherever |GELU| >= 0.05 a relative error below a quarter of the bf16
// half-unit that rounds the activation next.  11 VALU operations against ~40
// for erff.
__device__ __forceinline__ float gelu_poly_f(float x) {
  constexpr float c = 4.0f;
  const float xc = __builtin_amdgcn_fmed3f(x, -c, c);
  const float u = xc * xc;
  float p = -1.580823805e-09f;
  p = fmaf(p, u, 1.217132137e-07f);
  p = fmaf(p, u, -4.100912975e-06f);
  p = fmaf(p, u, 8.066791634e-05f);
  p = fmaf(p, u, -1.048207399e-03f);
  p = fmaf(p, u, 9.664882906e-03f);
  p = fmaf(p, u, -6.617539376e-02f);
  p = fmaf(p, u, 3.988475204e-01f);
  return x * fmaf(xc, p, 0.5f);
}

__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---------------------------------------------------------------------------
// GEMM (vector ALU): C[M][N] = op(A) op(B); op(A) is M x K, op(B) is K x N.
// TA: A stored [K][M] (else [M][K]); TB: B stored [N][K] (else [K][N]).
// 256 threads, 64 x 64 tile, K chunks of 16; thread owns 4 x 4 outputs.

// Split over K when the output has few tiles: slice z = blockIdx.z covers
// k in [z kc, (z + 1) kc) and writes its partial product to P[z]; the
// slices are then summed in order (k_splitk_sum).  With one slice the block
// writes C directly.
template <bool TA, bool TB, bool BF>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, const float* __restrict__ B,
                                              float* __restrict__ C, int M, int N, int K, int accumulate, int kc,
                                              float* __restrict__ P) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tid = threadIdx.x, tm = tid & 15, tn = tid >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int t = tid; t < 16 * 64; t += 256) {
      // A chunk: element (k, m)
      int kk, mm;
      if (TA) {
        kk = t / 64;
        mm = t % 64;
      } else {
        mm = t / 16;
        kk = t % 16;
      }
      const int gk = k0 + kk, gm = m0 + mm;
      float va = 0.f;
      if (gk < ke && gm < M) va = TA ? A[(int64_t)gk * M + gm] : A[(int64_t)gm * K + gk];
      As[kk][mm] = BF ? round_bf16f(va) : va;
      int kb, nb;
      if (TB) {
        nb = t / 16;
        kb = t % 16;
      } else {
        kb = t / 64;
        nb = t % 64;
      }
      const int gkb = k0 + kb, gn = n0 + nb;
      float vb = 0.f;
      if (gkb < ke && gn < N) vb = TB ? B[(int64_t)gn * K + gkb] : B[(int64_t)gkb * N + gn];
      Bs[kb][nb] = BF ? round_bf16f(vb) : vb;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[k][tm + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[k][tn + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int gm = m0 + tm + 16 * a;
    if (gm >= M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int gn = n0 + tn + 16 * b;
      if (gn >= N) continue;
      if (gridDim.z > 1) {
        P[((int64_t)blockIdx.z * M + gm) * N + gn] = acc[a][b];
      } else {
        float* dst = C + (int64_t)gm * N + gn;
        *dst = accumulate ? *dst + acc[a][b] : acc[a][b];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_splitk_sum(const float* __restrict__ P, int S, int64_t n,
                                                    float* __restrict__ C, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += P[(int64_t)z * n + i];
  C[i] = accumulate ? C[i] + s : s;
}

unsigned eblocks(int64_t n) { return (unsigned)ceil_div(n, 256); }

void launch_gemm(Ctx* c, bool ta, bool tb, bool bf, const float* A, const float* B, float* C, int M, int N, int K,
                 bool accumulate) {
  ProfScope ps(c, "mlp_gemm");
  if (M == 0 || N == 0) return;
  // enough blocks to fill the chip: split K when the output has few tiles
  const int64_t tiles = ceil_div(N, 64) * ceil_div(M, 64);
  int S = 1;
  if (tiles < 512 && K >= 256) S = (int)std::min<int64_t>({16, ceil_div(512, tiles), K / 128});
  const int kc = (int)round_up(ceil_div(std::max(K, 1), S), 16);
  S = (int)ceil_div(std::max(K, 1), kc);
  float* P = S > 1 ? c->buf<float>("gemm_splitk", (size_t)S * M * N) : nullptr;
  dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64), (unsigned)S);
#define PTS_GEMM(TA_, TB_, BF_) \
  hipLaunchKernelGGL((k_gemm<TA_, TB_, BF_>), grid, dim3(256), 0, c->stream, A, B, C, M, N, K, accumulate ? 1 : 0, \
                     kc, P)
  if (!ta && tb && !bf) PTS_GEMM(false, true, false);
  else if (!ta && tb && bf) PTS_GEMM(false, true, true);
  else if (!ta && !tb && !bf) PTS_GEMM(false, false, false);
  else if (!ta && !tb && bf) PTS_GEMM(false, false, true);
  else if (ta && !tb && !bf) PTS_GEMM(true, false, false);
  else if (ta && !tb && bf) PTS_GEMM(true, false, true);
  else fail(PTS_ERR_ARG, "gemm: unsupported transpose form");
#undef PTS_GEMM
  check_launch("k_gemm");
  if (S > 1) {
    hipLaunchKernelGGL(k_splitk_sum, dim3(eblocks((int64_t)M * N)), dim3(256), 0, c->stream, P, S, (int64_t)M * N, C,
                       accumulate ? 1 : 0);
    check_launch("k_splitk_sum");
  }
}

// ---------------------------------------------------------------------------
// elementwise pieces

// X[b][k] = Q[idx[b]][k] * scale[k] (k < n_in, Q rows of stride ld);
// labels gathered the same way.  idx == NULL: rows 0..n-1.
__global__ __launch_bounds__(256) void k_gather_scale(const float* __restrict__ Q, int ld, const float* __restrict__ scale,
                                                      int n_in, const int64_t* __restrict__ idx,
                                                      const int32_t* __restrict__ lab_in, int64_t n,
                                                      float* __restrict__ X, int32_t* __restrict__ lab_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n_in) return;
  const int64_t b = t / n_in;
  const int k = (int)(t - b * n_in);
  const int64_t r = idx ? idx[b] : b;
  X[t] = Q[r * ld + k] * scale[k];
  if (k == 0 && lab_out) lab_out[b] = lab_in[r];
}

// minibatch indices from a counter-based hash (splitmix64 finaliser)
__global__ __launch_bounds__(256) void k_sample_idx(uint64_t seed, int64_t step, int batch, int64_t n,
                                                    int64_t* __restrict__ idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(step * batch + b + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  idx[b] = (int64_t)(z % (uint64_t)n);
}

__global__ __launch_bounds__(256) void k_bias_act(float* __restrict__ Z, float* __restrict__ H,
                                                  const float* __restrict__ bias, int64_t M, int N, int gelu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  const int n = (int)(t % N);
  const float z = Z[t] + bias[n];
  Z[t] = z;
  if (gelu) H[t] = gelu_f(z);
}

// one wave per row: loss_row = lse - L[label]; G = (softmax - onehot) / M
__global__ __launch_bounds__(256) void k_softmax_ce(const float* __restrict__ L, const int32_t* __restrict__ lab,
                                                    int64_t M, int N, float* __restrict__ G,
                                                    float* __restrict__ row_loss) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= M) return;
  const float* lr = L + r * N;
  float m = -FLT_MAX;
  for (int j = lane; j < N; j += 64) m = fmaxf(m, lr[j]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  float s = 0.f;
  for (int j = lane; j < N; j += 64) s += expf(lr[j] - m);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  const float inv = 1.0f / s;
  const int y = lab[r];
  const float scale = 1.0f / (float)M;
  for (int j = lane; j < N; j += 64) {
    const float p = expf(lr[j] - m) * inv;
    G[r * N + j] = (p - (j == y ? 1.0f : 0.0f)) * scale;
  }
  if (lane == 0) row_loss[r] = (m + logf(s)) - ((y >= 0 && y < N) ? lr[y] : 0.f);
}

__global__ __launch_bounds__(256) void k_gelu_bwd(float* __restrict__ dH, const float* __restrict__ Z, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  dH[t] *= gelu_grad_f(Z[t]);
}

// out[n] = sum_m G[m][n]: segments of CS_ROWS rows summed in row order into
// part[seg][n], then the segments summed in order (a fixed order: the
// result does not depend on the launch).
constexpr int CS_ROWS = 64;

__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ G, int64_t M, int N,
                                                     float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t seg = blockIdx.y;
  if (n >= N) return;
  const int64_t m0 = seg * CS_ROWS, m1 = min(M, m0 + CS_ROWS);
  float s = 0.f;
  for (int64_t m = m0; m < m1; ++m) s += G[m * N + n];
  part[seg * N + n] = s;
}

__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part, int nseg, int N,
                                                      float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int g = 0; g < nseg; ++g) s += part[(int64_t)g * N + n];
  out[n] = s;
}

__global__ __launch_bounds__(256) void k_mean(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] / (float)n;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(256) void k_pad_f32(const float* __restrict__ src, int n, int n_p, float fill,
                                                 float* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_p) dst[t] = t < n ? src[t] : fill;
}

// dst [rows_p][cols_p] = bf16(src [rows][cols]), zero padded; with perm, the
// columns of each group of 16 are reordered to the matrix-core lane order
// (dst column k holds src column swap_bits23(k))
__global__ __launch_bounds__(256) void k_to_bf16_pad(const float* __restrict__ src, int rows, int cols, int rows_p,
                                                     int cols_p, int perm, uint16_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows_p * cols_p) return;
  const int r = (int)(t / cols_p), k = (int)(t % cols_p);
  const int cc = perm ? ((k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1)) : k;
  dst[t] = (r < rows && cc < cols) ? bf16_bits(src[(int64_t)r * cols + cc]) : (uint16_t)0;
}


void launch_sample_idx(Ctx* c, uint64_t seed, int64_t step, int batch, int64_t n, int64_t* idx) {
  hipLaunchKernelGGL(k_sample_idx, dim3(eblocks(batch)), dim3(256), 0, c->stream, seed, step, batch, n, idx);
  check_launch("k_sample_idx");
}
void launch_gather_scale(Ctx* c, const float* Q, int ld, const float* scale, int n_in, const int64_t* idx,
                         const int32_t* lab_in, int64_t n, float* X, int32_t* lab_out) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_scale, dim3(eblocks(n * n_in)), dim3(256), 0, c->stream, Q, ld, scale, n_in, idx, lab_in,
                     n, X, lab_out);
  check_launch("k_gather_scale");
}
void launch_bias_act(Ctx* c, float* Z, float* H, const float* bias, int64_t M, int N, bool gelu) {
  if (M == 0) return;
  hipLaunchKernelGGL(k_bias_act, dim3(eblocks(M * N)), dim3(256), 0, c->stream, Z, H, bias, M, N, gelu ? 1 : 0);
  check_launch("k_bias_act");
}
void launch_softmax_ce(Ctx* c, const float* L, const int32_t* lab, int64_t M, int N, float* G, float* row_loss) {
  if (M == 0) return;
  hipLaunchKernelGGL(k_softmax_ce, dim3((unsigned)ceil_div(M, 4)), dim3(256), 0, c->stream, L, lab, M, N, G, row_loss);
  check_launch("k_softmax_ce");
}
void launch_gelu_bwd(Ctx* c, float* dH, const float* Z, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gelu_bwd, dim3(eblocks(n)), dim3(256), 0, c->stream, dH, Z, n);
  check_launch("k_gelu_bwd");
}
void launch_colsum(Ctx* c, const float* G, int64_t M, int N, float* out) {
  const int nseg = (int)std::max<int64_t>(1, ceil_div(M, CS_ROWS));
  PTS_REQUIRE(nseg < 65536, PTS_ERR_UNSUPPORTED, "colsum: too many rows");
  float* part = c->buf<float>("colsum_part", (size_t)nseg * N);
  hipLaunchKernelGGL(k_colsum_part, dim3(eblocks(N), nseg), dim3(256), 0, c->stream, G, M, N, part);
  check_launch("k_colsum_part");
  hipLaunchKernelGGL(k_colsum_final, dim3(eblocks(N)), dim3(256), 0, c->stream, part, nseg, N, out);
  check_launch("k_colsum_final");
}
void launch_mean(Ctx* c, const float* v, int64_t n, float* out) {
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, c->stream, v, n, out);
  check_launch("k_mean");
}
void launch_adam(Ctx* c, float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                 float eps, int64_t t) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(eblocks(n)), dim3(256), 0, c->stream, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  check_launch("k_adam");
}
void launch_pad_f32(Ctx* c, const float* src, int n, int n_p, float fill, float* dst) {
  hipLaunchKernelGGL(k_pad_f32, dim3(eblocks(n_p)), dim3(256), 0, c->stream, src, n, n_p, fill, dst);
  check_launch("k_pad_f32");
}

void launch_to_bf16_pad(Ctx* c, const float* src, int rows, int cols, int rows_p, int cols_p, bool perm,
                        uint16_t* dst) {
  PTS_REQUIRE(!perm || cols_p % 16 == 0, PTS_ERR_ARG, "to_bf16_pad: permuted width must be a multiple of 16");
  hipLaunchKernelGGL(k_to_bf16_pad, dim3(eblocks((int64_t)rows_p * cols_p)), dim3(256), 0, c->stream, src, rows, cols,
                     rows_p, cols_p, perm ? 1 : 0, dst);
  check_launch("k_to_bf16_pad");
}

// ---------------------------------------------------------------------------
// matrix-core inference
//
// v_mfma_f32_32x32x16_bf16 with A = 32 weight rows (neurons), B = 32
// queries: lane l supplies query l % 32 and the 8 k-values 16 kk + 8 (l / 32)
// + 0..7 of k-chunk kk, and receives 16 outputs of its query: neurons
// 32 T + 8 g + 4 (l / 32) + i of tile T (g, i = 0..3, register 4 g + i).
// Registers 8 c .. 8 c + 7 of tile T are therefore exactly a B operand of
// the next layer if that layer's k-chunk 2 T + c lists its neurons in the
// order in which the lanes hold them: k = 16 kk + 8 h + j stands for neuron
// 16 kk + 8 (j / 4) + 4 h + j % 4, i.e. bits 2 and 3 of k swapped.  The bf16
// copies of W2 and W3 have their columns permuted that way, so the hidden
// activations go from one layer to the next without leaving the registers,
// and the second hidden layer is stored in that same order for the output
// layer.

constexpr int ML_WAVES = 8;
constexpr int ML_THREADS = ML_WAVES * 64;
constexpr int ML_QPB = ML_WAVES * 32;  // queries per block (one 32-query tile per wave)
constexpr int ML_P = 8;                // most proposals per query
constexpr float ML_LOG2E = 1.4426950408889634f;

__device__ __forceinline__ int swap_bits23(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }

// Workgroup barrier for the LDS double buffers: this wave's LDS reads and
// writes complete, then s_barrier.  Unlike __syncthreads() it does not wait
// for the wave's global loads, so a weight-tile prefetch stays in flight
// across the barrier.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int KS>
struct WTile {
  static constexpr int CH = KS * 2, NCH = 32 * CH, PER = (NCH + ML_THREADS - 1) / ML_THREADS;
};

// Staging registers of one weight tile: at most two 16-byte chunks per
// thread (32 rows x 16 KS bf16 over 512 threads, KS <= 16) and one bias.
// Plain scalars, so they never become a memory object.
struct TileRegs {
  uint4 c0, c1;
  float b;
};

// One 32-row weight tile (rows n0 .. n0+31 of W [.][16 KS] bf16, which the
// caller pads to whole tiles) into registers.  The loads carry no condition
// (threads past the tile's chunks re-read its last chunk and do not store
// it), so the registers are not touched until the store: the compiler waits
// for them only there and a prefetch stays in flight across the matrix
// products.
template <int KS>
__device__ __forceinline__ uint4 wt_chunk(const uint16_t* __restrict__ Wb, int n0, int cidx) {
  cidx = min(cidx, WTile<KS>::NCH - 1);
  const int row = cidx / WTile<KS>::CH, ch = cidx - row * WTile<KS>::CH;
  return reinterpret_cast<const uint4*>(Wb + (int64_t)(n0 + row) * (KS * 16))[ch];
}

template <int KS>
__device__ __forceinline__ TileRegs wt_load(const uint16_t* __restrict__ Wb, const float* __restrict__ bias, int n0,
                                            int tid) {
  static_assert(WTile<KS>::PER <= 2, "at most two chunks per thread");
  TileRegs T;
  T.c0 = wt_chunk<KS>(Wb, n0, tid);
  T.c1 = WTile<KS>::PER > 1 ? wt_chunk<KS>(Wb, n0, tid + ML_THREADS) : T.c0;
  T.b = bias[n0 + (tid & 31)];
  return T;
}

// LDS fragment layout of one weight tile, in 16-byte units: k-chunk kk,
// half hh (k-values 16 kk + 8 hh .. + 7), row r at kk * WF_KK + hh * WF_HALF
// + r.  The MFMA read (lane l: half l / 32, row l % 32) is contiguous for
// every 16 lanes; the padding (33 and 66 instead of 32 and 64) spreads the
// stores, where the 32 chunks of one row go to 16 KS different (kk, hh), over
// all banks: (2 kk + hh + r) mod 16 differs for the 16 lanes of a store
// cycle.
constexpr int WF_HALF = 33, WF_KK = 2 * WF_HALF;

// registers -> LDS in fragment order
// (free of branches, so that a step of the tile stream stays one block, when
// every thread has its chunks - KS = 8, 16 - or when the buffer, of CAP
// chunks, has room past the tile for the surplus threads' copies; every
// thread writes its bias, the 16 threads of a row the same value)
template <int KS, int CAP = KS * WF_KK>
__device__ __forceinline__ void wt_store(const TileRegs& T, uint4* frag, float* bs, int tid) {
  constexpr int NCH = WTile<KS>::NCH;
  auto slot = [&](int cidx) {
    const int row = cidx / WTile<KS>::CH, ch = cidx - row * WTile<KS>::CH;
    return (ch >> 1) * WF_KK + (ch & 1) * WF_HALF + row;
  };
  auto put = [&](int cidx, const uint4& c) { frag[slot(cidx)] = c; };
  if constexpr (ML_THREADS <= NCH) {
    put(tid, T.c0);
  } else if constexpr (KS * WF_KK + ML_THREADS - NCH <= CAP) {
    // threads NCH.. write into the unused tail KS WF_KK .. of the buffer
    frag[tid < NCH ? slot(tid) : KS * WF_KK + (tid - NCH)] = T.c0;
  } else if (tid < NCH) {
    put(tid, T.c0);
  }
  if constexpr (WTile<KS>::PER > 1) {
    if constexpr (2 * ML_THREADS <= NCH) put(tid + ML_THREADS, T.c1);
    else if (tid + ML_THREADS < NCH) put(tid + ML_THREADS, T.c1);
  }
  bs[tid & 31] = T.b;
}

// acc = bias (of the lane's 16 rows) + sum_kk A[kk] B[kk]; the A fragments
// are read from LDS four k-chunks ahead of their matrix product
template <int KS>
__device__ __forceinline__ floatx16 tile_mfma(const uint4* frag, const float* bs, const bf16x8 (&B)[KS], int lane) {
  constexpr int AH = KS < 4 ? KS : 4;
  const uint4* fp = frag + (lane >> 5) * WF_HALF + (lane & 31);
  uint4 a[AH];
#pragma unroll
  for (int j = 0; j < AH; ++j) a[j] = fp[j * WF_KK];
  floatx16 acc;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 b4 = *reinterpret_cast<const float4*>(&bs[8 * g + 4 * (lane >> 5)]);
    acc[4 * g + 0] = b4.x;
    acc[4 * g + 1] = b4.y;
    acc[4 * g + 2] = b4.z;
    acc[4 * g + 3] = b4.w;
  }
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(&a[kk % AH]), B[kk], acc, 0, 0, 0);
    if (kk + AH < KS) a[kk % AH] = fp[(kk + AH) * WF_KK];
  }
  // keep that order (the scheduler would otherwise pull the reads next to
  // their products): the AH + 4 first LDS reads (fragments, bias), then one
  // product and one read at a time
  __builtin_amdgcn_sched_group_barrier(0x100, AH + 4, 0);
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    if (kk + AH < KS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  return acc;
}

// the order of tile_mfma_epi: one product, one LDS read, the vector work of
// the slots that follow product kk (vector and transcendental instructions)
template <int KS, int AH, int VPS, int NS, int kk>
__device__ __forceinline__ void epi_order_step() {
  constexpr int ns = (NS * (kk + 1)) / KS - (NS * kk) / KS;
  __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
  if constexpr (kk + AH < KS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  if constexpr (ns > 0) __builtin_amdgcn_sched_group_barrier(0x402, VPS * ns, 0);
}
template <int KS, int AH, int VPS, int NS, int... KK>
__device__ __forceinline__ void epi_order(std::integer_sequence<int, KK...>) {
  (epi_order_step<KS, AH, VPS, NS, KK>(), ...);
}

// tile_mfma with a per-slot epilogue of the previous tile woven in: after
// product kk, slots (NS kk / KS) .. (NS (kk + 1) / KS) - 1 of the previous
// tile's epilogue, about VPS vector instructions each.  A lone wave issues
// dependent vector work at about half the SIMD's rate, so the epilogue of a
// wave is cheapest when the other wave of the SIMD is doing the same work at
// the same time, its own matrix products running underneath.
template <int KS, int VPS, int NS = 16, class SlotFn>
__device__ __forceinline__ floatx16 tile_mfma_epi(const uint4* frag, const float* bs, const bf16x8 (&B)[KS], int lane,
                                                  SlotFn&& slot) {
  constexpr int AH = KS < 4 ? KS : 4;
  const uint4* fp = frag + (lane >> 5) * WF_HALF + (lane & 31);
  uint4 a[AH];
#pragma unroll
  for (int j = 0; j < AH; ++j) a[j] = fp[j * WF_KK];
  floatx16 acc;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 b4 = *reinterpret_cast<const float4*>(&bs[8 * g + 4 * (lane >> 5)]);
    acc[4 * g + 0] = b4.x;
    acc[4 * g + 1] = b4.y;
    acc[4 * g + 2] = b4.z;
    acc[4 * g + 3] = b4.w;
  }
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(&a[kk % AH]), B[kk], acc, 0, 0, 0);
    if (kk + AH < KS) a[kk % AH] = fp[(kk + AH) * WF_KK];
#pragma unroll
    for (int r = (NS * kk) / KS; r < (NS * (kk + 1)) / KS; ++r) slot(r);
  }
  __builtin_amdgcn_sched_group_barrier(0x100, AH + 4, 0);
  epi_order<KS, AH, VPS, NS>(std::make_integer_sequence<int, KS>{});
  return acc;
}

// stream_tiles for an epilogue made of 16 independent per-slot updates
// (slot(acc, t, r) for register r of tile t, free of branches): every wave
// runs the same schedule, and the steady-state step - loads of tile t + 2,
// the products of tile t woven with the epilogue of tile t - 1, the store of
// tile t + 1, barrier - is one straight block.  The first tile's products
// and the last tile's epilogue are peeled.  Past the end the loads re-read
// the last tile and the store writes it into the buffer no one reads again.
// first(acc) sees the first tile's accumulator before any slot update.
template <int KS, int VPS, class Slot, class First>
__device__ __forceinline__ void stream_tiles_slots(uint4 (*frag)[KS * WF_KK], float (*bs)[32],
                                                   const uint16_t* __restrict__ Wb, const float* __restrict__ bias,
                                                   int ntiles, const bf16x8 (&B)[KS], int tid, int lane, Slot&& slot,
                                                   First&& first) {
  const int last = ntiles - 1;
  TileRegs T0 = wt_load<KS>(Wb, bias, 0, tid);
  TileRegs T1 = wt_load<KS>(Wb, bias, min(1, last) * 32, tid);
  lds_barrier();  // earlier readers of the buffers are done
  wt_store<KS>(T0, frag[0], bs[0], tid);
  lds_barrier();
  floatx16 acc[2];
  T0 = wt_load<KS>(Wb, bias, min(2, last) * 32, tid);
  acc[0] = tile_mfma<KS>(frag[0], bs[0], B, lane);
  first(acc[0]);
  wt_store<KS>(T1, frag[1], bs[1], tid);
  lds_barrier();
  auto step = [&](auto U, int tt) {
    constexpr int u = decltype(U)::value;
    const int tn = min(tt + 2, last) * 32;
    if constexpr (u == 0) T0 = wt_load<KS>(Wb, bias, tn, tid);
    else T1 = wt_load<KS>(Wb, bias, tn, tid);
    const floatx16& prev = acc[u ^ 1];
    acc[u] = tile_mfma_epi<KS, VPS>(frag[u], bs[u], B, lane, [&](int r) { slot(prev, tt - 1, r); });
    if constexpr (u == 0) wt_store<KS>(T1, frag[1], bs[1], tid);
    else wt_store<KS>(T0, frag[0], bs[0], tid);
    lds_barrier();
    __builtin_amdgcn_sched_barrier(0);  // each step is scheduled on its own
  };
  int t = 1;
  for (; t + 1 <= last; t += 2) {
    step(std::integral_constant<int, 1>(), t);
    step(std::integral_constant<int, 0>(), t + 1);
  }
  if (t <= last) step(std::integral_constant<int, 1>(), t);
  if (last & 1) {
#pragma unroll
    for (int r = 0; r < 16; ++r) slot(acc[1], last, r);
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) slot(acc[0], last, r);
  }
}
template <int KS, int VPS, class Slot>
__device__ __forceinline__ void stream_tiles_slots(uint4 (*frag)[KS * WF_KK], float (*bs)[32],
                                                   const uint16_t* __restrict__ Wb, const float* __restrict__ bias,
                                                   int ntiles, const bf16x8 (&B)[KS], int tid, int lane, Slot&& slot) {
  stream_tiles_slots<KS, VPS>(frag, bs, Wb, bias, ntiles, B, tid, lane, slot, [](const floatx16&) {});
}

__device__ __forceinline__ bf16x8 gelu_bf16x8(const floatx16& acc, int c) {
  bf16x8 o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = (__bf16)gelu_poly_f(acc[8 * c + j]);
  return o;
}

// Both hidden layers: H2 = GELU(GELU(bf16(Qp * scale) W1^T + b1) W2p^T + b2)
// of query q, left in registers in the lanes' order (see above): H2[kk] is
// this lane's B operand of k-chunk kk of the next layer.  W1b [16 KSH][16
// KS1] (natural order, zero-padded inputs), W2b [16 KSH][16 KSH] (columns
// permuted).  frag / bs: the block's two LDS tile buffers (KSM >= KS1, KSH).
template <int KS1, int KSH, int KSM>
__device__ __forceinline__ void hidden_layers(const float* __restrict__ Qp, int ld, int64_t q, bool qok,
                                              const float* __restrict__ scale, int n_in,
                                              const uint16_t* __restrict__ W1b, const float* __restrict__ b1,
                                              const uint16_t* __restrict__ W2b, const float* __restrict__ b2,
                                              uint4 (*frag)[KSM * WF_KK], float (*bs)[32], int tid, int lane,
                                              bf16x8 (&H2)[KSH]) {
  static_assert(KSM >= KS1 && KSM >= KSH, "tile buffers too small");
  constexpr int NT = KSH / 2;  // tiles of 32 hidden units per layer
  const int h = lane >> 5;
  // every load unconditional, so that they are all in flight at once: inputs
  // past n_in repeat the last one and meet the zero columns of W1b; a query
  // past the end reads row 0 and its results are never written
  bf16x8 X[KS1];
  const float* qrow = Qp + (qok ? q : 0) * (int64_t)ld;
#pragma unroll
  for (int kk = 0; kk < KS1; ++kk) {
    const int k0 = 16 * kk + 8 * h;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kc = min(k0 + j, n_in - 1);
      X[kk][j] = (__bf16)(qrow[kc] * scale[kc]);
    }
  }
  bf16x8 H1[KSH];
  TileRegs T0, T1;
  // Software pipelined over the 2 NT tiles (NT of each layer), loads two
  // tiles ahead: step t issues the loads of tile t + 2, the matrix products
  // of tile t woven with the epilogue (bias is in the accumulator; GELU,
  // bf16) of tile t - 1, and stores tile t + 1 into LDS.  The first layer-2
  // tile needs every layer-1 activation, so there the epilogue goes first.
  auto epilogue = [&](const floatx16& acc, int t) {
    if (t < NT) {
      H1[2 * t] = gelu_bf16x8(acc, 0);
      H1[2 * t + 1] = gelu_bf16x8(acc, 1);
    } else {
      H2[2 * (t - NT)] = gelu_bf16x8(acc, 0);
      H2[2 * (t - NT) + 1] = gelu_bf16x8(acc, 1);
    }
  };
  // values 2 p, 2 p + 1 of tile t (one packed bf16 pair), p = 0 .. 7
  auto epilogue_pair = [&](const floatx16& acc, int t, int p) {
    bf16x8& o = t < NT ? H1[2 * t + (p >> 2)] : H2[2 * (t - NT) + (p >> 2)];
    o[2 * (p & 3)] = (__bf16)gelu_poly_f(acc[2 * p]);
    o[2 * (p & 3) + 1] = (__bf16)gelu_poly_f(acc[2 * p + 1]);
  };
  // tile k of the stream: layer-1 tile k (k < NT) or layer-2 tile k - NT
  // tile k of the stream goes through register set k % 2 (t is compile-time below)
  auto fetch = [&](int k) {
    return k < NT ? wt_load<KS1>(W1b, b1, k * 32, tid) : wt_load<KSH>(W2b, b2, (k - NT) * 32, tid);
  };
  auto load = [&](int k) {
    if (k & 1) T1 = fetch(k);
    else T0 = fetch(k);
  };
  auto store = [&](int k) {
    const TileRegs T = (k & 1) ? T1 : T0;
    if (k < NT) wt_store<KS1, KSM * WF_KK>(T, frag[k & 1], bs[k & 1], tid);
    else wt_store<KSH, KSM * WF_KK>(T, frag[k & 1], bs[k & 1], tid);
  };
  load(0);
  load(1);
  store(0);
  lds_barrier();
  floatx16 acc_prev = {};
#pragma unroll
  for (int t = 0; t <= 2 * NT; ++t) {
    if (t + 2 < 2 * NT) load(t + 2);
    floatx16 acc_cur = {};
    auto pair = [&](int p) { epilogue_pair(acc_prev, t - 1, p); };
    if (t == 0) {
      acc_cur = tile_mfma<KS1>(frag[0], bs[0], X, lane);
    } else if (t < NT) {
      acc_cur = tile_mfma_epi<KS1, 25, 8>(frag[t & 1], bs[t & 1], X, lane, pair);
    } else if (t == NT) {
      epilogue(acc_prev, t - 1);
      acc_cur = tile_mfma<KSH>(frag[t & 1], bs[t & 1], H1, lane);
    } else if (t < 2 * NT) {
      acc_cur = tile_mfma_epi<KSH, 25, 8>(frag[t & 1], bs[t & 1], H1, lane, pair);
    } else {
      epilogue(acc_prev, t - 1);
    }
    if (t + 1 < 2 * NT) store(t + 1);
    lds_barrier();
    __builtin_amdgcn_sched_barrier(0);  // each step is scheduled on its own
    acc_prev = acc_cur;
  }
}

// descending by value, ties to the lower id
__device__ __forceinline__ bool desc_lt(float a, int ia, float b, int ib) { return a > b || (a == b && ia < ib); }

template <int P>
struct TopP {
  float v[P];
  int i[P];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      v[t] = -FLT_MAX;
      i[t] = INT_MAX;
    }
  }
  __device__ __forceinline__ void insert(float x, int id) {
    bool b[P];
#pragma unroll
    for (int t = 0; t < P; ++t) b[t] = desc_lt(x, id, v[t], i[t]);
#pragma unroll
    for (int t = P - 1; t > 0; --t) {
      v[t] = b[t - 1] ? v[t - 1] : (b[t] ? x : v[t]);
      i[t] = b[t - 1] ? i[t - 1] : (b[t] ? id : i[t]);
    }
    v[0] = b[0] ? x : v[0];
    i[0] = b[0] ? id : i[0];
  }
};

// Software-pipelined stream of the ntiles 32-row tiles of W through the LDS
// double buffer.  Step t issues the global loads of tile t + 2 (into one of
// two register sets), the matrix products of tile t, the epilogue epi(acc,
// t - 1) of the previous tile, and stores tile t + 1 (loaded one step
// earlier) into the buffer tile t - 1 used; the barrier between steps does
// not wait for the loads in flight, so every load has two steps to arrive.
// Two steps per trip keep the register sets and accumulators static.
template <int KS, class Epi>
__device__ __forceinline__ void stream_tiles(uint4 (*frag)[KS * WF_KK], float (*bs)[32], const uint16_t* __restrict__ Wb,
                                             const float* __restrict__ bias, int ntiles, const bf16x8 (&B)[KS],
                                             int tid, int lane, Epi&& epi) {
  TileRegs T0 = wt_load<KS>(Wb, bias, 0, tid), T1 = T0;
  if (ntiles > 1) T1 = wt_load<KS>(Wb, bias, 32, tid);
  lds_barrier();  // earlier readers of the buffers are done
  wt_store<KS>(T0, frag[0], bs[0], tid);
  lds_barrier();
  floatx16 acc[2] = {{}, {}};
  const bool epi_first = (tid >> 8) & 1;
  // one step on tile tt with register set / buffer / accumulator U (= tt % 2)
  auto step = [&](auto U, int tt) {
    constexpr int u = decltype(U)::value;
    // issued unconditionally (past the end: the last tile again, never
    // stored), so the compiler's count of loads in flight is the same on
    // every path and the store below waits only for the older tile
    const int tn = min(tt + 2, ntiles - 1) * 32;
    if constexpr (u == 0) T0 = wt_load<KS>(Wb, bias, tn, tid);
    else T1 = wt_load<KS>(Wb, bias, tn, tid);
    // the second wave of each SIMD (waves 4..7) runs the epilogue first, so
    // that one wave's vector work overlaps the other's matrix products
    if (epi_first && tt >= 1) epi(acc[u ^ 1], tt - 1);
    if (tt < ntiles) acc[u] = tile_mfma<KS>(frag[u], bs[u], B, lane);
    if (!epi_first && tt >= 1) epi(acc[u ^ 1], tt - 1);
    if (tt + 1 < ntiles) {
      if constexpr (u == 0) wt_store<KS>(T1, frag[1], bs[1], tid);
      else wt_store<KS>(T0, frag[0], bs[0], tid);
    }
    lds_barrier();
  };
  for (int t = 0; t <= ntiles; t += 2) {
    step(std::integral_constant<int, 0>(), t);
    if (t + 1 <= ntiles) step(std::integral_constant<int, 1>(), t + 1);
  }
}

template <int PP>
__device__ __forceinline__ void topp_finish(const TopP<PP>& top, float s, int lane, int64_t q, int64_t nq, int kout,
                                            bool write, int32_t* __restrict__ leaves, float* __restrict__ margin);

// Output layer, exact top-P leaves and the softmax margin p1 - p2, in two
// passes over the weight tiles (the logits are never stored).
//  Pass 1: per value slot (lane, register) the largest and second-largest
//    logit and the tile of the largest (4 operations per logit).  Then per
//    query: m = the largest logit and tau = the P-th largest of the 64 slot
//    values, which are 64 distinct logits, so tau <= the P-th largest logit:
//    every top-P logit is >= tau, and usually only those are.
//  Pass 2: recompute the logits; append each logit >= tau (with its leaf) to
//    a per-lane list in LDS (into the in-register top-P should the list be
//    full) - only for slots whose second-largest logit is >= tau, the others
//    holding at most their maximum, appended before the pass - and
//    accumulate sum exp(l - m).
//  Finally each lane ranks its list, and the two lanes of each query merge
//  their top-P lists.
template <int KS, int PP>
__device__ __forceinline__ void out_topk(const bf16x8 (&B)[KS], int64_t q, int64_t nq,
                                         const uint16_t* __restrict__ Wb, const float* __restrict__ bias, int N,
                                         int kout, uint4 (*frag)[KS * WF_KK], float (*bs)[32],
                                         float (*hv)[ML_THREADS], int (*hid)[ML_THREADS], int tid, int lane,
                                         int32_t* __restrict__ leaves, float* __restrict__ margin) {
  constexpr int HC = 8;  // hit-list capacity per lane
  const int h = lane >> 5;
  const int ntiles = (N + 31) / 32;
  // pass 1
  float m1[16], m2[16];
  int i1[16];  // tile of m1 (the first one on ties)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    m1[r] = -FLT_MAX;
    m2[r] = -FLT_MAX;
    i1[r] = 0;
  }
  stream_tiles_slots<KS, 4>(frag, bs, Wb, bias, ntiles, B, tid, lane, [&](const floatx16& acc, int t, int r) {
    // with m2 <= m1, max(m2, min(m1, x)) is the median of the three; a
    // compare-select for the maximum (fmaxf would first quieten its
    // operands, one more instruction each)
    const bool gt = acc[r] > m1[r];
    m2[r] = __builtin_amdgcn_fmed3f(acc[r], m1[r], m2[r]);
    m1[r] = gt ? acc[r] : m1[r];
    i1[r] = gt ? t : i1[r];
  });
  // tau and m: the P-th largest and the largest of the query's 64 slot values
  // (values only: a max/min exchange network keeps v sorted descending)
  float tau, mxl2;
  {
    // (max / min as medians with an infinity: fmaxf / fminf would first
    // quieten their operands)
    float v[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) v[u] = -FLT_MAX;
    auto push = [&](float x) {
#pragma unroll
      for (int u = 0; u < PP; ++u) {
        const float hi = __builtin_amdgcn_fmed3f(v[u], x, INFINITY);
        x = __builtin_amdgcn_fmed3f(v[u], x, -INFINITY);
        v[u] = hi;
      }
    };
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      push(m1[r]);
      push(m2[r]);
    }
    float ov[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) ov[u] = __shfl_xor(v[u], 32, 64);
#pragma unroll
    for (int u = 0; u < PP; ++u) push(ov[u]);
    float tk = v[0];
#pragma unroll
    for (int u = 1; u < PP; ++u)
      if (u < kout) tk = v[u];
    tau = tk;
    mxl2 = v[0] * ML_LOG2E;
  }
  // A slot whose second-largest logit is below tau holds at most one logit
  // >= tau, its maximum, known with its tile from pass 1: appended here.
  // Only slots with m2 >= tau (several top logits in one slot, or ties) are
  // searched again in pass 2, and a slot index r that no lane of the wave
  // needs is skipped there by a wave-uniform branch.
  int cnt = 0;
  bool ovf = false;
  uint32_t need = 0, flagged = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const bool flag = m2[r] >= tau;
    if (__ballot(flag)) need |= 1u << r;
    flagged |= (flag ? 1u : 0u) << r;
    const bool direct = !flag && m1[r] >= tau;
    const bool app = direct && cnt < HC;
    ovf = ovf || (direct && !app);
    if (app) {
      hv[cnt][tid] = m1[r];
      hid[cnt][tid] = i1[r] * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      ++cnt;
    }
  }
  need = __builtin_amdgcn_readfirstlane(need);
  // pass 2: hits of the flagged slots into the per-lane LDS list, softmax
  // normaliser
  float ssum = 0.f;
  stream_tiles<KS>(frag, bs, Wb, bias, ntiles, B, tid, lane, [&](const floatx16& acc, int t) {
    float e[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) e[r] = __builtin_amdgcn_exp2f(fmaf(acc[r], ML_LOG2E, -mxl2));
#pragma unroll
    for (int r = 0; r < 16; r += 2) ssum += e[r] + e[r + 1];
    // the slot indices some lane needs, one at a time (a wave-uniform index
    // into the accumulator)
    for (uint32_t m = need; m != 0; m &= m - 1) {
      const int r = __builtin_ctz(m);
      const float v = acc[r];
      const bool hit = v >= tau && ((flagged >> r) & 1u);
      const bool app = hit && cnt < HC;
      ovf = ovf || (hit && !app);
      if (app) {
        hv[cnt][tid] = v;
        hid[cnt][tid] = t * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        ++cnt;
      }
    }
  });
  TopP<PP> top;
  top.init();
  // a full list (ties or many logits >= tau; not seen in practice): one more
  // pass in which the lanes concerned insert every hit into the top-P
  if (__syncthreads_or(ovf ? 1 : 0)) {
    stream_tiles<KS>(frag, bs, Wb, bias, ntiles, B, tid, lane, [&](const floatx16& acc, int t) {
      if (ovf) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (acc[r] >= tau) top.insert(acc[r], t * 32 + 8 * (r >> 2) + 4 * h + (r & 3));
      }
    });
  }
  if (!ovf)
    for (int c = 0; c < cnt; ++c) top.insert(hv[c][tid], hid[c][tid]);
  const float s = ssum + __shfl_xor(ssum, 32, 64);  // both halves use the same m
  topp_finish<PP>(top, s, lane, q, nq, kout, true, leaves, margin);
}

// The two lanes of query q merge their top-P lists; lane h = 0 writes the
// kout leaves and the margin p1 - p2 = (1 - exp(l2 - l1)) / s, with s =
// sum_j exp(l_j - l1) over all leaves (l1 the largest logit), if `write`.
template <int PP>
__device__ __forceinline__ void topp_finish(const TopP<PP>& top, float s, int lane, int64_t q, int64_t nq, int kout,
                                            bool write, int32_t* __restrict__ leaves, float* __restrict__ margin) {
  float ov[PP];
  int oi[PP];
#pragma unroll
  for (int t = 0; t < PP; ++t) {
    ov[t] = __shfl_xor(top.v[t], 32, 64);
    oi[t] = __shfl_xor(top.i[t], 32, 64);
  }
  if (write && lane < 32 && q < nq) {
    int a = 0, b = 0;
    float best[2] = {-FLT_MAX, -FLT_MAX};
#pragma unroll
    for (int t = 0; t < PP; ++t) {  // merge two descending lists
      float va = -FLT_MAX, vb = -FLT_MAX;
      int ia = INT_MAX, ib = INT_MAX;
#pragma unroll
      for (int u = 0; u < PP; ++u) {
        if (u == a) {
          va = top.v[u];
          ia = top.i[u];
        }
        if (u == b) {
          vb = ov[u];
          ib = oi[u];
        }
      }
      const bool take_a = desc_lt(va, ia, vb, ib);
      const int id = take_a ? ia : ib;
      const float vv = take_a ? va : vb;
      if (take_a) ++a;
      else ++b;
      if (t < kout) leaves[q * kout + t] = (id == INT_MAX) ? -1 : id;
      if (t < 2) best[t] = vv;
    }
    // p1 - p2 = (1 - exp(l2 - l1)) / sum_j exp(l_j - l1), l1 = m
    margin[q] = (best[1] == -FLT_MAX) ? 1.0f : (1.0f - exp2f((best[1] - best[0]) * ML_LOG2E)) / s;
  }
}

// Output layer in one pass over the weight tiles.  Per value slot (lane,
// register) the three largest logit keys - the logit with its low tb
// mantissa bits replaced by (2^tb - 1 - t), t the tile, so that a key names
// its leaf and, among equal logits, the lower tile ranks first - kept by
// medians (k1 >= k2 >= k3), and sum_j exp(l_j - R) over the slot, R the
// query's largest logit of the first tile: one fused multiply-add, one
// exponential, one add and four key operations per logit.  Then tau = the
// P-th largest of the query's 64 values k1, k2 (a lower bound of the P-th
// largest key, as in the two-pass form); a slot whose k3 is below tau holds
// no key >= tau beyond k1 and k2, so the top-P is exact unless some slot has
// k3 >= tau (three or more top logits in one slot, or ties), a hit list is
// full, or some logit exceeds R by so much that the sum may have lost
// precision.  Returns that case - the caller hands the query to the
// two-pass form - and writes nothing for it; otherwise writes the top-P and
// the margin (from keys: logits to 2^(tb - 23) relative).
template <int KS, int PP>
__device__ __forceinline__ bool out_topk_1pass(const bf16x8 (&B)[KS], int64_t q, int64_t nq,
                                               const uint16_t* __restrict__ Wb, const float* __restrict__ bias,
                                               int N, int kout, uint4 (*frag)[KS * WF_KK], float (*bs)[32],
                                               float (*hv)[ML_THREADS], int (*hid)[ML_THREADS], int tid, int lane,
                                               int32_t* __restrict__ leaves, float* __restrict__ margin) {
  constexpr int HC = 8;  // hit-list capacity per lane
  const int h = lane >> 5;
  const int ntiles = (N + 31) / 32;
  int tb = 1;
  while ((1 << tb) < ntiles) ++tb;
  const uint32_t lmask = (1u << tb) - 1u, kmask = ~lmask;
  float k1[16], k2[16], k3[16], sm[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    k1[r] = -INFINITY;
    k2[r] = -INFINITY;
    k3[r] = -INFINITY;
    sm[r] = 0.f;
  }
  float rl2 = 0.f;  // R log2(e)
  stream_tiles_slots<KS, 7>(
      frag, bs, Wb, bias, ntiles, B, tid, lane,
      [&](const floatx16& acc, int t, int r) {
        const float x = acc[r];
        sm[r] += __builtin_amdgcn_exp2f(fmaf(x, ML_LOG2E, -rl2));
        const float k = __uint_as_float((__float_as_uint(x) & kmask) | (lmask - (uint32_t)t));
        // with k3 <= k2 <= k1: the three largest of (k1, k2, k3, k)
        k3[r] = __builtin_amdgcn_fmed3f(k, k2[r], k3[r]);
        k2[r] = __builtin_amdgcn_fmed3f(k, k1[r], k2[r]);
        k1[r] = __builtin_amdgcn_fmed3f(k1[r], k, INFINITY);
      },
      [&](const floatx16& acc0) {
        float m = acc0[0];
#pragma unroll
        for (int r = 1; r < 16; ++r) m = __builtin_amdgcn_fmed3f(m, acc0[r], INFINITY);
        m = __builtin_amdgcn_fmed3f(m, __shfl_xor(m, 32, 64), INFINITY);
        rl2 = m * ML_LOG2E;
      });
  // the largest key M (the largest logit) and s = sum_j exp(l_j - M) over both halves
  float mx = k1[0];
#pragma unroll
  for (int r = 1; r < 16; ++r) mx = __builtin_amdgcn_fmed3f(mx, k1[r], INFINITY);
  mx = __builtin_amdgcn_fmed3f(mx, __shfl_xor(mx, 32, 64), INFINITY);
  float ssum = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) ssum += sm[r];
  ssum += __shfl_xor(ssum, 32, 64);
  // beyond 2^64 the sum's terms relative to R have grown too far
  bool fallback = !(mx * ML_LOG2E - rl2 <= 64.f);
  ssum *= __builtin_amdgcn_exp2f(rl2 - mx * ML_LOG2E);
  // tau: the P-th largest of the query's 64 slot values k1, k2
  float tau;
  {
    // (max / min as medians with an infinity: fmaxf / fminf would first
    // quieten their operands)
    float v[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) v[u] = -INFINITY;
    auto push = [&](float x) {
#pragma unroll
      for (int u = 0; u < PP; ++u) {
        const float hi = __builtin_amdgcn_fmed3f(v[u], x, INFINITY);
        x = __builtin_amdgcn_fmed3f(v[u], x, -INFINITY);
        v[u] = hi;
      }
    };
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      push(k1[r]);
      push(k2[r]);
    }
    float ov[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) ov[u] = __shfl_xor(v[u], 32, 64);
#pragma unroll
    for (int u = 0; u < PP; ++u) push(ov[u]);
    float tk = v[0];
#pragma unroll
    for (int u = 1; u < PP; ++u)
      if (u < kout) tk = v[u];
    tau = tk;
  }
  // the hits k1, k2 >= tau with their leaves; a slot with k3 >= tau (or a
  // full list) leaves the query to the two-pass form
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int off = 8 * (r >> 2) + 4 * h + (r & 3);
    fallback = fallback || (k3[r] >= tau);
    const float kv[2] = {k1[r], k2[r]};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (kv[u] >= tau) {
        if (cnt < HC) {
          hv[cnt][tid] = kv[u];
          hid[cnt][tid] = (int)(lmask - (__float_as_uint(kv[u]) & lmask)) * 32 + off;
          ++cnt;
        } else {
          fallback = true;
        }
      }
    }
  }
  fallback = __shfl_xor(fallback ? 1 : 0, 32, 64) != 0 || fallback;
  TopP<PP> top;
  top.init();
  for (int c = 0; c < cnt; ++c) top.insert(hv[c][tid], hid[c][tid]);
  topp_finish<PP>(top, ssum, lane, q, nq, kout, !fallback, leaves, margin);
  return fallback;
}

// The whole proposal network for 256 queries per block: both hidden layers,
// then the output layer's exact top-P and margin, the hidden activations
// never leaving the registers.  The two phases share the LDS tile buffers.
// ONE: the one-pass output layer; queries it cannot settle exactly are
// appended to (list, n_list).  Otherwise the two-pass form, over the queries
// of (list, n_list) when list is given, else over 0 .. nq - 1.
template <int KS1, int KSH, int PP, bool ONE>
__global__ __launch_bounds__(ML_THREADS) void k_mlp_propose(const float* __restrict__ Qp, int ld, int64_t nq,
                                                            const float* __restrict__ scale, int n_in,
                                                            const uint16_t* __restrict__ W1b,
                                                            const float* __restrict__ b1,
                                                            const uint16_t* __restrict__ W2b,
                                                            const float* __restrict__ b2,
                                                            const uint16_t* __restrict__ W3b,
                                                            const float* __restrict__ b3, int N, int kout,
                                                            int32_t* __restrict__ list, int32_t* __restrict__ n_list,
                                                            int32_t* __restrict__ leaves,
                                                            float* __restrict__ margin) {
  constexpr int KSM = KS1 > KSH ? KS1 : KSH;
  __shared__ uint4 frag[2][KSM * WF_KK];
  __shared__ float bs[2][32];
  __shared__ float hv[8][ML_THREADS];
  __shared__ int hid[8][ML_THREADS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t idx = (int64_t)blockIdx.x * ML_QPB + wave * 32 + (lane & 31);
  int64_t q = idx;
  if (!ONE && list) {
    const int64_t n = *n_list;
    if ((int64_t)blockIdx.x * ML_QPB >= n) return;  // uniform per block
    q = idx < n ? list[idx] : nq;
  }
  bf16x8 H2[KSH];
  hidden_layers<KS1, KSH, KSM>(Qp, ld, q, q < nq, scale, n_in, W1b, b1, W2b, b2, frag, bs, tid, lane, H2);
  // the output layer streams KSH-wide tiles through the first part of each buffer
  auto fo = reinterpret_cast<uint4(*)[KSH * WF_KK]>(&frag[0][0]);
  if constexpr (ONE) {
    const bool fb = out_topk_1pass<KSH, PP>(H2, q, nq, W3b, b3, N, kout, fo, bs, hv, hid, tid, lane, leaves, margin);
    if (fb && lane < 32 && q < nq) list[atomicAdd(n_list, 1)] = (int32_t)q;
  } else {
    out_topk<KSH, PP>(H2, q, nq, W3b, b3, N, kout, fo, bs, hv, hid, tid, lane, leaves, margin);
  }
}

#define PTS_MLP_KIN_SWITCH(K, ...)                                                                 \
  switch (K) {                                                                                     \
    case 32: { constexpr int KS1C = 2; __VA_ARGS__; } break;                                       \
    case 64: { constexpr int KS1C = 4; __VA_ARGS__; } break;                                       \
    case 96: { constexpr int KS1C = 6; __VA_ARGS__; } break;                                       \
    case 128: { constexpr int KS1C = 8; __VA_ARGS__; } break;                                      \
    default: ::pts::fail(PTS_ERR_UNSUPPORTED, "MLP input width must be 32/64/96/128");             \
  }
#define PTS_MLP_HID_SWITCH(H, ...)                                                                 \
  switch (H) {                                                                                     \
    case 32: { constexpr int KSC = 2; __VA_ARGS__; } break;                                        \
    case 64: { constexpr int KSC = 4; __VA_ARGS__; } break;                                        \
    case 128: { constexpr int KSC = 8; __VA_ARGS__; } break;                                       \
    case 256: { constexpr int KSC = 16; __VA_ARGS__; } break;                                      \
    default: ::pts::fail(PTS_ERR_UNSUPPORTED, "MLP hidden width must be 32/64/128/256");           \
  }

void launch_mlp_propose(Ctx* c, const float* Qp, int ld, int64_t nq, const float* scale, int n_in, int K1,
                        const uint16_t* W1b, const float* b1, const uint16_t* W2b, const float* b2, int hidden,
                        const uint16_t* W3b, const float* b3, int N, int k, int32_t* leaves, float* margin) {
  ProfScope ps(c, "mlp_propose_mfma");
  if (nq == 0) return;
  PTS_REQUIRE(n_in >= 1 && n_in <= K1 && n_in <= ld, PTS_ERR_ARG, "mlp_propose: bad input width");
  PTS_REQUIRE(k >= 1 && k <= ML_P && k <= N, PTS_ERR_ARG, "proposals must be 1..8 and at most n_out");
  PTS_REQUIRE(nq < INT_MAX, PTS_ERR_UNSUPPORTED, "mlp_propose: too many queries");
  // the one-pass output layer keeps two tile indices (N / 32 of them) in 16 bits each
  PTS_REQUIRE(N >= 1 && N <= 65536, PTS_ERR_UNSUPPORTED, "mlp_propose: at most 65536 outputs");
  // one pass for every query, then the two-pass form for those it could not settle
  int32_t* list = c->buf<int32_t>("mlp_fix_list", (size_t)nq);
  int32_t* n_list = c->buf<int32_t>("mlp_fix_n", 1);
  launch_zero_i32(c, n_list, 1);
  const dim3 grid((unsigned)ceil_div(nq, ML_QPB));
#define PTS_MLP_PROPOSE(PPV, ONEV)                                                                                   \
  PTS_MLP_KIN_SWITCH(K1, PTS_MLP_HID_SWITCH(hidden, hipLaunchKernelGGL((k_mlp_propose<KS1C, KSC, PPV, ONEV>), grid,   \
                                                                       dim3(ML_THREADS), 0, c->stream, Qp, ld, nq,    \
                                                                       scale, n_in, W1b, b1, W2b, b2, W3b, b3, N, k,  \
                                                                       list, n_list, leaves, margin)))
  if (k <= 4) {
    PTS_MLP_PROPOSE(4, true);
    PTS_MLP_PROPOSE(4, false);
  } else {
    PTS_MLP_PROPOSE(8, true);
    PTS_MLP_PROPOSE(8, false);
  }
#undef PTS_MLP_PROPOSE
  check_launch("k_mlp_propose");
}

}  // namespace pts
