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
// lane owns one query and 16 output features; weight tiles stream through
// LDS shared by the block's 4 waves (256 queries).  Hidden layers write
// GELU(acc + b) as bf16; the output layer never writes logits: the bias
// initialises the accumulator and each lane folds its 16 values into a
// running top-P (descending, ties to the lower leaf) and an online softmax
// normaliser, merged with the lane sharing its query at the end.
#include <cfloat>
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

// Inference GELU: Phi(x) = 1/2 + x P(t), t = 2 x^2 / c^2 - 1, |x| clamped to
// c = 4.5, P a degree-10 near-minimax fit (coefficients from fit_phi_poly.py
// beside this package); |error| <= 3e-6 in Phi, far below the bf16 rounding
// of the activations.  15 VALU operations against ~40 for erff.
__device__ __forceinline__ float gelu_poly_f(float x) {
  constexpr float c = 4.5f, a = 2.0f / (4.5f * 4.5f);
  const float xc = __builtin_amdgcn_fmed3f(x, -c, c);
  const float t = fmaf(xc * xc, a, -1.0f);
  float p = 8.193590911e-04f;
  p = fmaf(p, t, -2.259161556e-03f);
  p = fmaf(p, t, 3.079173155e-03f);
  p = fmaf(p, t, -5.413250532e-03f);
  p = fmaf(p, t, 1.115707587e-02f);
  p = fmaf(p, t, -1.891482994e-02f);
  p = fmaf(p, t, 2.837206237e-02f);
  p = fmaf(p, t, -4.013447464e-02f);
  p = fmaf(p, t, 5.469175428e-02f);
  p = fmaf(p, t, -7.719228417e-02f);
  p = fmaf(p, t, 1.569050848e-01f);
  return x * fmaf(xc, p, 0.5f);
}

__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---------------------------------------------------------------------------
// GEMM (vector ALU): C[M][N] = op(A) op(B); op(A) is M x K, op(B) is K x N.
// TA: A stored [K][M] (else [M][K]); TB: B stored [N][K] (else [K][N]).
// 256 threads, 64 x 64 tile, K chunks of 16; thread owns 4 x 4 outputs.

template <bool TA, bool TB, bool BF>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, const float* __restrict__ B,
                                              float* __restrict__ C, int M, int N, int K, int accumulate) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tid = threadIdx.x, tm = tid & 15, tn = tid >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
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
      if (gk < K && gm < M) va = TA ? A[(int64_t)gk * M + gm] : A[(int64_t)gm * K + gk];
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
      if (gkb < K && gn < N) vb = TB ? B[(int64_t)gn * K + gkb] : B[(int64_t)gkb * N + gn];
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
      float* dst = C + (int64_t)gm * N + gn;
      *dst = accumulate ? *dst + acc[a][b] : acc[a][b];
    }
  }
}

void launch_gemm(Ctx* c, bool ta, bool tb, bool bf, const float* A, const float* B, float* C, int M, int N, int K,
                 bool accumulate) {
  ProfScope ps(c, "mlp_gemm");
  if (M == 0 || N == 0) return;
  dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64));
#define PTS_GEMM(TA_, TB_, BF_) \
  hipLaunchKernelGGL((k_gemm<TA_, TB_, BF_>), grid, dim3(256), 0, c->stream, A, B, C, M, N, K, accumulate ? 1 : 0)
  if (!ta && tb && !bf) PTS_GEMM(false, true, false);
  else if (!ta && tb && bf) PTS_GEMM(false, true, true);
  else if (!ta && !tb && !bf) PTS_GEMM(false, false, false);
  else if (!ta && !tb && bf) PTS_GEMM(false, false, true);
  else if (ta && !tb && !bf) PTS_GEMM(true, false, false);
  else if (ta && !tb && bf) PTS_GEMM(true, false, true);
  else fail(PTS_ERR_ARG, "gemm: unsupported transpose form");
#undef PTS_GEMM
  check_launch("k_gemm");
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

// out[n] = sum_m G[m][n] in row order
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ G, int64_t M, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t m = 0; m < M; ++m) s += G[m * N + n];
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

__global__ __launch_bounds__(256) void k_to_bf16_pad(const float* __restrict__ src, int rows, int cols, int rows_p,
                                                     int cols_p, uint16_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows_p * cols_p) return;
  const int r = (int)(t / cols_p), cc = (int)(t % cols_p);
  dst[t] = (r < rows && cc < cols) ? bf16_bits(src[(int64_t)r * cols + cc]) : (uint16_t)0;
}

// Xb[q][k] = bf16(Qp[q][k] * scale[k]) for k < n_in, zero up to K
__global__ __launch_bounds__(256) void k_mlp_inputs(const float* __restrict__ Qp, int ld, int64_t nq,
                                                    const float* __restrict__ scale, int n_in, int K,
                                                    uint16_t* __restrict__ Xb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq * K) return;
  const int64_t q = t / K;
  const int k = (int)(t - q * K);
  Xb[t] = (k < n_in) ? bf16_bits(Qp[q * ld + k] * scale[k]) : (uint16_t)0;
}

unsigned eblocks(int64_t n) { return (unsigned)ceil_div(n, 256); }

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
  hipLaunchKernelGGL(k_colsum, dim3(eblocks(N)), dim3(256), 0, c->stream, G, M, N, out);
  check_launch("k_colsum");
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
void launch_to_bf16_pad(Ctx* c, const float* src, int rows, int cols, int rows_p, int cols_p, uint16_t* dst) {
  hipLaunchKernelGGL(k_to_bf16_pad, dim3(eblocks((int64_t)rows_p * cols_p)), dim3(256), 0, c->stream, src, rows, cols,
                     rows_p, cols_p, dst);
  check_launch("k_to_bf16_pad");
}
void launch_mlp_inputs(Ctx* c, const float* Qp, int ld, int64_t nq, const float* scale, int n_in, int K, uint16_t* Xb) {
  ProfScope ps(c, "mlp_inputs");
  if (nq == 0) return;
  hipLaunchKernelGGL(k_mlp_inputs, dim3(eblocks(nq * K)), dim3(256), 0, c->stream, Qp, ld, nq, scale, n_in, K, Xb);
  check_launch("k_mlp_inputs");
}

// ---------------------------------------------------------------------------
// matrix-core inference layers

constexpr int ML_WAVES = 8;
constexpr int ML_THREADS = ML_WAVES * 64;
constexpr int ML_QPB = ML_WAVES * 32;  // queries per block (one 32-query tile per wave)

template <int KS>
struct MlpSmem {
  uint4 frag[2][KS][64];  // one 32-row weight tile per buffer, fragment order
  float bias[2][32];
};

template <int KS>
__device__ __forceinline__ void wtile_load(uint4 (&R)[(32 * KS * 2 + ML_THREADS - 1) / ML_THREADS], float& rb,
                                           const uint16_t* __restrict__ Wb, const float* __restrict__ bias, int n0,
                                           int N, int tid) {
  constexpr int CH = KS * 2, NCH = 32 * CH, PER = (NCH + ML_THREADS - 1) / ML_THREADS;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int cidx = tid + u * ML_THREADS;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (cidx < NCH) {
      const int row = cidx / CH, ch = cidx - row * CH;
      if (n0 + row < N) v = reinterpret_cast<const uint4*>(Wb + (int64_t)(n0 + row) * (KS * 16))[ch];
    }
    R[u] = v;
  }
  if (tid < 32) rb = (n0 + tid < N) ? bias[n0 + tid] : -FLT_MAX;
}

template <int KS>
__device__ __forceinline__ void wtile_store(const uint4 (&R)[(32 * KS * 2 + ML_THREADS - 1) / ML_THREADS], float rb,
                                            MlpSmem<KS>& S, int buf, int tid) {
  constexpr int CH = KS * 2, NCH = 32 * CH, PER = (NCH + ML_THREADS - 1) / ML_THREADS;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int cidx = tid + u * ML_THREADS;
    if (cidx < NCH) {
      const int row = cidx / CH, ch = cidx - row * CH;
      S.frag[buf][ch >> 1][(ch & 1) * 32 + row] = R[u];
    }
  }
  if (tid < 32) S.bias[buf][tid] = rb;
}

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
  __device__ __forceinline__ void insert(float x, int id) {  // descending; ties keep the earlier (lower) id
#pragma unroll
    for (int t = P - 1; t > 0; --t) {
      const bool s = x > v[t - 1];
      const bool n = x > v[t];
      v[t] = s ? v[t - 1] : (n ? x : v[t]);
      i[t] = s ? i[t - 1] : (n ? id : i[t]);
    }
    if (x > v[0]) {
      v[0] = x;
      i[0] = id;
    }
  }
};

constexpr int ML_P = 8;
constexpr int ML_QT = 1;  // 32-query tiles per wave

// MODE 0: Y[q][n] = bf16(GELU(X W^T + b)); MODE 1: top-P leaves + margin.
template <int KS, int MODE>
__global__ __launch_bounds__(512) void k_mlp_layer(const uint16_t* __restrict__ X, int64_t nq,
                                                   const uint16_t* __restrict__ Wb, const float* __restrict__ bias,
                                                   int N, uint16_t* __restrict__ Y, int kout,
                                                   int32_t* __restrict__ leaves, float* __restrict__ margin) {
  __shared__ MlpSmem<KS> sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t qbase = (int64_t)blockIdx.x * ML_QPB + wave * 32;
  bf16x8 B[ML_QT][KS];
#pragma unroll
  for (int qt = 0; qt < ML_QT; ++qt) {
    const int64_t q = qbase + qt * 32 + (lane & 31);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      uint4 u = make_uint4(0, 0, 0, 0);
      if (q < nq) u = reinterpret_cast<const uint4*>(X + q * (KS * 16))[2 * kk + (lane >> 5)];
      B[qt][kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
  }
  TopP<ML_P> top[ML_QT];
  float smax[ML_QT], ssum[ML_QT];
  if (MODE == 1) {
#pragma unroll
    for (int qt = 0; qt < ML_QT; ++qt) {
      top[qt].init();
      smax[qt] = -FLT_MAX;
      ssum[qt] = 0.f;
    }
  }
  const int ntiles = (N + 31) / 32;
  uint4 R[(32 * KS * 2 + ML_THREADS - 1) / ML_THREADS];
  float rb = 0.f;
  wtile_load<KS>(R, rb, Wb, bias, 0, N, tid);
  wtile_store<KS>(R, rb, sm, 0, tid);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    const bool more = t + 1 < ntiles;
    if (more) wtile_load<KS>(R, rb, Wb, bias, (t + 1) * 32, N, tid);
    bf16x8 A[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const uint4 u = sm.frag[buf][kk][lane];
      A[kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
    floatx16 cinit;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 b4 = *reinterpret_cast<const float4*>(&sm.bias[buf][8 * g + 4 * (lane >> 5)]);
      cinit[4 * g + 0] = b4.x;
      cinit[4 * g + 1] = b4.y;
      cinit[4 * g + 2] = b4.z;
      cinit[4 * g + 3] = b4.w;
    }
    const int nbase = t * 32 + 4 * (lane >> 5);
#pragma unroll
    for (int qt = 0; qt < ML_QT; ++qt) {
      floatx16 acc = cinit;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[qt][kk], acc, 0, 0, 0);
      const int64_t q = qbase + qt * 32 + (lane & 31);
      if (MODE == 0) {
        if (q < nq) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int n = nbase + 8 * g;
            if (n < N) {  // N is a multiple of 4: a group of 4 is all in or all out
              uint2 pk;
              pk.x = (uint32_t)bf16_bits(gelu_poly_f(acc[4 * g + 0])) |
                     ((uint32_t)bf16_bits(gelu_poly_f(acc[4 * g + 1])) << 16);
              pk.y = (uint32_t)bf16_bits(gelu_poly_f(acc[4 * g + 2])) |
                     ((uint32_t)bf16_bits(gelu_poly_f(acc[4 * g + 3])) << 16);
              *reinterpret_cast<uint2*>(Y + q * kout + n) = pk;
            }
          }
        }
      } else {
        float mloc = acc[0];
#pragma unroll
        for (int r = 1; r < 16; ++r) mloc = fmaxf(mloc, acc[r]);
        if (mloc > smax[qt]) {  // rescale the running sum to the new maximum
          ssum[qt] *= expf(smax[qt] - mloc);
          smax[qt] = mloc;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int n = nbase + 8 * (r >> 2) + (r & 3);
          if (n < N) ssum[qt] += expf(acc[r] - smax[qt]);
        }
        if (__any(mloc > top[qt].v[ML_P - 1])) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int n = nbase + 8 * (r >> 2) + (r & 3);
            if (n < N && acc[r] > top[qt].v[ML_P - 1]) top[qt].insert(acc[r], n);
          }
        }
      }
    }
    if (more) wtile_store<KS>(R, rb, sm, buf ^ 1, tid);
    __syncthreads();
  }
  if (MODE == 1) {
#pragma unroll
    for (int qt = 0; qt < ML_QT; ++qt) {
      // merge with the partner lane (same query, other 16 rows of each tile)
      const float om = __shfl_xor(smax[qt], 32, 64);
      const float os = __shfl_xor(ssum[qt], 32, 64);
      const float m = fmaxf(smax[qt], om);
      const float s = ssum[qt] * expf(smax[qt] - m) + os * expf(om - m);
      float ov[ML_P];
      int oi[ML_P];
#pragma unroll
      for (int t = 0; t < ML_P; ++t) {
        ov[t] = __shfl_xor(top[qt].v[t], 32, 64);
        oi[t] = __shfl_xor(top[qt].i[t], 32, 64);
      }
      const int64_t q = qbase + qt * 32 + (lane & 31);
      if (lane < 32 && q < nq) {
        // merge two descending lists; equal scores: lower leaf first
        int a = 0, b = 0;
        float best[2] = {-FLT_MAX, -FLT_MAX};
#pragma unroll
        for (int t = 0; t < ML_P; ++t) {
          float va = -FLT_MAX, vb = -FLT_MAX;
          int ia = INT_MAX, ib = INT_MAX;
#pragma unroll
          for (int u = 0; u < ML_P; ++u) {
            if (u == a) {
              va = top[qt].v[u];
              ia = top[qt].i[u];
            }
            if (u == b) {
              vb = ov[u];
              ib = oi[u];
            }
          }
          const bool take_a = (va > vb) || (va == vb && ia < ib);
          const int id = take_a ? ia : ib;
          const float vv = take_a ? va : vb;
          if (take_a) ++a;
          else ++b;
          if (t < kout) leaves[q * kout + t] = (id == INT_MAX) ? -1 : id;
          if (t < 2) best[t] = vv;
        }
        // p1 - p2 = (1 - exp(l2 - l1)) / sum_j exp(l_j - l1)
        const float denom = s * expf(m - best[0]);
        margin[q] = (best[1] == -FLT_MAX) ? 1.0f : (1.0f - expf(best[1] - best[0])) / denom;
      }
    }
  }
}

// Output layer, exact top-P in two passes over the weight tiles.  Pass 1
// keeps, per value slot, the running maximum of the logits (one max per
// logit, no ids).  After it the query's largest logit m is known, and the
// P-th largest of its 32 slot maxima (two half-lanes x 16 slots) is at most
// its P-th largest logit.  Pass 2 recomputes the logits on the matrix cores,
// inserts only logits at or above that bound into the sorted top-P, and sums
// exp(l - m) for the softmax normaliser, skipping tiles whose logits are all
// below m - 30 (their terms are below 1e-13 of the largest).
template <int KS, int PP>
__global__ __launch_bounds__(512) void k_mlp_out_topk(const uint16_t* __restrict__ X, int64_t nq,
                                                      const uint16_t* __restrict__ Wb, const float* __restrict__ bias,
                                                      int N, int kout, int32_t* __restrict__ leaves,
                                                      float* __restrict__ margin) {
  __shared__ MlpSmem<KS> sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t qbase = (int64_t)blockIdx.x * ML_QPB + wave * 32;
  bf16x8 B[ML_QT][KS];
#pragma unroll
  for (int qt = 0; qt < ML_QT; ++qt) {
    const int64_t q = qbase + qt * 32 + (lane & 31);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      uint4 u = make_uint4(0, 0, 0, 0);
      if (q < nq) u = reinterpret_cast<const uint4*>(X + q * (KS * 16))[2 * kk + (lane >> 5)];
      B[qt][kk] = *reinterpret_cast<const bf16x8*>(&u);
    }
  }
  float slot[ML_QT][16], tau[ML_QT], mx[ML_QT], ssum[ML_QT];
  TopP<PP> top[ML_QT];
#pragma unroll
  for (int qt = 0; qt < ML_QT; ++qt) {
    ssum[qt] = 0.f;
    top[qt].init();
#pragma unroll
    for (int r = 0; r < 16; ++r) slot[qt][r] = -FLT_MAX;
  }
  const int ntiles = (N + 31) / 32;
  uint4 R[(32 * KS * 2 + ML_THREADS - 1) / ML_THREADS];
  float rb = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    wtile_load<KS>(R, rb, Wb, bias, 0, N, tid);
    __syncthreads();  // the previous pass has finished reading the buffers
    wtile_store<KS>(R, rb, sm, 0, tid);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
      const int buf = t & 1;
      const bool more = t + 1 < ntiles;
      if (more) wtile_load<KS>(R, rb, Wb, bias, (t + 1) * 32, N, tid);
      bf16x8 A[KS];
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const uint4 u = sm.frag[buf][kk][lane];
        A[kk] = *reinterpret_cast<const bf16x8*>(&u);
      }
      floatx16 cinit;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 b4 = *reinterpret_cast<const float4*>(&sm.bias[buf][8 * g + 4 * (lane >> 5)]);
        cinit[4 * g + 0] = b4.x;
        cinit[4 * g + 1] = b4.y;
        cinit[4 * g + 2] = b4.z;
        cinit[4 * g + 3] = b4.w;
      }
      const int nbase = t * 32 + 4 * (lane >> 5);
#pragma unroll
      for (int qt = 0; qt < ML_QT; ++qt) {
        floatx16 acc = cinit;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[kk], B[qt][kk], acc, 0, 0, 0);
        // rows past N carry bias -FLT_MAX and zero weights: acc = -FLT_MAX, never selected
        if (pass == 0) {
#pragma unroll
          for (int r = 0; r < 16; ++r) slot[qt][r] = fmaxf(slot[qt][r], acc[r]);
        } else {
          float mloc = acc[0];
#pragma unroll
          for (int r = 1; r < 16; ++r) mloc = fmaxf(mloc, acc[r]);
          if (__any(mloc >= tau[qt])) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int n = nbase + 8 * (r >> 2) + (r & 3);
              if (acc[r] >= tau[qt] && acc[r] > top[qt].v[PP - 1]) top[qt].insert(acc[r], n);
            }
          }
          if (__any(mloc >= mx[qt] - 30.0f)) {
#pragma unroll
            for (int r = 0; r < 16; ++r) ssum[qt] += __expf(acc[r] - mx[qt]);
          }
        }
      }
      if (more) wtile_store<KS>(R, rb, sm, buf ^ 1, tid);
      __syncthreads();
    }
    if (pass == 0) {
      // m = largest logit; tau = kout-th largest of the 32 slot maxima
#pragma unroll
      for (int qt = 0; qt < ML_QT; ++qt) {
        TopP<ML_P> s8;
        s8.init();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          s8.insert(slot[qt][r], r);
          s8.insert(__shfl_xor(slot[qt][r], 32, 64), 16 + r);
        }
        float tk = s8.v[0];
#pragma unroll
        for (int u = 1; u < ML_P; ++u)
          if (u < kout) tk = s8.v[u];
        tau[qt] = tk;
        mx[qt] = s8.v[0];
      }
    }
  }
#pragma unroll
  for (int qt = 0; qt < ML_QT; ++qt) {
    const float s = ssum[qt] + __shfl_xor(ssum[qt], 32, 64);  // both halves share mx
    float ov[PP];
    int oi[PP];
#pragma unroll
    for (int t = 0; t < PP; ++t) {
      ov[t] = __shfl_xor(top[qt].v[t], 32, 64);
      oi[t] = __shfl_xor(top[qt].i[t], 32, 64);
    }
    const int64_t q = qbase + qt * 32 + (lane & 31);
    if (lane < 32 && q < nq) {
      int a = 0, b = 0;
      float best[2] = {-FLT_MAX, -FLT_MAX};
#pragma unroll
      for (int t = 0; t < PP; ++t) {
        float va = -FLT_MAX, vb = -FLT_MAX;
        int ia = INT_MAX, ib = INT_MAX;
#pragma unroll
        for (int u = 0; u < PP; ++u) {
          if (u == a) {
            va = top[qt].v[u];
            ia = top[qt].i[u];
          }
          if (u == b) {
            vb = ov[u];
            ib = oi[u];
          }
        }
        const bool take_a = (va > vb) || (va == vb && ia < ib);
        const int id = take_a ? ia : ib;
        const float vv = take_a ? va : vb;
        if (take_a) ++a;
        else ++b;
        if (t < kout) leaves[q * kout + t] = (id == INT_MAX) ? -1 : id;
        if (t < 2) best[t] = vv;
      }
      // p1 - p2 = (1 - exp(l2 - l1)) / sum_j exp(l_j - l1), with l1 = mx
      margin[q] = (best[1] == -FLT_MAX) ? 1.0f : (1.0f - __expf(best[1] - best[0])) / s;
    }
  }
}

#define PTS_MLP_KS_SWITCH(K, ...)                                                                  \
  switch (K) {                                                                                     \
    case 32: { constexpr int KSC = 2; __VA_ARGS__; } break;                                        \
    case 64: { constexpr int KSC = 4; __VA_ARGS__; } break;                                        \
    case 96: { constexpr int KSC = 6; __VA_ARGS__; } break;                                        \
    case 128: { constexpr int KSC = 8; __VA_ARGS__; } break;                                       \
    case 256: { constexpr int KSC = 16; __VA_ARGS__; } break;                                      \
    default: ::pts::fail(PTS_ERR_UNSUPPORTED, "MLP layer width must be 32/64/96/128/256");         \
  }

void launch_mlp_hidden(Ctx* c, const uint16_t* X, int64_t nq, int K, const uint16_t* Wb, const float* bias, int N,
                       uint16_t* Y) {
  ProfScope ps(c, "mlp_hidden_mfma");
  if (nq == 0) return;
  PTS_REQUIRE(N % 4 == 0, PTS_ERR_UNSUPPORTED, "MLP hidden width must be a multiple of 4");
  PTS_MLP_KS_SWITCH(K, hipLaunchKernelGGL((k_mlp_layer<KSC, 0>), dim3((unsigned)ceil_div(nq, ML_QPB)), dim3(ML_THREADS), 0,
                                          c->stream, X, nq, Wb, bias, N, Y, N, nullptr, nullptr));
  check_launch("k_mlp_layer<hidden>");
}

void launch_mlp_out_topk(Ctx* c, const uint16_t* X, int64_t nq, int K, const uint16_t* Wb, const float* bias, int N,
                         int k, int32_t* leaves, float* margin) {
  ProfScope ps(c, "mlp_out_topk_mfma");
  if (nq == 0) return;
  PTS_REQUIRE(k >= 1 && k <= ML_P, PTS_ERR_ARG, "proposals must be 1..8");
  if (k <= 4) {
    PTS_MLP_KS_SWITCH(K, hipLaunchKernelGGL((k_mlp_out_topk<KSC, 4>), dim3((unsigned)ceil_div(nq, ML_QPB)), dim3(ML_THREADS),
                                            0, c->stream, X, nq, Wb, bias, N, k, leaves, margin));
  } else {
    PTS_MLP_KS_SWITCH(K, hipLaunchKernelGGL((k_mlp_out_topk<KSC, 8>), dim3((unsigned)ceil_div(nq, ML_QPB)), dim3(ML_THREADS),
                                            0, c->stream, X, nq, Wb, bias, N, k, leaves, margin));
  }
  check_launch("k_mlp_out_topk");
}

}  // namespace pts
