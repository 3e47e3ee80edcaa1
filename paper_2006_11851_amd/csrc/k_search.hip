// Exhaustive search kernels and the winner distance.
//
// Methodology 2.1 (Eq. 4): z_q is the exemplar neighbourhood nearest to the
// output neighbourhood x_q in the Euclidean norm.  The exhaustive kernel
// below is the exact reference of the search (full D or PCA space), FP32,
// direct form sum (x - z)^2 accumulated in a fixed order so that identical
// windows give identical distances; ties go to the lowest window id.
#include <cfloat>
#include <climits>

#include "kernels.hpp"
#include "device_util.hpp"

namespace pts {

void validate_grid(int H, int W, int w, int s) {
  PTS_REQUIRE(w >= 2 && w <= 32 && w % 2 == 0, PTS_ERR_UNSUPPORTED, "w must be even, 2..32");
  PTS_REQUIRE(s >= 1 && s <= w, PTS_ERR_UNSUPPORTED, "stride must be in 1..w");
  PTS_REQUIRE(H >= w && W >= w, PTS_ERR_ARG, "output smaller than a window");
  PTS_REQUIRE((H - w) % s == 0 && W % s == 0, PTS_ERR_UNSUPPORTED, "stride must tile the output: (H-w)%s==0, W%s==0");
  PTS_REQUIRE(H % 2 == 0 && W % 2 == 0, PTS_ERR_UNSUPPORTED, "2x2 patches need even H and W");
  PTS_REQUIRE((int64_t)H * W <= (int64_t)1 << 28, PTS_ERR_UNSUPPORTED, "output larger than 2^28 pixels");
}

// ---------------------------------------------------------------------------
// window materialisation: out[win][(dy*w+dx)*4+c]

__global__ __launch_bounds__(256) void k_gather_windows(const float4* __restrict__ img, int H, int W, int w,
                                                        int s, int rows, int cols, int wrap,
                                                        float4* __restrict__ out) {
  const int64_t ww = (int64_t)w * w;
  const int64_t total = (int64_t)rows * cols * ww;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t win = t / ww;
    const int p = (int)(t - win * ww);
    const int i = (int)(win / cols), j = (int)(win - (int64_t)i * cols);
    const int dy = p / w, dx = p - dy * w;
    const int y = i * s + dy;
    int x = j * s + dx;
    if (wrap) x %= W;
    out[t] = img[(int64_t)y * W + x];
  }
}

void launch_gather_windows(Ctx* c, const float* img, int H, int W, int w, int s, bool wrap, float* out) {
  ProfScope ps(c, "gather_windows");
  int rows, cols;
  if (wrap) {
    rows = (H - w) / s + 1;
    cols = W / s;
  } else {
    rows = (H - w) / s + 1;
    cols = (W - w) / s + 1;
  }
  int64_t total = (int64_t)rows * cols * w * w;
  if (total == 0) return;
  unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 65536);
  hipLaunchKernelGGL(k_gather_windows, dim3(blocks), dim3(256), 0, c->stream,
                     reinterpret_cast<const float4*>(img), H, W, w, s, rows, cols, wrap ? 1 : 0,
                     reinterpret_cast<float4*>(out));
  check_launch("k_gather_windows");
}

// ---------------------------------------------------------------------------
// exhaustive argmin, direct form.  Block: 256 threads, 64 queries x 64
// exemplar rows per tile, D in chunks of 32 through LDS.  Thread (tq, te)
// owns queries tq + 16 i and rows te + 16 j (i, j < 4).  Grid: x = query
// tiles, y = splits of the exemplar rows; partial winners merged after.

constexpr int AM_TQ = 64, AM_TE = 64, AM_KC = 32;

__device__ __forceinline__ bool better(float d, int id, float bd, int bid) {
  return d < bd || (d == bd && id < bid);
}

__global__ __launch_bounds__(256) void k_argmin_direct(const float* __restrict__ Q, int64_t nq,
                                                       const float* __restrict__ Z, int64_t N, int D,
                                                       const int32_t* __restrict__ zid, int64_t per_split,
                                                       float* __restrict__ part_d, int32_t* __restrict__ part_i) {
  __shared__ float Qs[AM_TQ][AM_KC + 1];
  __shared__ float Zs[AM_TE][AM_KC + 1];
  __shared__ float rd[16][AM_TQ];
  __shared__ int ri[16][AM_TQ];
  const int tid = threadIdx.x, tq = tid & 15, te = tid >> 4;
  const int64_t q0 = (int64_t)blockIdx.x * AM_TQ;
  const int64_t e_begin = (int64_t)blockIdx.y * per_split;
  const int64_t e_end = min(N, e_begin + per_split);
  float bd[4];
  int bi[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bd[i] = FLT_MAX;
    bi[i] = INT_MAX;
  }
  for (int64_t e0 = e_begin; e0 < e_end; e0 += AM_TE) {
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int k0 = 0; k0 < D; k0 += AM_KC) {
      for (int t = tid; t < AM_TQ * AM_KC; t += 256) {
        const int r = t / AM_KC, cc = t - r * AM_KC;
        const int64_t q = q0 + r;
        const int k = k0 + cc;
        Qs[r][cc] = (q < nq && k < D) ? Q[q * D + k] : 0.f;
        const int64_t e = e0 + r;
        Zs[r][cc] = (e < e_end && k < D) ? Z[e * D + k] : 0.f;
      }
      __syncthreads();
#pragma unroll 4
      for (int k = 0; k < AM_KC; ++k) {
        float qv[4], zv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) qv[i] = Qs[tq + 16 * i][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) zv[j] = Zs[te + 16 * j][k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float t = qv[i] - zv[j];
            acc[i][j] = fmaf(t, t, acc[i][j]);
          }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t e = e0 + te + 16 * j;
      if (e < e_end) {
        const int id = zid ? zid[e] : (int)e;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (better(acc[i][j], id, bd[i], bi[i])) {
            bd[i] = acc[i][j];
            bi[i] = id;
          }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rd[te][tq + 16 * i] = bd[i];
    ri[te][tq + 16 * i] = bi[i];
  }
  __syncthreads();
  if (tid < AM_TQ) {
    float b = rd[0][tid];
    int id = ri[0][tid];
    for (int t = 1; t < 16; ++t)
      if (better(rd[t][tid], ri[t][tid], b, id)) {
        b = rd[t][tid];
        id = ri[t][tid];
      }
    const int64_t q = q0 + tid;
    if (q < nq) {
      part_d[(int64_t)blockIdx.y * nq + q] = b;
      part_i[(int64_t)blockIdx.y * nq + q] = id;
    }
  }
}

__global__ __launch_bounds__(256) void k_argmin_merge(const float* __restrict__ part_d,
                                                      const int32_t* __restrict__ part_i, int64_t nq, int splits,
                                                      int32_t* __restrict__ best_id, float* __restrict__ best_d2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  float b = part_d[q];
  int id = part_i[q];
  for (int s = 1; s < splits; ++s) {
    const float d = part_d[(int64_t)s * nq + q];
    const int i = part_i[(int64_t)s * nq + q];
    if (better(d, i, b, id)) {
      b = d;
      id = i;
    }
  }
  best_id[q] = id;
  if (best_d2) best_d2[q] = b;
}

void launch_argmin_direct(Ctx* c, const float* Q, int64_t nq, const float* Z, int64_t N, int D,
                          const int32_t* zid, int32_t* best_id, float* best_d2) {
  ProfScope ps(c, "argmin_direct");
  if (nq == 0) return;
  PTS_REQUIRE(N > 0 && N < INT_MAX && D > 0, PTS_ERR_ARG, "argmin: bad sizes");
  const int64_t qtiles = ceil_div(nq, AM_TQ);
  // enough blocks to fill 256 CUs several times; each split holds >= 4 tiles of rows
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(ceil_div(4096, qtiles), ceil_div(N, 4 * AM_TE)));
  splits = std::min<int64_t>(splits, 65535);
  const int64_t per_split = round_up(ceil_div(N, splits), AM_TE);
  splits = ceil_div(N, per_split);
  float* pd = c->buf<float>("argmin_pd", (size_t)(splits * nq));
  int32_t* pi = c->buf<int32_t>("argmin_pi", (size_t)(splits * nq));
  hipLaunchKernelGGL(k_argmin_direct, dim3((unsigned)qtiles, (unsigned)splits), dim3(256), 0, c->stream, Q, nq, Z,
                     N, D, zid, per_split, pd, pi);
  check_launch("k_argmin_direct");
  hipLaunchKernelGGL(k_argmin_merge, dim3((unsigned)ceil_div(nq, 256)), dim3(256), 0, c->stream, pd, pi, nq,
                     (int)splits, best_id, best_d2);
  check_launch("k_argmin_merge");
}

// ---------------------------------------------------------------------------
// winner distance: one wave per query, lanes over the window's pixels.

__global__ __launch_bounds__(256) void k_winner_dist(const float4* __restrict__ x, int H, int W, int w, int s,
                                                     int cols, const float4* __restrict__ ex, int Hz, int Wz,
                                                     const int32_t* __restrict__ nn, int64_t nq,
                                                     float* __restrict__ dist) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;  // uniform per wave
  const int i = (int)(q / cols), j = (int)(q - (int64_t)i * cols);
  const int v = i * s, u = j * s;
  const int nu = Wz - w + 1;
  const int64_t N = (int64_t)(Hz - w + 1) * nu;
  const int e = nn[q];
  if (e < 0 || e >= N) {  // invalid match id: report NaN, read nothing
    if (lane == 0) dist[q] = __int_as_float(0x7fc00000);
    return;
  }
  const int ey = e / nu, exx = e - ey * nu;
  float acc = 0.f;
  for (int p = lane; p < w * w; p += 64) {
    const int dy = p / w, dx = p - dy * w;
    int xx = u + dx;
    if (xx >= W) xx -= W;
    const float4 a = x[(int64_t)(v + dy) * W + xx];
    const float4 b = ex[(int64_t)(ey + dy) * Wz + exx + dx];
    const float t0 = a.x - b.x, t1 = a.y - b.y, t2 = a.z - b.z, t3 = a.w - b.w;
    acc = fmaf(t0, t0, acc);
    acc = fmaf(t1, t1, acc);
    acc = fmaf(t2, t2, acc);
    acc = fmaf(t3, t3, acc);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) dist[q] = sqrtf(acc);
}

void launch_winner_dist(Ctx* c, const float* x, int H, int W, int w, int s, const float* ex, int Hz, int Wz,
                        const int32_t* nn, float* dist) {
  ProfScope ps(c, "winner_dist");
  Grid g{H, W, w, s};
  const int64_t nq = g.nq();
  if (nq == 0) return;
  hipLaunchKernelGGL(k_winner_dist, dim3((unsigned)ceil_div(nq, 4)), dim3(256), 0, c->stream,
                     reinterpret_cast<const float4*>(x), H, W, w, s, g.cols(), reinterpret_cast<const float4*>(ex),
                     Hz, Wz, nn, nq, dist);
  check_launch("k_winner_dist");
}

}  // namespace pts

namespace pts {

__global__ __launch_bounds__(256) void k_count_diff(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                                    int64_t n, int32_t* __restrict__ count) {
  __shared__ int s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  int local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    local += (a[i] != b[i]) ? 1 : 0;
  if (local) atomicAdd(&s, local);
  __syncthreads();
  if (threadIdx.x == 0 && s) atomicAdd(count, s);
}

void launch_count_diff(Ctx* c, const int32_t* a, const int32_t* b, int64_t n, int32_t* count) {
  ProfScope ps(c, "count_diff");
  if (n == 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, ceil_div(n, 256));
  hipLaunchKernelGGL(k_count_diff, dim3(blocks), dim3(256), 0, c->stream, a, b, n, count);
  check_launch("k_count_diff");
}

}  // namespace pts

namespace pts {

// windows of a listed subset of output-grid ids: out[r][(dy*w+dx)*4+c]
__global__ __launch_bounds__(256) void k_gather_windows_list(const float4* __restrict__ img, int H, int W, int w,
                                                             int s, int cols, int64_t nq,
                                                             const int32_t* __restrict__ qids, int64_t n,
                                                             float4* __restrict__ out) {
  const int64_t ww = (int64_t)w * w;
  const int64_t total = n * ww;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / ww;
    const int p = (int)(t - r * ww);
    int64_t q = qids[r];
    if (q < 0 || q >= nq) q = 0;  // invalid ids read window 0; the caller validated
    const int i = (int)(q / cols), j = (int)(q - (int64_t)i * cols);
    const int dy = p / w, dx = p - dy * w;
    int x = j * s + dx;
    if (x >= W) x -= W;
    out[t] = img[(int64_t)(i * s + dy) * W + x];
  }
}

__global__ __launch_bounds__(256) void k_sqrt(const float* __restrict__ a, int64_t n, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = sqrtf(a[i]);
}

void launch_exact_subset(Ctx* c, const float* x, int H, int W, int w, int s, const float* ex, int Hz, int Wz,
                         const int32_t* qids, int64_t n, int32_t* nn, float* dist) {
  ProfScope ps(c, "exact_subset");
  if (n == 0) return;
  const Grid g{H, W, w, s};
  const int D = 4 * w * w;
  const int64_t N = (int64_t)(Hz - w + 1) * (Wz - w + 1);
  float* zw = c->buf<float>("exact_zw", (size_t)N * D);
  float* qw = c->buf<float>("exact_qw_sub", (size_t)n * D);
  float* d2 = c->buf<float>("exact_d2_sub", (size_t)n);
  launch_gather_windows(c, ex, Hz, Wz, w, 1, false, zw);
  const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(n * w * w, 256), 65536);
  hipLaunchKernelGGL(k_gather_windows_list, dim3(blocks), dim3(256), 0, c->stream, reinterpret_cast<const float4*>(x), H,
                     W, w, s, g.cols(), g.nq(), qids, n, reinterpret_cast<float4*>(qw));
  check_launch("k_gather_windows_list");
  launch_argmin_direct(c, qw, n, zw, N, D, nullptr, nn, d2);
  hipLaunchKernelGGL(k_sqrt, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, d2, n, dist);
  check_launch("k_sqrt");
}

}  // namespace pts
