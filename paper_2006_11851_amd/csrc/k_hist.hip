// Histogram matching (Section 3, Eq. 9, and Section 4 step 4).
//
// Eq. 9 lowers the blend weight of a matched neighbourhood whose colour is
// over-represented in the output: W' = W / (1 + sum_j max[0, H_x,j(b_j(c)) -
// H_z,j(b_j(c))]), H_x,j / H_z,j the channel-j histograms (fractions) of the
// output and of the exemplar, c the colour of the matched exemplar window
// (its centre pixel), b_j(c) its bin.  The output histogram is a reduction
// over every pixel per iteration (privatised in LDS, one global atomic per
// bin and block); the factor is one gather and three lookups per window.
//
// The final match gives each colour channel of the output the exemplar's
// distribution rank for rank: the output values are sorted (stable: ties in
// pixel order) and the i-th of n takes the exemplar's sorted value of rank
// floor((i + 1/2) n_z / n).
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace pts {

constexpr int HIST_MAX_BINS = 256;

__device__ __forceinline__ int bin_of(float v, int bins) {
  const int b = (int)floorf(v * (float)bins);
  return min(max(b, 0), bins - 1);
}

// counts [3][bins] += the R, G, B bins of the image's pixels
__global__ __launch_bounds__(256) void k_channel_hist(const float4* __restrict__ img, int64_t n, int bins,
                                                      unsigned* __restrict__ counts) {
  __shared__ unsigned h[3 * HIST_MAX_BINS];
  for (int i = threadIdx.x; i < 3 * bins; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = img[p];
    atomicAdd(&h[bin_of(v.x, bins)], 1u);
    atomicAdd(&h[bins + bin_of(v.y, bins)], 1u);
    atomicAdd(&h[2 * bins + bin_of(v.z, bins)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * bins; i += blockDim.x)
    if (h[i]) atomicAdd(&counts[i], h[i]);
}

// factor[q] = 1 / (1 + histogram excess of the centre colour of window nn[q])
__global__ __launch_bounds__(256) void k_hist_factor(const int32_t* __restrict__ nn, int64_t nq,
                                                     const float4* __restrict__ ex, int Hz, int Wz, int w,
                                                     const unsigned* __restrict__ hx, const unsigned* __restrict__ hz,
                                                     float inv_nx, float inv_nz, int bins,
                                                     float* __restrict__ factor) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int nu = Wz - w + 1;
  const int64_t N = (int64_t)(Hz - w + 1) * nu;
  const int e = nn[q];
  if (e < 0 || e >= N) {
    factor[q] = 1.f;
    return;
  }
  const int ey = e / nu, exx = e - ey * nu;
  const float4 c = ex[(int64_t)(ey + w / 2) * Wz + exx + w / 2];
  const float cv[3] = {c.x, c.y, c.z};
  float exc = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int b = j * bins + bin_of(cv[j], bins);
    exc += fmaxf(0.f, (float)hx[b] * inv_nx - (float)hz[b] * inv_nz);
  }
  factor[q] = 1.f / (1.f + exc);
}

// keys[p] = channel j of pixel p, idx[p] = p
__global__ __launch_bounds__(256) void k_extract_channel(const float4* __restrict__ img, int64_t n, int j,
                                                         float* __restrict__ keys, int32_t* __restrict__ idx) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float4 v = img[p];
  keys[p] = j == 0 ? v.x : (j == 1 ? v.y : v.z);
  if (idx) idx[p] = (int32_t)p;
}

// pixel order[i] (the i-th smallest) takes zsorted[floor((2 i + 1) nz / (2 n))]
__global__ __launch_bounds__(256) void k_match_scatter(const int32_t* __restrict__ order, int64_t n, int j,
                                                       const float* __restrict__ zsorted, int64_t nz,
                                                       float4* __restrict__ img) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t src = min(((2 * i + 1) * nz) / (2 * n), nz - 1);
  float* px = reinterpret_cast<float*>(img + order[i]);
  px[j] = zsorted[src];
}

// W[q] = max(dist[q], delta)^(r - 2) (Eq. 7), times factor[q] when given (Eq. 9)
__global__ __launch_bounds__(256) void k_irls_weights(const float* __restrict__ dist,
                                                      const float* __restrict__ factor, int64_t nq, float r,
                                                      float delta, float* __restrict__ W) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const float wq = powf(fmaxf(dist[q], delta), r - 2.0f);
  W[q] = factor ? wq * factor[q] : wq;
}

static unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, 256)); }

void launch_irls_weights(Ctx* c, const float* dist, const float* factor, int64_t nq, float r, float delta, float* W) {
  ProfScope ps(c, "irls_weights");
  if (nq == 0) return;
  hipLaunchKernelGGL(k_irls_weights, grid_for(nq), dim3(256), 0, c->stream, dist, factor, nq, r, delta, W);
  check_launch("k_irls_weights");
}

void launch_channel_hist(Ctx* c, const float* img, int64_t n, int bins, unsigned* counts) {
  ProfScope ps(c, "channel_hist");
  PTS_REQUIRE(bins >= 2 && bins <= HIST_MAX_BINS, PTS_ERR_ARG, "histogram bins must be 2..256");
  launch_zero_i32(c, reinterpret_cast<int32_t*>(counts), 3 * bins);
  if (n == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 4 * (int64_t)c->n_cu);
  hipLaunchKernelGGL(k_channel_hist, dim3(grid), dim3(256), 0, c->stream, reinterpret_cast<const float4*>(img), n,
                     bins, counts);
  check_launch("k_channel_hist");
}

void launch_hist_factor(Ctx* c, const int32_t* nn, int64_t nq, const float* ex, int Hz, int Wz, int w,
                        const unsigned* hx, int64_t nx, const unsigned* hz, int64_t nz, int bins, float* factor) {
  ProfScope ps(c, "hist_factor");
  if (nq == 0) return;
  hipLaunchKernelGGL(k_hist_factor, grid_for(nq), dim3(256), 0, c->stream, nn, nq,
                     reinterpret_cast<const float4*>(ex), Hz, Wz, w, hx, hz, 1.0f / (float)nx, 1.0f / (float)nz,
                     bins, factor);
  check_launch("k_hist_factor");
}

const float* hist_weight_factors(Ctx* c, const int32_t* nn, int64_t nq, const float* x, int H, int W,
                                 const float* ex, int Hz, int Wz, int w, int bins) {
  unsigned* hx = c->buf<unsigned>("hist_x", 3 * HIST_MAX_BINS);
  unsigned* hz = c->buf<unsigned>("hist_z", 3 * HIST_MAX_BINS);
  float* factor = c->buf<float>("hist_factor", (size_t)std::max<int64_t>(1, nq));
  launch_channel_hist(c, x, (int64_t)H * W, bins, hx);
  launch_channel_hist(c, ex, (int64_t)Hz * Wz, bins, hz);
  launch_hist_factor(c, nn, nq, ex, Hz, Wz, w, hx, (int64_t)H * W, hz, (int64_t)Hz * Wz, bins, factor);
  return factor;
}

// ascending sort of (keys, values) pairs, stable; the scratch comes from the context
static void sort_pairs(Ctx* c, const float* kin, float* kout, const int32_t* vin, int32_t* vout, int64_t n) {
  PTS_REQUIRE(n < ((int64_t)1 << 31), PTS_ERR_UNSUPPORTED, "histogram match: image too large");
  size_t bytes = 0;
  PTS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, (int)n, 0, 32, c->stream));
  void* tmp = c->buf<uint8_t>("hm_sort_tmp", bytes + 1);
  PTS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, (int)n, 0, 32, c->stream));
}

void histogram_match(Ctx* c, float* x, int H, int W, const float* ex, int Hz, int Wz) {
  ProfScope ps(c, "histogram_match");
  const int64_t n = (int64_t)H * W, nz = (int64_t)Hz * Wz;
  if (n == 0) return;
  float* keys = c->buf<float>("hm_keys", (size_t)std::max(n, nz));
  float* ksorted = c->buf<float>("hm_ksorted", (size_t)n);
  int32_t* idx = c->buf<int32_t>("hm_idx", (size_t)n);
  int32_t* order = c->buf<int32_t>("hm_order", (size_t)n);
  float* zsorted = c->buf<float>("hm_zsorted", (size_t)nz);
  int32_t* zidx = c->buf<int32_t>("hm_zidx", (size_t)nz);
  int32_t* zorder = c->buf<int32_t>("hm_zorder", (size_t)nz);
  for (int j = 0; j < 3; ++j) {
    // the exemplar's sorted channel
    hipLaunchKernelGGL(k_extract_channel, grid_for(nz), dim3(256), 0, c->stream, reinterpret_cast<const float4*>(ex),
                       nz, j, keys, zidx);
    check_launch("k_extract_channel");
    sort_pairs(c, keys, zsorted, zidx, zorder, nz);
    // the output's order, then the rank-for-rank values
    hipLaunchKernelGGL(k_extract_channel, grid_for(n), dim3(256), 0, c->stream, reinterpret_cast<const float4*>(x), n,
                       j, keys, idx);
    check_launch("k_extract_channel");
    sort_pairs(c, keys, ksorted, idx, order, n);
    hipLaunchKernelGGL(k_match_scatter, grid_for(n), dim3(256), 0, c->stream, order, n, j, zsorted, nz,
                       reinterpret_cast<float4*>(x));
    check_launch("k_match_scatter");
  }
}

}  // namespace pts
