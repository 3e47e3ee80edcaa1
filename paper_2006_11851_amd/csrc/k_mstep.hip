// Optimisation phase (M-step) and energy.
//
// Methodology 2.1, Eqs. 6-8: with the matches fixed, IRLS minimises
// sum_q W_q ||x_q - z_q||^2 with W_q = ||x_q - z_q||^(r-2), r = 0.8.
// Methodology 2.2: points are processed as 2x2 patches, each patch from the
// neighbourhoods that contain all of it.  Here one thread owns one patch and
// gathers the matched exemplar pixels of every covering window - a gather,
// so no two threads write the same pixel and no atomics are needed.
//
// The distance is floored at delta before the power (the weight is undefined
// at zero distance); wscale (optional) multiplies each window's weight (the
// histogram factor of Eq. 9).  The energy uses the matching smooth penalty
//   rho(d) = d^r (d >= delta),  (1 - r/2) delta^r + (r/2) delta^(r-2) d^2 (d < delta).
#include <map>
#include <mutex>

#include "kernels.hpp"
#include "device_util.hpp"

namespace pts {

// Patch (a, b) of offset o: rows {2b+o, 2b+o+1} clipped to [0, H), columns
// {2a+o, 2a+o+1} mod W.  For o = 1, b runs from -1 (the 1-row patch of row 0).
// PK: the exemplar's RGB comes from its 8-bit form pk (channel value / 255,
// the rounded product the RGBS image holds), 4 bytes a pixel instead of 16.
template <bool PK>
__global__ __launch_bounds__(256) void k_mstep_patch2x2(const int32_t* __restrict__ nn,
                                                        const float* __restrict__ dist, float4* __restrict__ x,
                                                        int H, int W, int w, int s, const float4* __restrict__ ex,
                                                        const uint32_t* __restrict__ pk, int Hz, int Wz, float r,
                                                        float delta, int o, int npx, int npy,
                                                        const float* __restrict__ wscale) {
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= (int64_t)npx * npy) return;
  const int a = (int)(t % npx);
  const int b = (int)(t / npx) - o;
  const int py0 = 2 * b + o;
  const int lo = max(py0, 0), hi = min(py0 + 1, H - 1);
  const int c0 = (2 * a + o) % W;
  const int c1 = (c0 + 1 == W) ? 0 : c0 + 1;
  const int cols = W / s;
  const int nu = Wz - w + 1;
  const int64_t N = (int64_t)(Hz - w + 1) * nu;

  // covering window rows: v = i*s with hi - w + 1 <= v <= lo and 0 <= v <= H - w
  int vmin = max(hi - w + 1, 0);
  vmin = ((vmin + s - 1) / s) * s;
  const int vmax = min(lo, H - w);

  float acc[2][2][3];
#pragma unroll
  for (int yy = 0; yy < 2; ++yy)
#pragma unroll
    for (int xx = 0; xx < 2; ++xx) acc[yy][xx][0] = acc[yy][xx][1] = acc[yy][xx][2] = 0.f;
  float wsum = 0.f;
  const int nrow = hi - lo + 1;

  for (int v = vmin; v <= vmax; v += s) {
    const int i = v / s;
    // covering columns: u = c0 - t (mod W), t = 0 .. w-2, u a multiple of s
    for (int tt = 0; tt <= w - 2; ++tt) {
      int u = c0 - tt;
      if (((u % s) + s) % s != 0) continue;
      if (u < 0) u += W;
      const int64_t q = (int64_t)i * cols + u / s;
      const int e = nn[q];
      if (e < 0 || e >= N) continue;
      const float Wq = powf(fmaxf(dist[q], delta), r - 2.0f) * (wscale ? wscale[q] : 1.0f);
      const int ey = e / nu, exx = e - ey * nu;
      wsum += Wq;
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        if (yy >= nrow) break;
        const int oy = lo + yy - v;
        const int64_t rb = (int64_t)(ey + oy) * Wz + exx;
        float4 z0, z1;  // pixel c0: offset (c0 - u) mod W = tt; pixel c1: offset tt + 1
        if constexpr (PK) {
#pragma clang fp contract(off)
          const float i255 = 1.0f / 255.0f;
          const uint32_t p0 = pk[rb + tt], p1 = pk[rb + tt + 1];
          z0.x = (float)(p0 & 255u) * i255;
          z0.y = (float)((p0 >> 8) & 255u) * i255;
          z0.z = (float)((p0 >> 16) & 255u) * i255;
          z1.x = (float)(p1 & 255u) * i255;
          z1.y = (float)((p1 >> 8) & 255u) * i255;
          z1.z = (float)((p1 >> 16) & 255u) * i255;
        } else {
          z0 = ex[rb + tt];
          z1 = ex[rb + tt + 1];
        }
        acc[yy][0][0] = fmaf(Wq, z0.x, acc[yy][0][0]);
        acc[yy][0][1] = fmaf(Wq, z0.y, acc[yy][0][1]);
        acc[yy][0][2] = fmaf(Wq, z0.z, acc[yy][0][2]);
        acc[yy][1][0] = fmaf(Wq, z1.x, acc[yy][1][0]);
        acc[yy][1][1] = fmaf(Wq, z1.y, acc[yy][1][1]);
        acc[yy][1][2] = fmaf(Wq, z1.z, acc[yy][1][2]);
      }
    }
  }
  if (wsum > 0.f) {
    const float inv = 1.0f / wsum;
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) {
      if (yy >= nrow) break;
      const int64_t rowb = (int64_t)(lo + yy) * W;
      float4 p0 = x[rowb + c0];
      p0.x = acc[yy][0][0] * inv;
      p0.y = acc[yy][0][1] * inv;
      p0.z = acc[yy][0][2] * inv;
      x[rowb + c0] = p0;
      float4 p1 = x[rowb + c1];
      p1.x = acc[yy][1][0] * inv;
      p1.y = acc[yy][1][1] * inv;
      p1.z = acc[yy][1][2] * inv;
      x[rowb + c1] = p1;
    }
  }
}

void launch_mstep(Ctx* c, const int32_t* nn, const float* dist, float* x, int H, int W, int w, int s,
                  const float* ex, const uint32_t* ex_pk, int Hz, int Wz, float r, float delta, int o,
                  const float* wscale) {
  ProfScope ps(c, "mstep_patch2x2");
  PTS_REQUIRE(o == 0 || o == 1, PTS_ERR_ARG, "patch_offset must be 0 or 1");
  const int npx = W / 2;
  const int npy = H / 2 + o;
  const int64_t n = (int64_t)npx * npy;
  if (n == 0) return;
  const dim3 grid((unsigned)ceil_div(n, 256));
  if (ex_pk)
    hipLaunchKernelGGL(k_mstep_patch2x2<true>, grid, dim3(256), 0, c->stream, nn, dist, reinterpret_cast<float4*>(x),
                       H, W, w, s, reinterpret_cast<const float4*>(ex), ex_pk, Hz, Wz, r, delta, o, npx, npy, wscale);
  else
    hipLaunchKernelGGL(k_mstep_patch2x2<false>, grid, dim3(256), 0, c->stream, nn, dist, reinterpret_cast<float4*>(x),
                       H, W, w, s, reinterpret_cast<const float4*>(ex), ex_pk, Hz, Wz, r, delta, o, npx, npy, wscale);
  check_launch("k_mstep_patch2x2");
}

// ---------------------------------------------------------------------------
// energy: per-thread Kahan sums over a grid-stride range, fixed-order tree in
// LDS, then one block folds the block partials the same way.  The grid size
// depends only on n, so the result is bitwise reproducible.

__device__ __forceinline__ void kahan_add(float& s, float& comp, float v) {
  const float y = v - comp;
  const float t = s + y;
  comp = (t - s) - y;
  s = t;
}

__device__ __forceinline__ void block_sum2(float& a, float& b, float* sa, float* sb) {
  const int tid = threadIdx.x;
  sa[tid] = a;
  sb[tid] = b;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) {
      sa[tid] += sa[tid + off];
      sb[tid] += sb[tid + off];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
}

__global__ __launch_bounds__(256) void k_energy_partial(const float* __restrict__ d, int64_t n, float r,
                                                        float delta, float c0, float c1, float* __restrict__ part) {
  __shared__ float sa[256], sb[256];
  float e = 0.f, ec = 0.f, e2 = 0.f, e2c = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = d[i];
    const float rv = (v >= delta) ? powf(v, r) : fmaf(c1, v * v, c0);
    kahan_add(e, ec, rv);
    kahan_add(e2, e2c, v * v);
  }
  block_sum2(e, e2, sa, sb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = e;
    part[2 * blockIdx.x + 1] = e2;
  }
}

__global__ __launch_bounds__(256) void k_energy_final(const float* __restrict__ part, int nb, float* __restrict__ out) {
  __shared__ float sa[256], sb[256];
  float e = 0.f, ec = 0.f, e2 = 0.f, e2c = 0.f;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    kahan_add(e, ec, part[2 * i]);
    kahan_add(e2, e2c, part[2 * i + 1]);
  }
  block_sum2(e, e2, sa, sb);
  if (threadIdx.x == 0) {
    out[0] = e;
    out[1] = e2;
  }
}

// The energy entry point that allocates nothing keeps its per-block
// partial sums (E, E2) in this array: one copy per device, at its own
// address, held until the process ends.  In host code the name is a
// host-side stand-in, never the device address: kernels get the pointer
// that energy_scratch_init returned for the device.
constexpr int ENERGY_MAX_BLOCKS = 1024;
static __device__ __align__(256) float scratch[2 * ENERGY_MAX_BLOCKS];

float* energy_scratch_init(int device) {
  static std::mutex mu;
  static std::map<int, float*> ptrs;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = ptrs.find(device);
  if (it != ptrs.end()) return it->second;
  int cur = -1;
  PTS_HIP(hipGetDevice(&cur));
  PTS_REQUIRE(cur == device, PTS_ERR_STATE, "energy scratch: the device must be current");
  void* p = nullptr;
  PTS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  PTS_REQUIRE(p != nullptr, PTS_ERR_HIP, "energy scratch: no device address");
  ptrs[device] = static_cast<float*>(p);
  return static_cast<float*>(p);
}

// part: 2 x (at most ENERGY_MAX_BLOCKS) floats, each written before it is read
static void energy_into(Ctx* c, const float* dist, int64_t n, float r, float delta, float* out2, float* part,
                        int nb) {
  const double dr = r, dd = delta;
  const float c0 = (float)((1.0 - dr / 2.0) * std::pow(dd, dr));
  const float c1 = (float)((dr / 2.0) * std::pow(dd, dr - 2.0));
  hipLaunchKernelGGL(k_energy_partial, dim3(nb), dim3(256), 0, c->stream, dist, n, r, delta, c0, c1, part);
  check_launch("k_energy_partial");
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, c->stream, part, nb, out2);
  check_launch("k_energy_final");
}

static int energy_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(ENERGY_MAX_BLOCKS, ceil_div(n, 256)));
}

void launch_energy(Ctx* c, const float* dist, int64_t n, float r, float delta, float* out2) {
  ProfScope ps(c, "energy");
  const int nb = energy_blocks(n);
  energy_into(c, dist, n, r, delta, out2, c->buf<float>("energy_part", 2 * (size_t)nb), nb);
}

void launch_energy_scratch(Ctx* c, const float* dist, int64_t n, float r, float delta, float* out2,
                           float* scratch_ptr) {
  // no profiling scope: its events would be created here
  PTS_REQUIRE(scratch_ptr != nullptr, PTS_ERR_STATE, "energy scratch: not set up on this device");
  energy_into(c, dist, n, r, delta, out2, scratch_ptr, energy_blocks(n));
}

}  // namespace pts
