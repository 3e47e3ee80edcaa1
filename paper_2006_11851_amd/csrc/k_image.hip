// Image kernels: RGBS assembly, guidance channel, exemplar pyramid level,
// 2x bilinear upsampling.  One thread per output pixel, float4 per pixel.
//
// Guidance: Section 4 of the paper takes the perspective scale map as a
// fourth channel; with zero tilt its Eq. 3 is affine in the row, so the
// channel here is S = weight * (y + 0.5) / H of the image's own height.
// Coarse-to-fine (Methodology 2.1): a coarse result is upsampled by
// interpolation to start the next resolution.
#include "kernels.hpp"

namespace pts {

__global__ __launch_bounds__(256) void k_rgbs_from_u8(const uint8_t* __restrict__ u8, int H, int W, float gw,
                                                      float4* __restrict__ out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  int y = (int)(p / W);
  const float inv = 1.0f / 255.0f;
  float4 v;
  v.x = (float)u8[3 * p + 0] * inv;
  v.y = (float)u8[3 * p + 1] * inv;
  v.z = (float)u8[3 * p + 2] * inv;
  v.w = gw * ((float)y + 0.5f) / (float)H;
  out[p] = v;
}

__global__ __launch_bounds__(256) void k_fill_guidance(float4* __restrict__ x, int H, int W, float gw) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  int y = (int)(p / W);
  x[p].w = gw * ((float)y + 0.5f) / (float)H;
}

__device__ __forceinline__ int mirror(int i, int n) {
  // mirrored border without repeating the edge sample: -1 -> 1, n -> n - 2
  if (i < 0) i = -i;
  if (i >= n) i = 2 * (n - 1) - i;
  return i;
}

// [1 4 6 4 1] / 16 separable blur evaluated at the even samples (2xo, 2yo):
// rows first, then columns, as a 5x5 tensor-product sum.  gw >= 0: the
// guidance is recomputed at the coarse size; gw < 0: the image's own
// guidance channel (a scale map) is blurred like the colours.
__global__ __launch_bounds__(256) void k_blur_decimate(const float4* __restrict__ in, int H, int W, float gw,
                                                       float4* __restrict__ out) {
  const int Ho = H / 2, Wo = W / 2;
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)Ho * Wo) return;
  const int yo = (int)(p / Wo), xo = (int)(p % Wo);
  const float k5[5] = {1.f / 16, 4.f / 16, 6.f / 16, 4.f / 16, 1.f / 16};
  float r = 0.f, g = 0.f, b = 0.f, sg = 0.f;
  for (int kx = 0; kx < 5; ++kx) {
    const int xx = mirror(2 * xo + kx - 2, W);
    float cr = 0.f, cg = 0.f, cb = 0.f, cs = 0.f;
    for (int ky = 0; ky < 5; ++ky) {
      const int yy = mirror(2 * yo + ky - 2, H);
      const float4 v = in[(int64_t)yy * W + xx];
      cr = fmaf(k5[ky], v.x, cr);
      cg = fmaf(k5[ky], v.y, cg);
      cb = fmaf(k5[ky], v.z, cb);
      cs = fmaf(k5[ky], v.w, cs);
    }
    r = fmaf(k5[kx], cr, r);
    g = fmaf(k5[kx], cg, g);
    b = fmaf(k5[kx], cb, b);
    sg = fmaf(k5[kx], cs, sg);
  }
  out[p] = make_float4(r, g, b, gw < 0.f ? sg : gw * ((float)yo + 0.5f) / (float)Ho);
}

// Bilinear at coarse position ((x + 0.5) / 2 - 0.5, (y + 0.5) / 2 - 0.5),
// x wraps, y clamps; guidance recomputed at the fine size (gw >= 0) or
// interpolated like the colours (gw < 0: the image's own scale map).
__global__ __launch_bounds__(256) void k_upsample2(const float4* __restrict__ in, int Hc, int Wc, float gw,
                                                   float4* __restrict__ out) {
  const int H = 2 * Hc, W = 2 * Wc;
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int y = (int)(p / W), x = (int)(p % W);
  const float yc = ((float)y + 0.5f) * 0.5f - 0.5f;
  const float xc = ((float)x + 0.5f) * 0.5f - 0.5f;
  const int y0 = (int)floorf(yc), x0 = (int)floorf(xc);
  const float fy = yc - (float)y0, fx = xc - (float)x0;
  const int ya = min(max(y0, 0), Hc - 1), yb = min(max(y0 + 1, 0), Hc - 1);
  const int xa = (x0 % Wc + Wc) % Wc, xb = ((x0 + 1) % Wc + Wc) % Wc;
  const float4 a = in[(int64_t)ya * Wc + xa], b = in[(int64_t)ya * Wc + xb];
  const float4 c = in[(int64_t)yb * Wc + xa], d = in[(int64_t)yb * Wc + xb];
  float4 o;
  o.x = (1.f - fy) * ((1.f - fx) * a.x + fx * b.x) + fy * ((1.f - fx) * c.x + fx * d.x);
  o.y = (1.f - fy) * ((1.f - fx) * a.y + fx * b.y) + fy * ((1.f - fx) * c.y + fx * d.y);
  o.z = (1.f - fy) * ((1.f - fx) * a.z + fx * b.z) + fy * ((1.f - fx) * c.z + fx * d.z);
  o.w = gw < 0.f ? (1.f - fy) * ((1.f - fx) * a.w + fx * b.w) + fy * ((1.f - fx) * c.w + fx * d.w)
                 : gw * ((float)y + 0.5f) / (float)H;
  out[p] = o;
}

__global__ __launch_bounds__(256) void k_pack_exemplar(const uint8_t* __restrict__ u8, int H, int W,
                                                       const float4* __restrict__ img, uint32_t* __restrict__ pk,
                                                       float* __restrict__ srow) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  pk[p] = (uint32_t)u8[3 * p] | ((uint32_t)u8[3 * p + 1] << 8) | ((uint32_t)u8[3 * p + 2] << 16);
  const int y = (int)(p / W);
  if (p - (int64_t)y * W == 0) srow[y] = img[p].w;
}

// cnt[0] += the number of values of x [n] that are not finite
__global__ __launch_bounds__(256) void k_count_nonfinite(const float* __restrict__ x, int64_t n, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool bad = i < n && !isfinite(x[i]);
  const uint64_t m = __ballot(bad);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(cnt, (int)__popcll(m));
}

static unsigned blocks_for(int64_t n, int per) { return (unsigned)ceil_div(n, per); }

int64_t count_nonfinite(Ctx* c, const float* x, int64_t n) {
  if (n == 0) return 0;
  int* d = c->buf<int>("nonfinite_count", 1);
  launch_zero_i32(c, d, 1);
  hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, x, n, d);
  check_launch("k_count_nonfinite");
  int h = 0;
  PTS_HIP(hipMemcpyAsync(&h, d, 4, hipMemcpyDeviceToHost, c->stream));
  PTS_HIP(hipStreamSynchronize(c->stream));
  return h;
}

void launch_pack_exemplar(Ctx* c, const uint8_t* u8, int H, int W, const float* img, uint32_t* pk, float* srow) {
  ProfScope ps(c, "pack_exemplar");
  int64_t n = (int64_t)H * W;
  if (n == 0) return;
  hipLaunchKernelGGL(k_pack_exemplar, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, u8, H, W,
                     reinterpret_cast<const float4*>(img), pk, srow);
  check_launch("k_pack_exemplar");
}

void launch_rgbs_from_u8(Ctx* c, const uint8_t* u8, int H, int W, float gw, float* out) {
  ProfScope ps(c, "rgbs_from_u8");
  int64_t n = (int64_t)H * W;
  if (n == 0) return;
  hipLaunchKernelGGL(k_rgbs_from_u8, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, u8, H, W, gw,
                     reinterpret_cast<float4*>(out));
  check_launch("k_rgbs_from_u8");
}

void launch_fill_guidance(Ctx* c, float* x, int H, int W, float gw) {
  ProfScope ps(c, "fill_guidance");
  int64_t n = (int64_t)H * W;
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_guidance, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                     reinterpret_cast<float4*>(x), H, W, gw);
  check_launch("k_fill_guidance");
}

void launch_blur_decimate(Ctx* c, const float* in, int H, int W, float gw, float* out) {
  ProfScope ps(c, "blur_decimate");
  PTS_REQUIRE(H >= 4 && W >= 4 && H % 2 == 0 && W % 2 == 0, PTS_ERR_ARG, "pyramid level needs even sides >= 4");
  int64_t n = (int64_t)(H / 2) * (W / 2);
  hipLaunchKernelGGL(k_blur_decimate, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                     reinterpret_cast<const float4*>(in), H, W, gw, reinterpret_cast<float4*>(out));
  check_launch("k_blur_decimate");
}

void launch_upsample2(Ctx* c, const float* in, int H, int W, float gw, float* out) {
  ProfScope ps(c, "upsample2");
  int64_t n = (int64_t)(2 * H) * (2 * W);
  if (n == 0) return;
  hipLaunchKernelGGL(k_upsample2, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                     reinterpret_cast<const float4*>(in), H, W, gw, reinterpret_cast<float4*>(out));
  check_launch("k_upsample2");
}

}  // namespace pts
