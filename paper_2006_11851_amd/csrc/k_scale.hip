// Perspective scale map (Methodology 1, Eqs. 1-3) as the guidance channel,
// and the scale-matched initial output (Section 4, steps 1-3).
//
// The map of an exemplar of ref_h x ref_w pixels under slant sigma and tilt
// tau (origin at the bottom-left corner, so the paper's y is
// ref_h - 1 - row):
//   S_max = 1 / cos sigma, S_min = cos sigma, S_D = S_max - S_min     (Eq. 1)
//   Y_max = (ref_w - 1 - ref_w/2) sin tau + (ref_h - 1 - ref_h/2) cos tau,
//   Y_min = -Y_max                                                    (Eq. 2)
//   p(Y) = (x - ref_w/2) sin tau + (y - ref_h/2) cos tau,
//   S = S_max - (p(Y) - Y_min) S_D / (Y_max - Y_min)                  (Eq. 3)
// with Eq. 3's leading term read as S_max (S then runs from S_max at Y_min
// to S_min at Y_max).  The channel written is gw (S - S_min) / S_D (zero
// when sigma = 0 makes the map flat).  An image of another size H x W takes
// the map resampled bilinearly (pixel centres aligned, coordinates clamped
// to the edge pixels); since the map is affine that is Eq. 3 evaluated at
// the clamped source coordinate, which is what the kernels compute, in
// FP64, once per pixel.
//
// Step 3 (equal scale = equal p(Y)): each t x t output tile takes the
// exemplar window whose centre lies nearest the line of constant p(Y)
// through the exemplar point its own centre samples, at a column (or, for
// lines closer to vertical, a row) drawn by the caller.  The corner is a
// rounding decision in FP64 with contraction off, the same arithmetic in
// the same order on every device.
#include <cmath>

#include "kernels.hpp"

namespace pts {

ScaleGeom scale_geom(double slant, double tilt, int ref_h, int ref_w) {
  PTS_REQUIRE(std::isfinite(slant) && std::isfinite(tilt) && slant >= 0.0 && slant < M_PI / 2 && tilt >= 0.0 &&
                  tilt <= M_PI / 2,
              PTS_ERR_ARG, "scale map: slant must be in [0, pi/2), tilt in [0, pi/2]");
  PTS_REQUIRE(ref_h >= 3 && ref_w >= 3, PTS_ERR_ARG, "scale map: the image needs at least 3 x 3 pixels");
  ScaleGeom g;
  g.smax = 1.0 / std::cos(slant);
  g.smin = std::cos(slant);
  g.sd = g.smax - g.smin;
  g.sin_t = std::sin(tilt);
  g.cos_t = std::cos(tilt);
  g.ymax = (ref_w - 1 - ref_w / 2.0) * g.sin_t + (ref_h - 1 - ref_h / 2.0) * g.cos_t;
  g.ref_h = ref_h;
  g.ref_w = ref_w;
  return g;
}

// the normalised map at output pixel (r, col) of an H x W image
__device__ double scale_norm(const ScaleGeom& g, int r, int col, int H, int W) {
  if (g.sd == 0.0) return 0.0;
  const double v = fmin(fmax((r + 0.5) * g.ref_h / H - 0.5, 0.0), g.ref_h - 1.0);
  const double u = fmin(fmax((col + 0.5) * g.ref_w / W - 0.5, 0.0), g.ref_w - 1.0);
  const double pY = (u - g.ref_w / 2.0) * g.sin_t + ((g.ref_h - 1.0 - v) - g.ref_h / 2.0) * g.cos_t;
  const double S = g.smax - (pY + g.ymax) * g.sd / (2.0 * g.ymax);
  return (S - g.smin) / g.sd;
}

__global__ __launch_bounds__(256) void k_scale_guidance(float4* __restrict__ x, int H, int W, ScaleGeom g, float gw) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int r = (int)(p / W), col = (int)(p - (int64_t)r * W);
  x[p].w = (float)(gw * scale_norm(g, r, col, H, W));
}

// corner (u, v) of the exemplar window for tile (ti, tj)
__device__ int2 matched_corner(const ScaleGeom& g, int ti, int tj, int t, int H, int W, uint32_t ru32,
                               uint32_t rv32) {
#pragma clang fp contract(off)
  const int h = g.ref_h, w = g.ref_w;
  const int nu = w - t + 1, nv = h - t + 1;
  const int ru = (int)(ru32 % (uint32_t)nu), rv = (int)(rv32 % (uint32_t)nv);
  if (g.sd == 0.0) return make_int2(ru, rv);
  const double Vc = fmin(fmax(((double)(ti * t) + t / 2.0 + 0.5) * h / H - 0.5, 0.0), h - 1.0);
  const double Uc = fmin(fmax(((double)(tj * t) + t / 2.0 + 0.5) * w / W - 0.5, 0.0), w - 1.0);
  if (g.cos_t >= g.sin_t) {
    const double row = Vc + (((double)ru + t / 2.0) - Uc) * g.sin_t / g.cos_t;
    const int v = (int)floor((row - t / 2.0) + 0.5);
    return make_int2(ru, min(max(v, 0), nv - 1));
  }
  const double colp = Uc + (((double)rv + t / 2.0) - Vc) * g.cos_t / g.sin_t;
  const int u = (int)floor((colp - t / 2.0) + 0.5);
  return make_int2(min(max(u, 0), nu - 1), rv);
}

__global__ __launch_bounds__(256) void k_scale_init(const float4* __restrict__ ex, int Wz, float4* __restrict__ x,
                                                    int H, int W, int t, const uint32_t* __restrict__ rnd,
                                                    ScaleGeom g, float gw) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int r = (int)(p / W), col = (int)(p - (int64_t)r * W);
  const int ti = r / t, tj = col / t, ntx = (W + t - 1) / t;
  const int64_t k = (int64_t)ti * ntx + tj;
  const int2 uv = matched_corner(g, ti, tj, t, H, W, rnd[2 * k], rnd[2 * k + 1]);
  const float4 e = ex[(int64_t)(uv.y + r - ti * t) * Wz + uv.x + col - tj * t];
  x[p] = make_float4(e.x, e.y, e.z, (float)(gw * scale_norm(g, r, col, H, W)));
}

static unsigned blocks_for(int64_t n, int per) { return (unsigned)ceil_div(n, per); }

void launch_scale_guidance(Ctx* c, float* x, int H, int W, const ScaleGeom& g, float gw) {
  ProfScope ps(c, "scale_guidance");
  const int64_t n = (int64_t)H * W;
  if (n == 0) return;
  hipLaunchKernelGGL(k_scale_guidance, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                     reinterpret_cast<float4*>(x), H, W, g, gw);
  check_launch("k_scale_guidance");
}

void launch_scale_init(Ctx* c, const float* ex, int Hz, int Wz, float* x, int H, int W, int t, const uint32_t* rnd,
                       const ScaleGeom& g, float gw) {
  ProfScope ps(c, "scale_init");
  PTS_REQUIRE(g.ref_h == Hz && g.ref_w == Wz, PTS_ERR_ARG, "scale init: map and exemplar sizes differ");
  PTS_REQUIRE(t >= 1 && t <= Hz && t <= Wz, PTS_ERR_ARG, "scale init: tile side must be in 1..min(Hz, Wz)");
  const int64_t n = (int64_t)H * W;
  if (n == 0) return;
  hipLaunchKernelGGL(k_scale_init, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                     reinterpret_cast<const float4*>(ex), Wz, reinterpret_cast<float4*>(x), H, W, t, rnd, g, gw);
  check_launch("k_scale_init");
}

}  // namespace pts
