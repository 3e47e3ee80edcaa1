// Index-build kernels (Methodology 2.2: PCA before the k-means search tree).
//
//  * mean and covariance of all exemplar windows, gathered straight from the
//    exemplar image, accumulated in FP64 (the covariance feeds the FP64
//    eigensolve; centred products avoid the cancellation of E[zz^T]-mu mu^T);
//  * projection of windows onto the basis, P = (x - mu) B, FP32 on the
//    matrix cores, gathered
//    from an image on either window grid (exemplar: all corners; output:
//    stride s with the x wrap) - used for the index and for every query;
//  * k-means helpers: nearest-centre assignment (ties to the lowest centre),
//    centroid sums in 2^-30 fixed point with 64-bit integer atomics (integer
//    addition is associative, so the centroids are bitwise reproducible),
//    running minimum distance for k-means++ seeding.
#include <algorithm>
#include <climits>

#include "kernels.hpp"
#include "device_util.hpp"

namespace pts {

struct WinGeom {
  const float4* img;
  int W;      // image width (pixels)
  int w;      // window width
  int s;      // grid stride
  int cols;   // windows per grid row
  int wrap;   // 1: columns wrap modulo W
};

__device__ __forceinline__ float4 win_pixel(const WinGeom& g, int64_t win, int pix) {
  const int i = (int)(win / g.cols), j = (int)(win - (int64_t)i * g.cols);
  const int dy = pix / g.w, dx = pix - dy * g.w;
  int x = j * g.s + dx;
  if (g.wrap && x >= g.W) x -= g.W;
  return g.img[(int64_t)(i * g.s + dy) * g.W + x];
}

static WinGeom geom(const float* img, int H, int W, int w, int s, bool wrap) {
  WinGeom g;
  g.img = reinterpret_cast<const float4*>(img);
  g.W = W;
  g.w = w;
  g.s = s;
  g.cols = wrap ? W / s : (W - w) / s + 1;
  g.wrap = wrap ? 1 : 0;
  (void)H;
  return g;
}

// ---------------------------------------------------------------------------
// mean: partial column sums over a split of the windows, FP64

__global__ __launch_bounds__(256) void k_mean_partial(WinGeom g, int64_t N, int D, int64_t per_split,
                                                      double* __restrict__ part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D) return;
  const int64_t e0 = (int64_t)blockIdx.y * per_split;
  const int64_t e1 = min(N, e0 + per_split);
  const int pix = j >> 2, ch = j & 3;
  double acc = 0.0;
  for (int64_t e = e0; e < e1; ++e) {
    const float4 p = win_pixel(g, e, pix);
    acc += (double)(ch == 0 ? p.x : ch == 1 ? p.y : ch == 2 ? p.z : p.w);
  }
  part[(int64_t)blockIdx.y * D + j] = acc;
}

__global__ __launch_bounds__(256) void k_reduce_splits(const double* __restrict__ part, int64_t len, int splits,
                                                       double scale, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  double a = 0.0;
  for (int s = 0; s < splits; ++s) a += part[(int64_t)s * len + j];
  out[j] = a * scale;
}

// covariance tile (bi <= bj) of 64 x 64 over a split of windows; 256
// threads, each 4 x 4 outputs; windows streamed 16 at a time through LDS.
constexpr int CV_T = 64, CV_E = 16;

__global__ __launch_bounds__(256) void k_cov_partial(WinGeom g, int64_t N, int D, const double* __restrict__ mu,
                                                     const int2* __restrict__ tiles, int64_t per_split,
                                                     double* __restrict__ part) {
  __shared__ double As[CV_E][CV_T + 1];
  __shared__ double Bs[CV_E][CV_T + 1];
  const int2 tile = tiles[blockIdx.x];
  const int i0 = tile.x * CV_T, j0 = tile.y * CV_T;
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  const int64_t e0 = (int64_t)blockIdx.y * per_split;
  const int64_t e1 = min(N, e0 + per_split);
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t eb = e0; eb < e1; eb += CV_E) {
    // 16 windows x 64 elements for each of the two blocks: 16 x 16 pixels
    {
      const int r = tid >> 4;     // window within chunk
      const int pp = tid & 15;    // pixel within the 64-element block
      const int64_t e = eb + r;
      double4 va = make_double4(0, 0, 0, 0), vb = make_double4(0, 0, 0, 0);
      if (e < e1) {
        const int ja = i0 + 4 * pp, jb = j0 + 4 * pp;
        if (ja < D) {
          const float4 p = win_pixel(g, e, ja >> 2);
          va = make_double4((double)p.x - mu[ja], (double)p.y - mu[ja + 1], (double)p.z - mu[ja + 2],
                            (double)p.w - mu[ja + 3]);
        }
        if (jb < D) {
          const float4 p = win_pixel(g, e, jb >> 2);
          vb = make_double4((double)p.x - mu[jb], (double)p.y - mu[jb + 1], (double)p.z - mu[jb + 2],
                            (double)p.w - mu[jb + 3]);
        }
      }
      As[r][4 * pp + 0] = va.x;
      As[r][4 * pp + 1] = va.y;
      As[r][4 * pp + 2] = va.z;
      As[r][4 * pp + 3] = va.w;
      Bs[r][4 * pp + 0] = vb.x;
      Bs[r][4 * pp + 1] = vb.y;
      Bs[r][4 * pp + 2] = vb.z;
      Bs[r][4 * pp + 3] = vb.w;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < CV_E; ++r) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[r][ti + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[r][tj + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (CV_T * CV_T);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) out[(ti + 16 * a) * CV_T + (tj + 16 * b)] = acc[a][b];
}

__global__ __launch_bounds__(256) void k_cov_reduce(const double* __restrict__ part, const int2* __restrict__ tiles,
                                                    int ntiles, int splits, int D, double scale,
                                                    double* __restrict__ cov) {
  const int t = blockIdx.x;
  const int2 tile = tiles[t];
  for (int k = threadIdx.x; k < CV_T * CV_T; k += blockDim.x) {
    double a = 0.0;
    for (int s = 0; s < splits; ++s) a += part[((int64_t)s * ntiles + t) * (CV_T * CV_T) + k];
    const int i = tile.x * CV_T + k / CV_T, j = tile.y * CV_T + k % CV_T;
    if (i < D && j < D) {
      cov[(int64_t)i * D + j] = a * scale;
      cov[(int64_t)j * D + i] = a * scale;
    }
  }
}

void launch_mean_cov_image(Ctx* c, const float* img, int H, int W, int w, double* mean, double* cov) {
  ProfScope ps(c, "mean_cov");
  const WinGeom g = geom(img, H, W, w, 1, false);
  const int64_t N = (int64_t)(H - w + 1) * (W - w + 1);
  const int D = 4 * w * w;
  // mean
  {
    const int64_t splits = std::max<int64_t>(1, std::min<int64_t>(ceil_div(N, 256), 1024 / ceil_div(D, 256) + 1));
    const int64_t per = ceil_div(N, splits);
    double* part = c->buf<double>("mean_part", (size_t)(splits * D));
    hipLaunchKernelGGL(k_mean_partial, dim3((unsigned)ceil_div(D, 256), (unsigned)splits), dim3(256), 0, c->stream, g,
                       N, D, per, part);
    check_launch("k_mean_partial");
    hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)ceil_div(D, 256)), dim3(256), 0, c->stream, part, (int64_t)D,
                       (int)splits, 1.0 / (double)N, mean);
    check_launch("k_reduce_splits");
  }
  // covariance, upper block-triangle tiles
  const int nb = (int)ceil_div(D, CV_T);
  std::vector<int2> tiles;
  for (int i = 0; i < nb; ++i)
    for (int j = i; j < nb; ++j) tiles.push_back(make_int2(i, j));
  const int nt = (int)tiles.size();
  int2* dtiles = c->buf<int2>("cov_tiles", tiles.size());
  PTS_HIP(hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, c->stream));
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(ceil_div(2048, nt), ceil_div(N, 4 * CV_E)));
  // bound the partial buffer to ~512 MB
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, ((int64_t)512 << 20) / ((int64_t)nt * CV_T * CV_T * 8)));
  const int64_t per = round_up(ceil_div(N, splits), CV_E);
  splits = ceil_div(N, per);
  double* part = c->buf<double>("cov_part", (size_t)(splits * nt * CV_T * CV_T));
  hipLaunchKernelGGL(k_cov_partial, dim3(nt, (unsigned)splits), dim3(256), 0, c->stream, g, N, D, mean, dtiles, per,
                     part);
  check_launch("k_cov_partial");
  hipLaunchKernelGGL(k_cov_reduce, dim3(nt), dim3(256), 0, c->stream, part, dtiles, nt, (int)splits, D,
                     1.0 / (double)N, cov);
  check_launch("k_cov_reduce");
}

// ---------------------------------------------------------------------------
// projection P[win][k] = sum_j (x_win[j] - mu[j]) B[j][k], FP32, on the
// matrix cores (v_mfma_f32_16x16x4_f32: FP32 operands, FP32 accumulation).
// One MFMA step covers one pixel of the window (its 4 channels are the 4
// k-slices of the instruction): A = 16 basis columns of those 4 rows (from
// LDS), B = that pixel of 16 windows (read straight from the image: windows
// overlap, so the reads hit in cache).  The output tile is 16 basis columns
// x 16 windows; lane l holds window l % 16, columns 4 (l / 16) + 0..3.
// Each wave owns 2 tiles of 16 windows; the basis goes through LDS in
// chunks of 16 pixels (64 rows), shared by the 4 waves of the block.

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int PM_WT = 2;              // 16-window tiles per wave
constexpr int PM_WPB = 4 * 16 * PM_WT;  // windows per block (4 waves)
constexpr int PM_CP = 16;             // pixels per basis chunk

template <int NKT>
__global__ __launch_bounds__(256) void k_project_mfma(WinGeom g, int64_t n, int D, const float* __restrict__ mu,
                                                      const float* __restrict__ B, int dp, float* __restrict__ P,
                                                      uint16_t* __restrict__ Qb, int dk) {
  constexpr int DPAD = 16 * NKT;
  constexpr int LS = DPAD + ((DPAD % 32 == 0) ? 16 : 0);  // row stride: the two half-waves hit disjoint banks
  __shared__ float Bs[PM_CP * 4][LS];
  __shared__ float mus[PM_CP * 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const float* img = reinterpret_cast<const float*>(g.img);
  int64_t win[PM_WT];
  int vrow[PM_WT], ucol[PM_WT];
  bool ok[PM_WT];
#pragma unroll
  for (int wt = 0; wt < PM_WT; ++wt) {
    win[wt] = (int64_t)xcd_block(blockIdx.x, gridDim.x) * PM_WPB + wave * (16 * PM_WT) + wt * 16 + col;
    ok[wt] = win[wt] < n;
    const int64_t wc = ok[wt] ? win[wt] : 0;
    const int i = (int)(wc / g.cols), j = (int)(wc - (int64_t)i * g.cols);
    vrow[wt] = i * g.s;
    ucol[wt] = j * g.s;
  }
  floatx4 acc[PM_WT][NKT];
#pragma unroll
  for (int wt = 0; wt < PM_WT; ++wt)
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) acc[wt][kt] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int npx = D / 4;
  for (int p0 = 0; p0 < npx; p0 += PM_CP) {
    __syncthreads();  // the previous chunk has been consumed
    for (int t = tid; t < PM_CP * 4 * DPAD; t += 256) {
      const int r = t / DPAD, k = t - r * DPAD;
      const int d = 4 * p0 + r;
      Bs[r][k] = (d < D && k < dp) ? B[(int64_t)d * dp + k] : 0.f;
    }
    if (tid < PM_CP * 4) mus[tid] = (4 * p0 + tid < D) ? mu[4 * p0 + tid] : 0.f;
    __syncthreads();
    const int pend = min(PM_CP, npx - p0);
    int dy = p0 / g.w, dx = p0 - dy * g.w;
#pragma unroll
    for (int pp = 0; pp < PM_CP; ++pp) {
      if (pp < pend) {  // uniform
        float xv[PM_WT];
        const float m = mus[pp * 4 + kq];
#pragma unroll
        for (int wt = 0; wt < PM_WT; ++wt) {
          int xx = ucol[wt] + dx;
          if (g.wrap && xx >= g.W) xx -= g.W;
          xv[wt] = ok[wt] ? img[((int64_t)(vrow[wt] + dy) * g.W + xx) * 4 + kq] - m : 0.f;
        }
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
          const float a = Bs[pp * 4 + kq][kt * 16 + col];
#pragma unroll
          for (int wt = 0; wt < PM_WT; ++wt)
            acc[wt][kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xv[wt], acc[wt][kt], 0, 0, 0);
        }
        if (++dx == g.w) {
          dx = 0;
          ++dy;
        }
      }
    }
  }
#pragma unroll
  for (int wt = 0; wt < PM_WT; ++wt) {
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      const int k = kt * 16 + 4 * kq;  // dp is a multiple of 8: a group of 4 is all in or all out
      if (ok[wt] && k < dp)
        *reinterpret_cast<float4*>(P + win[wt] * dp + k) =
            make_float4(acc[wt][kt][0], acc[wt][kt][1], acc[wt][kt][2], acc[wt][kt][3]);
    }
    // optional bf16(-2 q') [n][dk] for the matrix-core search (zero past dp)
    if (Qb && ok[wt]) {
#pragma unroll
      for (int kt = 0; kt < 8; ++kt) {
        const int k = kt * 16 + 4 * kq;
        if (k < dk) {
          float v[4] = {0.f, 0.f, 0.f, 0.f};
          if (kt < NKT && k < dp) {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = -2.0f * acc[wt][kt < NKT ? kt : 0][r];
          }
          const __bf16 b0 = (__bf16)v[0], b1 = (__bf16)v[1], b2 = (__bf16)v[2], b3 = (__bf16)v[3];
          uint2 pk;
          pk.x = (uint32_t)__builtin_bit_cast(uint16_t, b0) | ((uint32_t)__builtin_bit_cast(uint16_t, b1) << 16);
          pk.y = (uint32_t)__builtin_bit_cast(uint16_t, b2) | ((uint32_t)__builtin_bit_cast(uint16_t, b3) << 16);
          *reinterpret_cast<uint2*>(Qb + win[wt] * dk + k) = pk;
        }
      }
    }
  }
}

// Resident-basis form for D <= 256 and an even window (w = 2, 4, 6, 8): one
// block of 16 waves per compute unit keeps the whole basis (and mu) in LDS,
// loaded once, and its waves walk over 32-window tiles with no further
// barrier.  The k-steps are regrouped so that every lane loads whole pixels:
// for 4 consecutive pixels of a window, lane (col, kq) reads pixel 4 pp + kq
// of window col as one float4, and 4 matrix products (one per channel c)
// take k-slice kq = that pixel's channel c, against basis rows 4 (4 pp + kq)
// + c.  Same products and FP32 accumulation as k_project_mfma, in another
// order.
constexpr int PR_ROWS = 256;  // basis rows held in LDS
constexpr int PR_WAVES = 16;

template <int NKT>
__global__ __launch_bounds__(PR_WAVES * 64) void k_project_res(WinGeom g, int64_t n, int D,
                                                               const float* __restrict__ mu,
                                                               const float* __restrict__ B, int dp,
                                                               float* __restrict__ P, uint16_t* __restrict__ Qb,
                                                               int dk) {
  constexpr int DPAD = 16 * NKT;
  // row stride = 4 mod 16 (in floats): the four k-rows of a step, 4 rows
  // apart, start 16 banks apart
  constexpr int LS = DPAD + 4;
  __shared__ float Bs[PR_ROWS][LS];
  __shared__ float4 mus4[PR_ROWS / 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  for (int t = tid; t < PR_ROWS * DPAD; t += PR_WAVES * 64) {
    const int r = t / DPAD, k = t - r * DPAD;
    Bs[r][k] = (r < D && k < dp) ? B[(int64_t)r * dp + k] : 0.f;
  }
  if (tid < PR_ROWS / 4) {
    float4 m;
    m.x = 4 * tid < D ? mu[4 * tid] : 0.f;
    m.y = 4 * tid + 1 < D ? mu[4 * tid + 1] : 0.f;
    m.z = 4 * tid + 2 < D ? mu[4 * tid + 2] : 0.f;
    m.w = 4 * tid + 3 < D ? mu[4 * tid + 3] : 0.f;
    mus4[tid] = m;
  }
  __syncthreads();
  const float4* img = g.img;
  const int ngroups = D / 16;  // groups of 4 pixels
  const int64_t ntile = ceil_div(n, (int64_t)(16 * PM_WT));
  for (int64_t tile = (int64_t)blockIdx.x * PR_WAVES + wave; tile < ntile; tile += (int64_t)gridDim.x * PR_WAVES) {
    int64_t win[PM_WT];
    int vrow[PM_WT], ucol[PM_WT];
    bool ok[PM_WT];
#pragma unroll
    for (int wt = 0; wt < PM_WT; ++wt) {
      win[wt] = tile * (16 * PM_WT) + wt * 16 + col;
      ok[wt] = win[wt] < n;
      const int64_t wc = ok[wt] ? win[wt] : 0;
      const int i = (int)(wc / g.cols), j = (int)(wc - (int64_t)i * g.cols);
      vrow[wt] = i * g.s;
      ucol[wt] = j * g.s;
    }
    floatx4 acc[PM_WT][NKT];
#pragma unroll
    for (int wt = 0; wt < PM_WT; ++wt)
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) acc[wt][kt] = floatx4{0.f, 0.f, 0.f, 0.f};
    // the pixels of group pg + 1 are loaded while group pg's products run
    float4 xn[PM_WT];
    auto load_group = [&](int pg) {
      const int px = 4 * pg + kq;  // this lane's pixel of the group
      const int dy = px / g.w, dx = px - dy * g.w;
#pragma unroll
      for (int wt = 0; wt < PM_WT; ++wt) {
        int xx = ucol[wt] + dx;
        if (g.wrap && xx >= g.W) xx -= g.W;
        // windows past the end read the first one's pixel; their results are not stored
        xn[wt] = img[(int64_t)((ok[wt] ? vrow[wt] : 0) + dy) * g.W + (ok[wt] ? xx : dx)];
      }
    };
    load_group(0);
    for (int pg = 0; pg < ngroups; ++pg) {
      const int px = 4 * pg + kq;
      const float4 m = mus4[px];
      float4 xv[PM_WT];
#pragma unroll
      for (int wt = 0; wt < PM_WT; ++wt) {
        const float4 v = xn[wt];
        xv[wt] = make_float4(v.x - m.x, v.y - m.y, v.z - m.z, v.w - m.w);
      }
      if (pg + 1 < ngroups) load_group(pg + 1);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int kt = 0; kt < NKT; ++kt) {
          const float a = Bs[4 * px + c][kt * 16 + col];
#pragma unroll
          for (int wt = 0; wt < PM_WT; ++wt) {
            const float b = c == 0 ? xv[wt].x : c == 1 ? xv[wt].y : c == 2 ? xv[wt].z : xv[wt].w;
            acc[wt][kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[wt][kt], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int wt = 0; wt < PM_WT; ++wt) {
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        const int k = kt * 16 + 4 * kq;
        if (ok[wt] && k < dp)
          *reinterpret_cast<float4*>(P + win[wt] * dp + k) =
              make_float4(acc[wt][kt][0], acc[wt][kt][1], acc[wt][kt][2], acc[wt][kt][3]);
      }
      if (Qb && ok[wt]) {
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) {
          const int k = kt * 16 + 4 * kq;
          if (k < dk) {
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (kt < NKT && k < dp) {
#pragma unroll
              for (int r = 0; r < 4; ++r) v[r] = -2.0f * acc[wt][kt < NKT ? kt : 0][r];
            }
            const __bf16 b0 = (__bf16)v[0], b1 = (__bf16)v[1], b2 = (__bf16)v[2], b3 = (__bf16)v[3];
            uint2 pk;
            pk.x = (uint32_t)__builtin_bit_cast(uint16_t, b0) | ((uint32_t)__builtin_bit_cast(uint16_t, b1) << 16);
            pk.y = (uint32_t)__builtin_bit_cast(uint16_t, b2) | ((uint32_t)__builtin_bit_cast(uint16_t, b3) << 16);
            *reinterpret_cast<uint2*>(Qb + win[wt] * dk + k) = pk;
          }
        }
      }
    }
  }
}

void launch_project_image(Ctx* c, const float* img, int H, int W, int w, int s, bool wrap, const float* mu,
                          const float* B, int dp, float* P, uint16_t* Qb, int dk) {
  ProfScope ps(c, wrap ? "project_queries" : "project_exemplar");
  PTS_REQUIRE(dp >= 8 && dp <= 128 && dp % 8 == 0, PTS_ERR_UNSUPPORTED, "projection: padded width must be 8..128, /8");
  PTS_REQUIRE(!Qb || (dk >= dp && dk <= 128 && dk % 16 == 0), PTS_ERR_UNSUPPORTED, "projection: bad bf16 width");
  const WinGeom g = geom(img, H, W, w, s, wrap);
  const int64_t rows = (H - w) / s + 1;
  const int64_t n = rows * g.cols;
  if (n == 0) return;
  const int D = 4 * w * w;
  if (D <= PR_ROWS && w % 2 == 0) {
    const int64_t ntile = ceil_div(n, (int64_t)(16 * PM_WT));
    const dim3 gr((unsigned)std::min<int64_t>(c->n_cu, ceil_div(ntile, PR_WAVES)));
    switch ((dp + 15) / 16) {
      case 1: hipLaunchKernelGGL(k_project_res<1>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      case 2: hipLaunchKernelGGL(k_project_res<2>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      case 3: hipLaunchKernelGGL(k_project_res<3>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      case 4: hipLaunchKernelGGL(k_project_res<4>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      case 5: hipLaunchKernelGGL(k_project_res<5>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      case 6: hipLaunchKernelGGL(k_project_res<6>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      case 7: hipLaunchKernelGGL(k_project_res<7>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
      default: hipLaunchKernelGGL(k_project_res<8>, gr, dim3(PR_WAVES * 64), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    }
    check_launch("k_project_res");
    return;
  }
  const dim3 grid((unsigned)ceil_div(n, PM_WPB));
  switch ((dp + 15) / 16) {
    case 1: hipLaunchKernelGGL(k_project_mfma<1>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    case 2: hipLaunchKernelGGL(k_project_mfma<2>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    case 3: hipLaunchKernelGGL(k_project_mfma<3>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    case 4: hipLaunchKernelGGL(k_project_mfma<4>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    case 5: hipLaunchKernelGGL(k_project_mfma<5>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    case 6: hipLaunchKernelGGL(k_project_mfma<6>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    case 7: hipLaunchKernelGGL(k_project_mfma<7>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
    default: hipLaunchKernelGGL(k_project_mfma<8>, grid, dim3(256), 0, c->stream, g, n, D, mu, B, dp, P, Qb, dk); break;
  }
  check_launch("k_project_mfma");
}

// ---------------------------------------------------------------------------
// k-means helpers.  Points are rows of P [N][dp] (original exemplar order);
// `members` lists the points of every active segment back to back,
// seg_of[i] is the segment of member i; the k centres of segment s are rows
// seg_cent_off[s] .. seg_cent_off[s] + seg_k[s] - 1 of `cents`.

__device__ __forceinline__ float sqdist_rows(const float* __restrict__ a, const float* __restrict__ b, int dp) {
  float acc = 0.f;
  for (int k = 0; k < dp; k += 4) {
    const float4 x = *reinterpret_cast<const float4*>(a + k);
    const float4 y = *reinterpret_cast<const float4*>(b + k);
    const float t0 = x.x - y.x, t1 = x.y - y.y, t2 = x.z - y.z, t3 = x.w - y.w;
    acc = fmaf(t0, t0, acc);
    acc = fmaf(t1, t1, acc);
    acc = fmaf(t2, t2, acc);
    acc = fmaf(t3, t3, acc);
  }
  return acc;
}

__global__ __launch_bounds__(256) void k_kmeans_mindist(const float* __restrict__ P, int dp,
                                                        const int32_t* __restrict__ members, int64_t m,
                                                        const int32_t* __restrict__ seg_of,
                                                        const float* __restrict__ cand, float* __restrict__ mind,
                                                        int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float d = sqdist_rows(P + (int64_t)members[i] * dp, cand + (int64_t)seg_of[i] * dp, dp);
  mind[i] = first ? d : fminf(mind[i], d);
}

__global__ __launch_bounds__(256) void k_kmeans_assign(const float* __restrict__ P, int dp,
                                                       const int32_t* __restrict__ members, int64_t m,
                                                       const int32_t* __restrict__ seg_of,
                                                       const int32_t* __restrict__ seg_cent_off,
                                                       const int32_t* __restrict__ seg_k,
                                                       const float* __restrict__ cents, int32_t* __restrict__ assign,
                                                       int32_t* __restrict__ changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int s = seg_of[i];
  const int off = seg_cent_off[s], k = seg_k[s];
  const float* p = P + (int64_t)members[i] * dp;
  float best = __int_as_float(0x7f800000);
  int bi = 0;
  for (int c = 0; c < k; ++c) {
    const float d = sqdist_rows(p, cents + (int64_t)(off + c) * dp, dp);
    if (d < best) {
      best = d;
      bi = c;
    }
  }
  if (assign[i] != bi) {
    assign[i] = bi;
    atomicAdd(changed, 1);
  }
}

constexpr double KM_FIX = 1073741824.0;  // 2^30

__global__ __launch_bounds__(256) void k_kmeans_accumulate(const float* __restrict__ P, int dp,
                                                           const int32_t* __restrict__ members, int64_t m,
                                                           const int32_t* __restrict__ seg_of,
                                                           const int32_t* __restrict__ seg_cent_off,
                                                           const int32_t* __restrict__ assign,
                                                           unsigned long long* __restrict__ sums,
                                                           int32_t* __restrict__ counts) {
  // one thread per (member, 4-dimension group)
  const int ng = dp >> 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ng) return;
  const int64_t i = t / ng;
  const int gidx = (int)(t - i * ng);
  const int cidx = seg_cent_off[seg_of[i]] + assign[i];
  const float4 v = *reinterpret_cast<const float4*>(P + (int64_t)members[i] * dp + 4 * gidx);
  unsigned long long* dst = sums + (int64_t)cidx * dp + 4 * gidx;
  atomicAdd(dst + 0, (unsigned long long)(long long)__double2ll_rn((double)v.x * KM_FIX));
  atomicAdd(dst + 1, (unsigned long long)(long long)__double2ll_rn((double)v.y * KM_FIX));
  atomicAdd(dst + 2, (unsigned long long)(long long)__double2ll_rn((double)v.z * KM_FIX));
  atomicAdd(dst + 3, (unsigned long long)(long long)__double2ll_rn((double)v.w * KM_FIX));
  if (gidx == 0) atomicAdd(counts + cidx, 1);
}

// Same sums with block-private LDS accumulators when the centroid table is
// small (ncent * dp <= 4096): every block adds its members into LDS with
// 64-bit LDS atomics and flushes its partial table once, instead of every
// member hitting the few global addresses of the table.
__global__ __launch_bounds__(256) void k_kmeans_accumulate_lds(const float* __restrict__ P, int dp,
                                                               const int32_t* __restrict__ members, int64_t m,
                                                               const int32_t* __restrict__ seg_of,
                                                               const int32_t* __restrict__ seg_cent_off,
                                                               const int32_t* __restrict__ assign, int ncent,
                                                               unsigned long long* __restrict__ sums,
                                                               int32_t* __restrict__ counts) {
  __shared__ unsigned long long s_sum[4096];
  __shared__ int s_cnt[1024];
  const int tab = ncent * dp;
  for (int i = threadIdx.x; i < tab; i += blockDim.x) s_sum[i] = 0ull;
  for (int i = threadIdx.x; i < ncent; i += blockDim.x) s_cnt[i] = 0;
  __syncthreads();
  const int ng = dp >> 2;
  const int64_t per_block = (m * ng + gridDim.x - 1) / gridDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * per_block;
  const int64_t t1 = min(m * ng, t0 + per_block);
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
    const int64_t i = t / ng;
    const int gidx = (int)(t - i * ng);
    const int cidx = seg_cent_off[seg_of[i]] + assign[i];
    const float4 v = *reinterpret_cast<const float4*>(P + (int64_t)members[i] * dp + 4 * gidx);
    unsigned long long* dst = s_sum + cidx * dp + 4 * gidx;
    atomicAdd(dst + 0, (unsigned long long)(long long)__double2ll_rn((double)v.x * KM_FIX));
    atomicAdd(dst + 1, (unsigned long long)(long long)__double2ll_rn((double)v.y * KM_FIX));
    atomicAdd(dst + 2, (unsigned long long)(long long)__double2ll_rn((double)v.z * KM_FIX));
    atomicAdd(dst + 3, (unsigned long long)(long long)__double2ll_rn((double)v.w * KM_FIX));
    if (gidx == 0) atomicAdd(s_cnt + cidx, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < tab; i += blockDim.x)
    if (s_sum[i]) atomicAdd(sums + i, s_sum[i]);
  for (int i = threadIdx.x; i < ncent; i += blockDim.x)
    if (s_cnt[i]) atomicAdd(counts + i, s_cnt[i]);
}

void launch_kmeans_mindist(Ctx* c, const float* P, int dp, const int32_t* members, int64_t m, const int32_t* seg_of,
                           const float* cand, float* mind, int first) {
  ProfScope ps(c, "kmeans_mindist");
  if (m == 0) return;
  hipLaunchKernelGGL(k_kmeans_mindist, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, c->stream, P, dp, members, m,
                     seg_of, cand, mind, first);
  check_launch("k_kmeans_mindist");
}

void launch_kmeans_assign(Ctx* c, const float* P, int dp, const int32_t* members, int64_t m, const int32_t* seg_of,
                          const int32_t* seg_cent_off, const int32_t* seg_k, const float* cents, int32_t* assign,
                          int32_t* changed) {
  ProfScope ps(c, "kmeans_assign");
  if (m == 0) return;
  hipLaunchKernelGGL(k_kmeans_assign, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, c->stream, P, dp, members, m,
                     seg_of, seg_cent_off, seg_k, cents, assign, changed);
  check_launch("k_kmeans_assign");
}

void launch_kmeans_accumulate(Ctx* c, const float* P, int dp, const int32_t* members, int64_t m,
                              const int32_t* seg_of, const int32_t* seg_cent_off, const int32_t* assign,
                              unsigned long long* sums, int32_t* counts, int ncent) {
  ProfScope ps(c, "kmeans_accumulate");
  if (m == 0) return;
  PTS_REQUIRE(dp % 4 == 0, PTS_ERR_ARG, "kmeans: dp must be a multiple of 4");
  const int64_t n = m * (dp / 4);
  if ((int64_t)ncent * dp <= 4096 && ncent <= 1024) {
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(n, 2048)));
    hipLaunchKernelGGL(k_kmeans_accumulate_lds, dim3(blocks), dim3(256), 0, c->stream, P, dp, members, m, seg_of,
                       seg_cent_off, assign, ncent, sums, counts);
    check_launch("k_kmeans_accumulate_lds");
    return;
  }
  hipLaunchKernelGGL(k_kmeans_accumulate, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, P, dp, members,
                     m, seg_of, seg_cent_off, assign, sums, counts);
  check_launch("k_kmeans_accumulate");
}

// ---------------------------------------------------------------------------
// ||z - mu||^2 of every exemplar window (original order): one wave per window

__global__ __launch_bounds__(256) void k_centered_norm(WinGeom g, int64_t n, const float* __restrict__ mu,
                                                       float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t win = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (win >= n) return;
  float acc = 0.f;
  for (int p = lane; p < g.w * g.w; p += 64) {
    const float4 v = win_pixel(g, win, p);
    const float t0 = v.x - mu[4 * p], t1 = v.y - mu[4 * p + 1], t2 = v.z - mu[4 * p + 2], t3 = v.w - mu[4 * p + 3];
    acc = fmaf(t0, t0, acc);
    acc = fmaf(t1, t1, acc);
    acc = fmaf(t2, t2, acc);
    acc = fmaf(t3, t3, acc);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) out[win] = acc;
}

void launch_centered_norm(Ctx* c, const float* img, int H, int W, int w, const float* mu, float* out) {
  ProfScope ps(c, "centered_norm");
  const WinGeom g = geom(img, H, W, w, 1, false);
  const int64_t n = (int64_t)(H - w + 1) * (W - w + 1);
  if (n == 0) return;
  hipLaunchKernelGGL(k_centered_norm, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, c->stream, g, n, mu, out);
  check_launch("k_centered_norm");
}

// res[i] = max(0, cn[perm[i]] - zn[i]);  bres[i] = bn[i] + res[i]
__global__ __launch_bounds__(256) void k_residual(const float* __restrict__ cn, const int32_t* __restrict__ perm,
                                                  const float* __restrict__ zn, const float* __restrict__ bn, int64_t n,
                                                  float* __restrict__ res, float* __restrict__ bres) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float r = fmaxf(cn[perm[i]] - zn[i], 0.f);
  res[i] = r;
  if (bres) bres[i] = bn[i] + r;
}

void launch_residual(Ctx* c, const float* cn, const int32_t* perm, const float* zn, const float* bn, int64_t n,
                     float* res, float* bres) {
  ProfScope ps(c, "residual");
  if (n == 0) return;
  hipLaunchKernelGGL(k_residual, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, cn, perm, zn, bn, n, res,
                     bres);
  check_launch("k_residual");
}

// ---------------------------------------------------------------------------
// leaf-order layout helpers

__global__ __launch_bounds__(256) void k_permute_rows(const float* __restrict__ src, const int32_t* __restrict__ perm,
                                                      int64_t n, int dp, float* __restrict__ dst,
                                                      float* __restrict__ norm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* s = src + (int64_t)perm[i] * dp;
  float* d = dst + i * dp;
  float acc = 0.f;
  for (int k = 0; k < dp; k += 4) {
    const float4 v = *reinterpret_cast<const float4*>(s + k);
    *reinterpret_cast<float4*>(d + k) = v;
    acc = fmaf(v.x, v.x, acc);
    acc = fmaf(v.y, v.y, acc);
    acc = fmaf(v.z, v.z, acc);
    acc = fmaf(v.w, v.w, acc);
  }
  if (norm) norm[i] = acc;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ __launch_bounds__(256) void k_to_bf16_rows(const float* __restrict__ P, int64_t n, int dp, int dk,
                                                      uint16_t* __restrict__ out, float* __restrict__ norm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int k = 0; k < dk; ++k) {
    const uint16_t h = (k < dp) ? f32_to_bf16_rne(P[i * dp + k]) : (uint16_t)0;
    out[i * dk + k] = h;
    const float f = bf16_to_f32(h);
    acc = fmaf(f, f, acc);
  }
  if (norm) norm[i] = acc;
}

__global__ __launch_bounds__(256) void k_leaf_of_ids(const int32_t* __restrict__ leaf_of_ex,
                                                     const int32_t* __restrict__ nn, int64_t n, int64_t N,
                                                     int32_t* __restrict__ leaf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e = nn[i];
  leaf[i] = (e >= 0 && e < N) ? leaf_of_ex[e] : -1;
}

void launch_permute_rows(Ctx* c, const float* src, const int32_t* perm, int64_t n, int dp, float* dst, float* norm) {
  ProfScope ps(c, "permute_rows");
  if (n == 0) return;
  hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, src, perm, n, dp, dst,
                     norm);
  check_launch("k_permute_rows");
}

void launch_to_bf16_rows(Ctx* c, const float* P, int64_t n, int dp, int dk, uint16_t* out, float* norm) {
  ProfScope ps(c, "to_bf16_rows");
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_bf16_rows, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, P, n, dp, dk, out,
                     norm);
  check_launch("k_to_bf16_rows");
}

void launch_leaf_of_ids(Ctx* c, const int32_t* leaf_of_ex, const int32_t* nn, int64_t n, int32_t* leaf, int64_t N) {
  ProfScope ps(c, "leaf_of_ids");
  if (n == 0) return;
  hipLaunchKernelGGL(k_leaf_of_ids, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, leaf_of_ex, nn, n, N,
                     leaf);
  check_launch("k_leaf_of_ids");
}

}  // namespace pts
