/*
 * pts.h - C ABI of libpts, the MI355X (gfx950) engine for the search and
 * optimisation phases of perspective texture optimisation
 * (Bashir & Ghouri, "Perspective Texture Synthesis Based on Improved Energy
 * Optimization", Methodology sections 2.1-2.2).
 *
 * Problem statement followed by the calls (Methodology 2.1, Eq. 4): an
 * exemplar Z and an output X, both images with channels R, G, B and a
 * perspective guidance channel S (Section 4, the scale map as a fourth
 * channel); a neighbourhood width w; output neighbourhoods x_q on a sparse
 * grid of stride s (Methodology 2.2: interval w/4); the texture energy
 * E = sum_q ||x_q - z_q||^r with r = 0.8 (Eq. 5) minimised by alternating a
 * search phase (nearest exemplar neighbourhood z_q of every x_q, here the
 * "E-step") and an optimisation phase (IRLS, Eqs. 6-8, processed as 2x2
 * pixel patches, here the "M-step").  The search runs in a PCA-reduced space
 * through a hierarchical k-means tree (Methodology 2.2).
 *
 * Conventions for every call:
 *  - Return value: PTS_OK (0) or a negative PTS_ERR_* code; the message is
 *    available from pts_last_error().  No C++ exception crosses the ABI.
 *  - Pointers without a _host suffix are DEVICE pointers owned by the caller
 *    (for example torch tensors).  The library never frees or keeps them past
 *    the call; work is ordered on the context's HIP stream, so the caller keeps
 *    them alive until that stream has finished the work.  _host pointers are
 *    host memory, read or written before the call returns.
 *  - Calls that return host results (energy, statistics, export) synchronise
 *    the context's stream.
 *  - Image layout: float32 [H][W][4] row-major, channels R, G, B in [0, 1]
 *    and S = lambda * (y + 0.5) / H (the guidance), 16 bytes per pixel.
 *  - Neighbourhood vector of the window with top-left (u, v): D = 4 w^2
 *    entries, index (dy * w + dx) * 4 + c.
 *  - Exemplar windows: every top-left corner at stride 1; window id
 *    e = v * (Wz - w + 1) + u; N = (Hz - w + 1) (Wz - w + 1).
 *  - Output windows: rows v_i = i * s, i = 0 .. (H - w) / s (no vertical
 *    wrap); columns u_j = j * s, j = 0 .. W / s - 1, wrapping in x; window
 *    id q = i * (W / s) + j; nq = ((H - w) / s + 1) * (W / s).  Requires
 *    (H - w) % s == 0, W % s == 0, even w, s, H and W.
 *  - A context is used by one thread at a time.  Device: gfx950 only.
 */
#ifndef PTS_H
#define PTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PTS_OK 0
#define PTS_ERR_ARG (-1)          /* invalid argument (shape, pointer, range) */
#define PTS_ERR_STATE (-2)        /* call out of order (no exemplar, no index, no MLP) */
#define PTS_ERR_OOM (-3)          /* device allocation failed; context stays usable */
#define PTS_ERR_HIP (-4)          /* HIP runtime error; message holds its string */
#define PTS_ERR_UNSUPPORTED (-5)  /* not a gfx950 device, or a shape outside the limits */

/* E-step search modes. */
#define PTS_MODE_EXACT_FULL 0   /* exhaustive, full D, FP32 (the exact reference) */
#define PTS_MODE_EXACT_PCA 1    /* exhaustive in PCA space, FP32 */
#define PTS_MODE_TREE 2         /* PCA + k-means tree descent + leaf scan, FP32 (the paper's search) */
#define PTS_MODE_BRUTE_BF16 3   /* PCA, all exemplars, BF16 MFMA distances, top-k, FP32 re-rank */
#define PTS_MODE_LEARNED 4      /* PCA, MLP proposes leaves, FP32 scan of the proposed leaves */
#define PTS_MODE_LEARNED_BF16 5 /* as LEARNED, leaves scanned with BF16 MFMA + top-k + FP32 re-rank */
/* As LEARNED_BF16 but in one BF16 pass whose candidates are not the exact
 * top-8: the scanned rows of each (query, leaf) are split into 16 classes
 * (rows i and i + 16 of every 32-row tile of the leaf), each class keeps
 * its smallest score and the row holding it, and the query's topk smallest
 * class minima over its leaves (always including the BF16 minimum) go to
 * the FP32 re-rank.  A departure from the top-8 definition, for speed: the
 * second pass and the per-query pass are saved. */
#define PTS_MODE_LEARNED_BF16_CLASS 6

typedef struct pts_ctx pts_ctx;

/* Optional device allocator.  alloc returns a device pointer (NULL on
 * failure) usable on `stream`; release frees it.  NULL -> hipMalloc/hipFree. */
typedef struct pts_alloc {
  void* (*alloc)(void* user, size_t bytes, void* stream);
  void (*release)(void* user, void* ptr, size_t bytes, void* stream);
  void* user;
} pts_alloc;

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Fails with PTS_ERR_UNSUPPORTED
 * if the device is not gfx950.  *out is NULL on failure. */
int pts_create(pts_ctx** out, int device, void* hip_stream, const pts_alloc* alloc_or_null);
void pts_destroy(pts_ctx* ctx);
/* Message of the last failed call on ctx ("" if none).  With ctx == NULL:
 * the message of the last failed pts_create. */
const char* pts_last_error(const pts_ctx* ctx);
/* Change the stream used by later calls. */
int pts_set_stream(pts_ctx* ctx, void* hip_stream);

/* ---- exemplar ---------------------------------------------------------- */

/* Set the exemplar Z from a device image rgbs [Hz][Wz][4] (guidance already
 * in channel 3).  The library keeps its own copy.  Invalidates the index and
 * the MLP.  Section 4: the scale map enters as a channel beside R, G, B.
 * An image holding a non-finite value is refused (PTS_ERR_ARG; the previous
 * exemplar stays).  Synchronous. */
int pts_set_exemplar(pts_ctx* ctx, const float* rgbs, int Hz, int Wz);
/* Convenience: host uint8 RGB [Hz][Wz][3]; R,G,B = u8 / 255 and
 * S = guidance_weight * (y + 0.5) / Hz. */
int pts_set_exemplar_u8(pts_ctx* ctx, const uint8_t* rgb_host, int Hz, int Wz, float guidance_weight);
/* Fill an output image's guidance channel: x[y][x][3] = weight * (y+0.5)/H,
 * leaving R, G, B unchanged. */
int pts_fill_guidance(pts_ctx* ctx, float* x_rgbs, int H, int W, float guidance_weight);
/* Convert a host uint8 RGB image to a device RGBS image (R,G,B = u8/255,
 * S as in pts_fill_guidance). */
int pts_rgbs_from_u8(pts_ctx* ctx, const uint8_t* rgb_host, int H, int W, float guidance_weight, float* x_rgbs);

/* ---- perspective scale map (Methodology 1, Eqs. 1-3; Section 4 steps 1-3) */

/* Fill the guidance channel of a device image x_rgbs [H][W][4] with the
 * scale map of a locally planar texture seen under slant `slant` and tilt
 * `tilt` (radians; slant in [0, pi/2), tilt in [0, pi/2]), computed for an
 * image of ref_h x ref_w pixels (>= 3 each) with its origin at the
 * bottom-left corner (Eqs. 1-3, the leading term of Eq. 3 read as S_max),
 * then resampled bilinearly to H x W (pixel centres aligned, edge
 * coordinates clamped).  The channel holds weight * (S - S_min) / S_D, the
 * map normalised to [0, 1] (zero when slant = 0 makes it flat).  ref = (H,
 * W) gives an image its own map (an exemplar), ref = the exemplar's size
 * the output's map (step 2).  R, G, B are untouched.  Out-of-range angles or
 * sizes: PTS_ERR_ARG, nothing written. */
int pts_scale_guidance(pts_ctx* ctx, float* x_rgbs, int H, int W, int ref_h, int ref_w, double slant, double tilt,
                       float weight);
/* Section 4 step 3, the scale-matched initial output: every tile x tile
 * block of x_rgbs [H][W][4] (row-major tiles, ragged last row and column
 * taking the window's top-left part) copies R, G, B of the exemplar window
 * (corner (u, v), tile x tile pixels) of ex_rgbs [Hz][Wz][4] (device, the
 * exemplar at the output's scale, e.g. the coarsest pyramid level) whose
 * centre (u + tile/2, v + tile/2) has the scale of the block's centre
 * pixel: equal scale is equal projected coordinate p(Y), a line through
 * the exemplar point the block's centre samples.  rnd (device uint32
 * [tiles][2]) holds the caller's uniform draws: the column rnd[k][0] mod
 * (Wz - tile + 1) when cos(tilt) >= sin(tilt), else the row rnd[k][1] mod
 * (Hz - tile + 1), the other coordinate being the nearest to the line
 * (rounded half up, clamped into the exemplar); with slant = 0 (a flat map)
 * both are drawn.  The guidance channel is that of pts_scale_guidance with
 * ref = (Hz, Wz).  tile in 1..min(Hz, Wz); the exemplar's own guidance is
 * not read. */
int pts_scale_init(pts_ctx* ctx, const float* ex_rgbs, int Hz, int Wz, float* x_rgbs, int H, int W, int tile,
                   const uint32_t* rnd, double slant, double tilt, float weight);

/* ---- index: PCA basis + k-means tree (Methodology 2.2) ----------------- */

typedef struct pts_index_params {
  int w;                  /* neighbourhood width (even, 2..32) */
  int pca_dims;           /* d (1..128); 0 = smallest d reaching variance_target, at
                             most 128 (the widest search kernels): where 128 dimensions
                             retain less, d = 128 and retained_variance reports it */
  double variance_target; /* used when pca_dims == 0 (the paper keeps 95 %) */
  int branching;          /* k of the k-means splits (paper: 4), 2..64 */
  int depth;              /* maximum tree depth, 0..8 (0 = a single leaf); -1 = no cap,
                             the paper's rule alone: split until every leaf holds
                             fewer than `branching` members */
  int kmeans_max_iter;    /* Lloyd iterations per split (default 50) */
  uint64_t seed;          /* seeds the k-means++ initial centres */
  int make_bf16;          /* also keep a bf16 copy of the projected exemplar */
} pts_index_params;

typedef struct pts_index_info {
  int64_t N;
  int D, d;
  double retained_variance; /* sum of the d largest eigenvalues / trace */
  int n_nodes, n_leaves;
  int64_t leaf_min, leaf_max;
  double leaf_mean;
  double build_ms;
} pts_index_info;

/* Build the index of the current exemplar: mean and covariance of all
 * exemplar windows (FP64 accumulation on the GPU), host FP64 symmetric
 * eigensolve, basis B = the d leading eigenvectors (largest-|entry| made
 * positive), projection z' = B^T (z - mu), and the k-means tree over z'
 * (nodes split while depth < `depth`, any depth with depth = -1, and the
 * node holds >= branching members - the paper's stop rule for small
 * clusters; a node whose k-means leaves one cluster, i.e. whose points are
 * identical, stays a leaf).  Synchronous. */
int pts_build_index(pts_ctx* ctx, const pts_index_params* p, pts_index_info* info_host);

/* Host form of an index, for export/import (parity tests share a basis and
 * tree with an independent implementation this way).  Nodes breadth-first,
 * children of a node contiguous; leaves numbered in node order; perm lists
 * exemplar ids leaf by leaf; leaf_off [n_leaves+1] indexes perm. */
typedef struct pts_index_host {
  int w, D, d, n_nodes, n_leaves;
  int64_t N;
  double* mu;            /* [D] */
  double* basis;         /* [D][d] row-major (column k = k-th axis) */
  double* eigenvalues;   /* [d] (export only; ignored on import) */
  double* centroids;     /* [n_nodes][d]; row 0 (root) unused */
  int32_t* first_child;  /* [n_nodes] */
  int32_t* n_children;   /* [n_nodes] (0 = leaf) */
  int32_t* leaf_of_node; /* [n_nodes] (-1 = internal) */
  int64_t* leaf_off;     /* [n_leaves + 1] */
  int32_t* perm;         /* [N] */
} pts_index_host;

/* Export: with any array pointer NULL, only the sizes are filled in; call
 * again with arrays of those sizes.  Import: replaces the index (sizes and
 * arrays read from *ix; ix->N and ix->w must match the exemplar) and
 * re-projects the exemplar with the imported basis. */
int pts_export_index(pts_ctx* ctx, pts_index_host* ix);
int pts_import_index(pts_ctx* ctx, const pts_index_host* ix, int make_bf16);

/* ---- E-step: search phase (Methodology 2.1-2.2) ------------------------ */

typedef struct pts_estep_params {
  int mode;        /* PTS_MODE_* */
  int w;           /* neighbourhood width; must equal the index's w for PCA modes */
  int stride;      /* grid stride s (the paper: w / 4) */
  int topk;        /* BF16 candidates kept for the FP32 re-rank (0 = 8; 1..16 for BRUTE_BF16
                      and LEARNED_BF16_CLASS, 1..8 for the other learned forms) */
  int rerank_full; /* 1: re-rank BF16 candidates by full-D distance; 0: PCA space */
  int n_proposals; /* leaves proposed by the MLP (4; 1..8) */
  float margin;    /* softmax margin p1 - p2 below which the tree is used (0.2) */
  int residual;    /* 1: rank PCA-space candidates by ||q' - z'||^2 + ||z - mu||^2 - ||z'||^2,
                      i.e. also charge each exemplar window its energy outside the PCA
                      subspace (leaf scans, BF16 scans and the PCA-space re-rank); 0: plain
                      PCA-space distance */
  int scan_slots;  /* LEARNED_BF16: rows the second scan pass may collect per (query, leaf)
                      pair and half-wave before the query is redone by its exact per-query
                      pass (0 = 14; 0..14).  Results do not depend on it. */
} pts_estep_params;

typedef struct pts_estep_stats {
  int64_t nq;             /* queries searched */
  int64_t fallbacks;      /* learned modes: queries that fell back to the tree */
  int64_t scan_overflows; /* LEARNED_BF16: queries redone by the exact per-query pass */
  int64_t scan_rows;      /* learned modes: (query, exemplar) scores of the leaf scan
                             (LEARNED_BF16: its first, bounding pass) */
  int64_t collect_rows;   /* LEARNED_BF16: (query, exemplar) scores of its second pass */
  double ms;              /* wall time of the call on the stream (hipEvent); with statistics
                             asked for, the counts above add synchronisations to it */
} pts_estep_stats;

/* For every output window q of x_rgbs [H][W][4]: nn[q] = id of the chosen
 * exemplar window (the original window id e), dist[q] = ||x_q - z_nn|| over
 * the full D in FP32, whatever space the search ran in.  Ties go to the
 * lowest e (exact modes) / lowest child index (tree descent).  nn: int32
 * [nq]; dist: float32 [nq].  st_host may be NULL (then no synchronisation).
 * With st_host given, x_rgbs is first checked: a non-finite value returns
 * PTS_ERR_ARG (without statistics the call does not wait for the stream,
 * and a non-finite window gets a non-finite distance). */
int pts_estep(pts_ctx* ctx, const float* x_rgbs, int H, int W, const pts_estep_params* p, int32_t* nn,
              float* dist, pts_estep_stats* st_host);

/* Exhaustive full-D search (the exact reference of Eq. 4's z_q) for the
 * listed output windows only: qids int32 [n] (window ids, each < nq of the
 * grid); nn int32 [n] and dist float32 [n] (||x_q - z_nn||, FP32), ties to
 * the lowest exemplar id.  Used to evaluate approximate searches on a sample. */
int pts_exact_search(pts_ctx* ctx, const float* x_rgbs, int H, int W, int w, int stride, const int32_t* qids,
                     int64_t n, int32_t* nn, float* dist);

/* PCA projection of the output windows: qproj float32 [nq][d] (row q =
 * B^T (x_q - mu)).  The first step of every PCA-space search. */
int pts_project(pts_ctx* ctx, const float* x_rgbs, int H, int W, int stride, float* qproj);
/* Projected exemplar windows in original id order, zproj float32 [N][d]. */
int pts_exemplar_projection(pts_ctx* ctx, float* zproj);
/* leaf[i] = the tree leaf holding exemplar window nn[i] (int32, device). */
int pts_leaf_of(pts_ctx* ctx, const int32_t* nn, int64_t n, int32_t* leaf);
/* Tree descent only: leaf[i] for projected queries qproj [n][d]. */
int pts_descend(pts_ctx* ctx, const float* qproj, int64_t n, int32_t* leaf);

/* ---- M-step: optimisation phase, 2x2 patches (Methodology 2.1-2.2) ----- */

typedef struct pts_mstep_params {
  int w, stride;
  float r;          /* robust exponent (Eq. 5), 0.8 */
  float delta;      /* distance floor for W = max(d, delta)^(r-2), 1e-3 */
  int patch_offset; /* 0: patches at even origins (exact IRLS minimiser);
                       1: odd origins (9 windows wholly contain a patch at w=8, s=2) */
  int hist_bins;    /* 0: weights of Eq. 7; 2..256: histogram-weighted (Section 3, Eq. 9):
                       W_q / (1 + sum_j max[0, H_x,j(b) - H_z,j(b)]) over the R, G, B
                       histograms (fractions, hist_bins equal bins over [0, 1]) of the
                       output as given and of the exemplar, b the bin of the centre pixel
                       of matched exemplar window nn[q] (exact binning for powers of two) */
} pts_mstep_params;

/* With W_q = max(dist[q], delta)^(r-2) (Eq. 7), set for every pixel p of
 * every 2x2 patch P and c in R,G,B:
 *   x(p,c) = sum_{q in C(P)} W_q Z_c(e_q + p - o_q) / sum_{q in C(P)} W_q,
 * C(P) = output windows containing every pixel of P (x wraps), o_q = window
 * corner, e_q = corner of exemplar window nn[q].  Channel S is not written.
 * In place: reads only nn, dist and the exemplar, so x_rgbs may be the image
 * the E-step read.  No atomics: each patch is written by one thread. */
int pts_mstep(pts_ctx* ctx, const int32_t* nn, const float* dist, float* x_rgbs, int H, int W,
              const pts_mstep_params* p);

/* The blend weights the M-step uses (Eq. 7; with hist_bins, Eq. 9 for the
 * output x_rgbs [H][W][4] as given): weights float32 [nq], device. */
int pts_irls_weights(pts_ctx* ctx, const int32_t* nn, const float* dist, const float* x_rgbs, int H, int W,
                     const pts_mstep_params* p, float* weights);

/* Final histogram match (Section 4, step 4): each of R, G, B of x_rgbs
 * [H][W][4] takes the context exemplar's distribution rank for rank - the
 * pixels sorted by value (ties in pixel order), the i-th smallest of n takes
 * the exemplar's sorted value of rank floor((i + 1/2) n_z / n).  Guidance
 * untouched; in place. */
int pts_histogram_match(pts_ctx* ctx, float* x_rgbs, int H, int W);

/* Energy (Eqs. 4-5): E = sum_q rho(dist[q]) with rho(d) = d^r for
 * d >= delta and (1 - r/2) delta^r + (r/2) delta^(r-2) d^2 below (the
 * smooth form matching W's floor), E2 = sum_q dist[q]^2.  Deterministic
 * reduction.  Synchronous. */
int pts_energy(pts_ctx* ctx, const float* dist, int64_t nq, float r, float delta, double* E_host,
               double* E2_host);

/* The same energy (Eqs. 4-5), left on the device: out_device[0] = E,
 * out_device[1] = E2 as float32, the same deterministic reduction and
 * values as pts_energy (which rounds them to double).  out_device: caller-owned device
 * memory of 2 floats.  Asynchronous: ordered on the context's stream and
 * returns without waiting, so iterations that only record their energy
 * need no host round trip.  nq == 0 writes zeros. */
int pts_energy_device(pts_ctx* ctx, const float* dist, int64_t nq, float r, float delta, float* out_device);
/* pts_energy_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or other allocating routine.
 * Same kernels, launch shape and results (bitwise) as pts_energy_device.
 * Its per-block partial sums live in a fixed library array of 2 x 1024
 * floats (8 KiB) per device, located when the first context is created on
 * that device and held until the process ends; every nq >= 0 fits (at most
 * 1024 blocks, each striding over the distances), so no size is refused.
 * Every call on a device shares that array and the next call overwrites it:
 * calls that overlap on one device (other streams, other contexts, other
 * threads) race and must be ordered by the caller.  The library's own
 * profiler does not record this call.  Errors as pts_energy_device. */
int pts_energy_device_noalloc(pts_ctx* ctx, const float* dist, int64_t nq, float r, float delta,
                              float* out_device);

/* ---- multiscale solve (Methodology 2.1: coarse-to-fine) ---------------- */

typedef struct pts_level_params {
  int w, stride, iters;
  int pca_dims, branching, depth;
} pts_level_params;

typedef struct pts_solve_params {
  int levels;                     /* 1..8, listed coarse to fine */
  const pts_level_params* level;  /* host array [levels] */
  int mode;                       /* search mode at the finest level */
  int coarse_mode;                /* search mode at the coarser levels */
  int topk, rerank_full, n_proposals;
  float margin;
  int residual;
  float r, delta;
  int patch_offset;
  float guidance_weight;          /* >= 0: every level's guidance is recomputed as
                                     weight * (y + 0.5) / H (exemplar pyramid and upsampled
                                     outputs); < 0: the exemplar's own guidance channel and
                                     x0's are carried through the pyramid and the upsampling
                                     by the same filters as the colours (a scale map) */
  uint64_t seed;                  /* k-means seed for indexes built by the solve */
  int kmeans_max_iter;
  int reuse_finest_index;         /* 1: use the context's current index (and MLP) at the finest
                                     level; that index must have been built from an exemplar
                                     whose guidance channel is the one the solve uses there */
  int hist_bins;                  /* every blend histogram-weighted (Eq. 9) with this many bins; 0: off */
  int final_hist_match;           /* 1: the result's histograms matched to the exemplar's at the end */
  int scale_map;                  /* 1: the guidance of every level is the perspective scale map
                                     (pts_scale_guidance) of slant and tilt instead of the row
                                     guidance: each exemplar level its own, each upsampled output
                                     the resample of its exemplar level's; guidance_weight >= 0 */
  double slant, tilt;             /* radians, used when scale_map = 1 */
} pts_solve_params;

typedef struct pts_solve_trace {
  int capacity;      /* entries available in the arrays below (host) */
  int count;         /* entries written */
  int32_t* level;
  double* E;         /* E(x^{t-1}; nn^t) recorded after each search */
  double* E2;
  double* ms;        /* search + blend + energy, per iteration */
  int64_t* nq;
  int64_t* changes;  /* matches that differ from the previous iteration */
  int64_t* fallbacks;
} pts_solve_trace;

/* Coarse-to-fine solve on the context's exemplar (x0 holding a non-finite
 * value: PTS_ERR_ARG).  The exemplar pyramid
 * (separable [1 4 6 4 1]/16 blur, mirrored borders, 2x decimation; guidance
 * recomputed per level) is built on the GPU.  x0_rgbs [H0][W0][4] is the
 * initial output at the coarsest level; each finer level starts from the
 * 2x bilinear upsampling (x wraps, y clamps) of the previous result.  The
 * final image [H][W][4] (H = H0 << (levels-1)) is written to x_rgbs.
 * trace_host may be NULL. */
int pts_solve(pts_ctx* ctx, const pts_solve_params* p, const float* x0_rgbs, int H0, int W0, float* x_rgbs,
              int H, int W, pts_solve_trace* trace_host);
/* The GPU's exemplar pyramid level `level` of `levels` (0 = coarsest) as an
 * RGBS image [Hz >> (levels-1-level)][...][4]. */
int pts_exemplar_pyramid_level(pts_ctx* ctx, int levels, int level, float guidance_weight, float* out_rgbs);
/* 2x bilinear upsampling of R,G,B (x wraps, y clamps), guidance recomputed. */
int pts_upsample2(pts_ctx* ctx, const float* x_rgbs, int H, int W, float guidance_weight, float* out_rgbs);

/* ---- learned leaf proposal ----------------------------------------------- */

/* MLP n_in -> hidden -> hidden -> n_out, GELU (exact erf; the matrix-core
 * inference of pts_mlp_propose and the learned modes evaluates it within
 * 4.2e-4, below the bf16 rounding of the activations), input scaled per
 * feature by a fixed vector (default 1 / sqrt(eigenvalue) of the index).
 * Parameters packed W1 [h][n_in], b1 [h], W2 [h][h], b2 [h], W3 [n_out][h],
 * b3 [n_out], float32.  n_out must equal the index's leaf count to be used
 * by the learned E-step modes.  Weights initialised from `seed`
 * (uniform +-1/sqrt(fan_in)). */
int pts_mlp_init(pts_ctx* ctx, int n_in, int hidden, int n_out, uint64_t seed);
int pts_mlp_n_params(pts_ctx* ctx, int64_t* n_host);
int pts_mlp_get_weights(pts_ctx* ctx, float* params_host);
int pts_mlp_set_weights(pts_ctx* ctx, const float* params_host);
int pts_mlp_set_input_scale(pts_ctx* ctx, const float* scale_host);
/* logits float32 [n][n_out] for queries q float32 [n][n_in].  bf16 != 0:
 * GEMM operands rounded to bf16 (FP32 accumulation). */
int pts_mlp_forward(pts_ctx* ctx, const float* q, int64_t n, int bf16, float* logits);
/* Mean softmax cross-entropy over the n pairs (q, label) and its gradient,
 * packed like the parameters, into grad (device, float32 [n_params]). */
int pts_mlp_loss_grad(pts_ctx* ctx, const float* q, const int32_t* label, int64_t n, int bf16, float* grad,
                      float* loss_host);

typedef struct pts_train_params {
  int64_t steps;
  int batch;
  float lr, beta1, beta2, eps;
  uint64_t seed;     /* minibatch sampling */
  int bf16;
  int log_every;     /* loss recorded every log_every steps */
} pts_train_params;

/* Adam training on n pairs (q [n][n_in], label [n]) held on the device.
 * loss_log_host [steps / log_every] may be NULL.  Synchronous at the end. */
int pts_mlp_train(pts_ctx* ctx, const float* q, const int32_t* label, int64_t n, const pts_train_params* p,
                  float* loss_log_host);
/* Top-k leaves (descending logit, ties to the lowest leaf) and the softmax
 * margin p1 - p2 per query, without writing the logits. */
int pts_mlp_propose(pts_ctx* ctx, const float* q, int64_t n, int k, int32_t* leaves, float* margin);

/* ---- host utilities (no device needed) ---------------------------------- */

/* The host FP64 symmetric eigensolver used by pts_build_index (Householder
 * tridiagonalisation, bisection, inverse iteration): the d leading
 * eigenpairs of the symmetric n x n matrix C_host (row-major).  evals_host
 * [d] descending; evecs_host [n][d] row-major, each column's
 * largest-magnitude entry positive.  nthreads <= 0: up to 16 threads. */
int pts_eig_sym_top(const double* C_host, int n, int d, double* evals_host, double* evecs_host, int nthreads);

/* ---- profiling -------------------------------------------------------- */

/* When enabled, every kernel launch is bracketed by hipEvents on the
 * context's stream and its duration accumulated per kernel name.  Enabling
 * clears the table. */
int pts_profile_enable(pts_ctx* ctx, int on);
/* Number of kernels in the table; for i < count fills the name, total ms
 * and launch count (synchronises the stream). */
int pts_profile_read(pts_ctx* ctx, int i, char* name_host, int name_cap, double* total_ms_host,
                     int64_t* launches_host);
int pts_profile_count(pts_ctx* ctx, int* count_host);

#ifdef __cplusplus
}
#endif

#endif /* PTS_H */
