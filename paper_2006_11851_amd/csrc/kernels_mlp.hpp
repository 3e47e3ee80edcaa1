// Launchers of the MLP kernels (internal).
#pragma once

#include "kernels.hpp"

namespace pts {

// C[M][N] = op(A) op(B); ta: A stored [K][M]; tb: B stored [N][K]; bf: round operands to bf16
void launch_gemm(Ctx* c, bool ta, bool tb, bool bf, const float* A, const float* B, float* C, int M, int N, int K,
                 bool accumulate);
void launch_sample_idx(Ctx* c, uint64_t seed, int64_t step, int batch, int64_t n, int64_t* idx);
void launch_gather_scale(Ctx* c, const float* Q, int ld, const float* scale, int n_in, const int64_t* idx,
                         const int32_t* lab_in, int64_t n, float* X, int32_t* lab_out);
void launch_bias_act(Ctx* c, float* Z, float* H, const float* bias, int64_t M, int N, bool gelu);
void launch_softmax_ce(Ctx* c, const float* L, const int32_t* lab, int64_t M, int N, float* G, float* row_loss);
void launch_gelu_bwd(Ctx* c, float* dH, const float* Z, int64_t n);
void launch_colsum(Ctx* c, const float* G, int64_t M, int N, float* out);
void launch_mean(Ctx* c, const float* v, int64_t n, float* out);
void launch_adam(Ctx* c, float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                 float eps, int64_t t);
// dst [n_p] = src [n] followed by `fill`
void launch_pad_f32(Ctx* c, const float* src, int n, int n_p, float fill, float* dst);
// bf16 copy, zero padded; perm: columns in the matrix-core lane order
void launch_to_bf16_pad(Ctx* c, const float* src, int rows, int cols, int rows_p, int cols_p, bool perm,
                        uint16_t* dst);
// leaves [nq][k] (descending logit, ties to the lower leaf) and margin p1 - p2
// of the network applied to bf16(Qp * scale): W1b [hidden][K1] natural order,
// W2b [hidden][hidden] and W3b [round_up(N, 32)][hidden] with columns in the
// lane order (zero rows past N), b3 padded to round_up(N, 32) with -FLT_MAX
void launch_mlp_propose(Ctx* c, const float* Qp, int ld, int64_t nq, const float* scale, int n_in, int K1,
                        const uint16_t* W1b, const float* b1, const uint16_t* W2b, const float* b2, int hidden,
                        const uint16_t* W3b, const float* b3, int N, int k, int32_t* leaves, float* margin);

// mlp.cpp: proposals for projected queries (rows of stride ld) with the context's MLP
void mlp_propose_rows(Ctx* c, const float* Qp, int ld, int64_t n, int k, int32_t* leaves, float* margin);

}  // namespace pts
