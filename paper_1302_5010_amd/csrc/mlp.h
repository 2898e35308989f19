// Launchers of the learned-proposal kernels (mlp.hip).  Internal; the public
// entry points are the bmpl_mlp_* calls of include/bmpl.h.
//
// Matrix products C = X W^T: X [M][ldx] and W [N][ldw] bfloat16 (raw 16-bit storage), both
// K-contiguous with kpad % 64 == 0 and zeros in columns past the true contraction length.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpl {

constexpr size_t TOPK_MAX_LDS = 152 * 1024;   // row keys of the top-k kernel (rows up to 38912 atoms)

hipError_t mlp_project(const float* At, int64_t lda, int n, int m, const float* P, int d, uint16_t* APt, int npad,
                       hipStream_t s);
hipError_t mlp_signals_bf16(const float* B, int64_t ldb, int n, int p, uint16_t* B16, int npad, hipStream_t s);
// C[r][c] = (X W^T)[r][c] (+ bias[c])
hipError_t mlp_gemm_store(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                          float* C, int64_t ldc, const float* bias, hipStream_t s);
// u = (X W^T)[r][c] + bias[c]; U[r][c] = u when U != null; H[r][c] = bf16(gelu(u))
hipError_t mlp_gemm_bias_gelu(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                              const float* bias, float* U, int64_t ldu, uint16_t* H, int64_t ldh, hipStream_t s);
// d = (X W^T)[r][c] * gelu'(U[r][c]); D = d (float32), D16 = bf16(d)
hipError_t mlp_gemm_gelu_back(const uint16_t* X, int64_t ldx, int M, const uint16_t* W, int64_t ldw, int N, int kpad,
                              const float* U, int64_t ldu, float* D, int64_t ldd, uint16_t* D16, int64_t ld16,
                              hipStream_t s);
// X0[r] = bf16(Z[r] sqrt(d) / ||Z[r]||); Zout (optional) receives X0 widened to float32
hipError_t mlp_embed_norm(const float* Z, int d, int p, uint16_t* X0, float* Zout, int64_t ldz_out, hipStream_t s);
// weighted BCE with logits: S (logits, in place -> dl/ds / rows), D16 its bfloat16 copy, loss (device double)
hipError_t mlp_bce_grad(float* S, int64_t lds, uint16_t* D16, int64_t ld16, int m, int mpad, int rows,
                        const int* supp, int64_t ld_supp, const int* supp_len, float pos_w, float* rowloss,
                        double* loss, hipStream_t s);
hipError_t mlp_colsum(const float* in, int64_t ld, int rows, int cols, float* out, hipStream_t s);
// out[c][r] = in[r][c]; zero for rows <= r < ldo (ldo % 64 == 0)
hipError_t mlp_transpose(const uint16_t* in, int64_t ldi, int rows, int cols, uint16_t* out, int64_t ldo,
                         hipStream_t s);
hipError_t mlp_adam(float* P, float* m1, float* m2, const float* g, uint16_t* P16, int64_t count, float lr,
                    float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t mlp_params_bf16(const float* P, uint16_t* P16, int64_t count, hipStream_t s);
// top-k indices per row of S [rows][lds] (first L columns), ascending by index, -1 padded
hipError_t mlp_topk(const float* S, int64_t lds, int rows, int L, int k, int* out, int64_t ldo, hipStream_t s);

}  // namespace bmpl
