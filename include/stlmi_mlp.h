/*
 * stlmi_mlp.h -- C ABI of the learned warm-start kernels (gfx950).
 *
 * A small multilayer perceptron proposes an initial trajectory for STL
 * trajectory optimisation; the STL robustness of the proposal (stlmi.h) is
 * then raised by plain gradient ascent, which is also the fallback without
 * the network.  These entry points are the building blocks the network is
 * trained and run with: a BF16 matrix product on the matrix cores with FP32
 * accumulation and fused bias / ReLU epilogue, BF16 rounding, the ReLU
 * derivative mask, column sums (bias gradients), the mean-squared-error
 * gradient, an Adam update on FP32 master weights, and the gradient-ascent
 * step on trajectories.  The robustness being optimised is the quantitative
 * semantics of arXiv 2501.04194 Sec. III-B with the smooth max/min of
 * Sec. III-C; its use as a differentiable objective for trajectory
 * optimisation follows Sec. VII-A.
 *
 * Conventions: every pointer is caller-owned device memory on the current
 * HIP device; `stream` is a hipStream_t (NULL = default stream); calls only
 * launch work on that stream (no allocation, no synchronisation).  BF16
 * values are stored as uint16_t bit patterns; float -> BF16 rounds to nearest
 * even.  Arguments are checked on the host; failures return a negative
 * stl_status (stlmi.h) with a message in stl_last_error().
 */
#ifndef STLMI_MLP_H
#define STLMI_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "stlmi.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * C = act(A * B + bias) with A an M x K and B a K x N BF16 matrix given by
 * element strides (A[m][k] at A[m*sam + k*sak], B[k][n] at B[k*sbk + n*sbn]),
 * FP32 accumulation on MFMA.  bias (length N, FP32) may be NULL; relu != 0
 * applies max(.,0).  Outputs: c32 (FP32, c32[m*ldc32 + n]) and/or c16 (BF16,
 * c16[m*ldc16 + n]); either may be NULL.  beta32 != 0 adds to c32 instead of
 * overwriting it.  M, N, K >= 0.
 */
stl_status stl_bf16_gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                         int64_t sbn, int32_t M, int32_t N, int32_t K, const float* bias, int32_t relu,
                         float* c32, int64_t ldc32, int32_t beta32, uint16_t* c16, int64_t ldc16, void* stream);

/* y[i] = bf16(x[i]) (round to nearest even), i < n. */
stl_status stl_cast_bf16(const float* x, uint16_t* y, int64_t n, void* stream);

/*
 * ReLU derivative: g16[i] = bf16(g[i] * (h[i] > 0)) where h is the BF16
 * post-activation (h may be NULL: no mask), i < n.
 */
stl_status stl_relu_grad_bf16(const float* g, const uint16_t* h, uint16_t* g16, int64_t n, void* stream);

/* out[j] = sum_i x[i*ld + j] for j < cols, i < rows (FP32, fixed order). */
stl_status stl_colsum(const float* x, int32_t rows, int32_t cols, int64_t ld, float* out, void* stream);

/*
 * Mean-squared error: g[i] = 2 (y[i] - t[i]) / n and loss[0] = sum (y-t)^2 / n
 * (loss may be NULL), i < n.
 */
stl_status stl_mse_grad(const float* y, const float* t, float* g, float* loss, int64_t n, void* stream);

/*
 * One Adam step (Kingma & Ba, with bias correction) on FP32 master weights:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps);
 * w16 (may be NULL) receives bf16(w).  step >= 1.
 */
stl_status stl_adam_step(float* w, const float* g, float* m, float* v, uint16_t* w16, int64_t n, float lr,
                         float b1, float b2, float eps, int32_t step, void* stream);

/*
 * Gradient-ascent step on trajectories x [N, T, D]:
 * x[n, t, d] += lr * dx[n, t, d] for t >= t0 and d < d_upd, only where
 * active[n] != 0 (active may be NULL: all).
 */
stl_status stl_ascent_update(float* x, const float* dx, const int32_t* active, int64_t N, int32_t T, int32_t D,
                             int32_t t0, int32_t d_upd, float lr, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STLMI_MLP_H */
