// Learned warm-start kernels for gfx950: BF16 matrix product on the matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) with a fused
// bias/ReLU epilogue, BF16 rounding, ReLU derivative mask, column sums, MSE
// gradient, Adam and the trajectory gradient-ascent step.  C ABI in
// include/stlmi_mlp.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/stlmi_mlp.h"

namespace stlmi_mlp {

#define DEV static __device__ __forceinline__

typedef float float4_t __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even on the 16 dropped mantissa bits
DEV uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

DEV float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int TM = 64, TN = 64, TK = 32;
constexpr int LDK = TK + 8;     // LDS row: 32 k-values and 8 of pad (rows 80 bytes apart fall on distinct banks)

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// 8 elements p[0], p[s], .., p[7 s] of which the first nvalid exist (zeros
// after them); one 16-byte load when vec (s = 1, nvalid = 8, aligned)
DEV void load8(const uint16_t* p, int64_t s, int nvalid, bool vec, uint16_t* v)
{
    if (vec) {
        const uint4 u = *(const uint4*)p;
        __builtin_memcpy(v, &u, 16);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = i < nvalid ? p[i * s] : (uint16_t)0;
    }
}

DEV bool al16(const void* p) { return (((uintptr_t)p) & 15) == 0; }

// C[M,N] = act(A[M,K] B[K,N] + bias) on v_mfma_f32_16x16x32_bf16.  Work-group
// tile 64x64, four waves of 32x32 (2x2 blocks of 16x16), K in steps of 32.
// LDS holds A as [m][k] and B as [n][k] (k contiguous), so each lane's MFMA
// operand (row or column l % 16, k = 8 (l / 16) .. + 7) is one 16-byte read.
// Each of the 256 threads stages 8 consecutive elements of A and of B along
// the dimension that is contiguous in memory (one 16-byte load when aligned
// and in range); any strides work, transposed operands included.
__global__ void __launch_bounds__(256) gemm_bf16_kernel(const uint16_t* A, int64_t sam, int64_t sak,
                                                        const uint16_t* B, int64_t sbk, int64_t sbn, int M, int N,
                                                        int K, const float* bias, int relu, float* c32,
                                                        int64_t ldc32, int beta32, uint16_t* c16, int64_t ldc16)
{
    __shared__ __align__(16) uint16_t As[TM][LDK];
    __shared__ __align__(16) uint16_t Bs[TN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const bool a_k = sak == 1;      // A rows contiguous in k (else chunks run along m)
    const bool b_k = sbk == 1;      // B columns contiguous in k (else chunks run along n)
    float4_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
        uint16_t v[8];
        if (a_k) {
            const int r = tid >> 2, kk = (tid & 3) * 8, gm = m0 + r, gk = k0 + kk;
            const int nv = gm < M ? max(0, min(8, K - gk)) : 0;
            const uint16_t* p = A + (int64_t)min(gm, M - 1) * sam + (int64_t)gk;
            load8(p, 1, nv, nv == 8 && al16(p), v);
            *(uint4*)&As[r][kk] = *(const uint4*)v;
        } else {
            const int kk = tid >> 3, m8 = (tid & 7) * 8, gm = m0 + m8, gk = k0 + kk;
            const int nv = gk < K ? max(0, min(8, M - gm)) : 0;
            const uint16_t* p = A + (int64_t)gm * sam + (int64_t)min(gk, K - 1) * sak;
            load8(p, sam, nv, sam == 1 && nv == 8 && al16(p), v);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[m8 + i][kk] = v[i];
        }
        if (b_k) {
            const int n = tid >> 2, kk = (tid & 3) * 8, gn = n0 + n, gk = k0 + kk;
            const int nv = gn < N ? max(0, min(8, K - gk)) : 0;
            const uint16_t* p = B + (int64_t)gk + (int64_t)min(gn, N - 1) * sbn;
            load8(p, 1, nv, nv == 8 && al16(p), v);
            *(uint4*)&Bs[n][kk] = *(const uint4*)v;
        } else {
            const int kk = tid >> 3, n8 = (tid & 7) * 8, gn = n0 + n8, gk = k0 + kk;
            const int nv = gk < K ? max(0, min(8, N - gn)) : 0;
            const uint16_t* p = B + (int64_t)min(gk, K - 1) * sbk + (int64_t)gn * sbn;
            load8(p, sbn, nv, sbn == 1 && nv == 8 && al16(p), v);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[n8 + i][kk] = v[i];
        }
        __syncthreads();
        const int kq = 8 * (lane >> 4);
        bf16x8_t a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8_t*)&As[wm + 16 * i + (lane & 15)][kq];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8_t*)&Bs[wn + 16 * j + (lane & 15)][kq];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                const int col = n0 + wn + 16 * j + (lane & 15);
                if (row >= M || col >= N) continue;
                float v = acc[i][j][q];
                if (bias) v += bias[col];
                if (relu) v = v > 0.f ? v : 0.f;
                if (c32) {
                    float* p = c32 + (int64_t)row * ldc32 + col;
                    *p = beta32 ? *p + v : v;
                }
                if (c16) c16[(int64_t)row * ldc16 + col] = f2bf(v);
            }
}

__global__ void cast_bf16_kernel(const float* x, uint16_t* y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

__global__ void relu_grad_kernel(const float* g, const uint16_t* h, uint16_t* g16, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float v = g[i];
        if (h && !(bf2f(h[i]) > 0.f)) v = 0.f;
        g16[i] = f2bf(v);
    }
}

// one thread per column, rows summed in order (deterministic)
__global__ void colsum_kernel(const float* x, int rows, int cols, int64_t ld, float* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += x[(int64_t)i * ld + j];
    out[j] = s;
}

__global__ void mse_grad_kernel(const float* y, const float* t, float* g, float* partial, int64_t n)
{
    __shared__ float red[256];
    float s = 0.f;
    const float sc = 2.f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = y[i] - t[i];
        g[i] = sc * d;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x >> 1; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (partial && threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void finish_loss_kernel(const float* partial, int nb, int64_t n, float* loss)
{
    if (threadIdx.x != 0) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partial[b];
    loss[0] = s / (float)n;
}

__global__ void adam_kernel(float* w, const float* g, float* m, float* v, uint16_t* w16, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (w16) w16[i] = f2bf(wi);
    }
}

__global__ void ascent_kernel(float* x, const float* dx, const int32_t* active, int64_t N, int T, int D, int t0,
                              int dupd, float lr)
{
    const int64_t total = N * (int64_t)T * D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int d = (int)(i % D);
        const int64_t r = i / D;
        const int t = (int)(r % T);
        const int64_t nn = r / T;
        if (t < t0 || d >= dupd) continue;
        if (active && !active[nn]) continue;
        x[i] += lr * dx[i];
    }
}

}  // namespace stlmi_mlp

// ------------------------------------------------------------------ C ABI

using namespace stlmi_mlp;

// sets the library's thread-local message returned by stl_last_error()
void stlmi_set_error(const char* msg);

namespace {
stl_status mfail(stl_status s, const char* msg)
{
    stlmi_set_error(msg);
    return s;
}

int grid_for(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

stl_status launched(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: launch failed: %s", what, hipGetErrorString(e));
        return mfail(STL_E_HIP, buf);
    }
    return STL_OK;
}
}  // namespace

extern "C" stl_status stl_bf16_gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                                    int64_t sbn, int32_t M, int32_t N, int32_t K, const float* bias, int32_t relu,
                                    float* c32, int64_t ldc32, int32_t beta32, uint16_t* c16, int64_t ldc16,
                                    void* stream)
{
    if (M < 0 || N < 0 || K < 0) return mfail(STL_E_ARG, "stl_bf16_gemm: negative size");
    if (M == 0 || N == 0) return STL_OK;
    if ((K > 0 && (!A || !B)) || (!c32 && !c16)) return mfail(STL_E_ARG, "stl_bf16_gemm: null pointer");
    if ((int64_t)(M + TM - 1) / TM > 65535) return mfail(STL_E_UNSUPPORTED, "stl_bf16_gemm: M too large");
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, (hipStream_t)stream, A, sam, sak, B, sbk, sbn, M, N, K,
                       bias, relu, c32, ldc32, beta32, c16, ldc16);
    return launched("stl_bf16_gemm");
}

extern "C" stl_status stl_cast_bf16(const float* x, uint16_t* y, int64_t n, void* stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return mfail(STL_E_ARG, "stl_cast_bf16: bad arguments");
    if (n == 0) return STL_OK;
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, n);
    return launched("stl_cast_bf16");
}

extern "C" stl_status stl_relu_grad_bf16(const float* g, const uint16_t* h, uint16_t* g16, int64_t n, void* stream)
{
    if (n < 0 || (n > 0 && (!g || !g16))) return mfail(STL_E_ARG, "stl_relu_grad_bf16: bad arguments");
    if (n == 0) return STL_OK;
    hipLaunchKernelGGL(relu_grad_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, g, h, g16, n);
    return launched("stl_relu_grad_bf16");
}

extern "C" stl_status stl_colsum(const float* x, int32_t rows, int32_t cols, int64_t ld, float* out, void* stream)
{
    if (rows < 0 || cols < 0 || (cols > 0 && (!x || !out))) return mfail(STL_E_ARG, "stl_colsum: bad arguments");
    if (cols == 0) return STL_OK;
    hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256), dim3(256), 0, (hipStream_t)stream, x, rows, cols,
                       ld, out);
    return launched("stl_colsum");
}

extern "C" stl_status stl_mse_grad(const float* y, const float* t, float* g, float* loss, int64_t n, void* stream)
{
    if (n <= 0 || !y || !t || !g) return mfail(STL_E_ARG, "stl_mse_grad: bad arguments");
    // partial sums live in the first blocks of `loss` (caller passes >= 1 float);
    // the reduction uses a single block so that no scratch buffer is needed
    hipLaunchKernelGGL(mse_grad_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, y, t, g, loss, n);
    stl_status s = launched("stl_mse_grad");
    if (s != STL_OK || !loss) return s;
    hipLaunchKernelGGL(finish_loss_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, loss, 1, n, loss);
    return launched("stl_mse_grad");
}

extern "C" stl_status stl_adam_step(float* w, const float* g, float* m, float* v, uint16_t* w16, int64_t n, float lr,
                                    float b1, float b2, float eps, int32_t step, void* stream)
{
    if (n < 0 || step < 1 || (n > 0 && (!w || !g || !m || !v))) return mfail(STL_E_ARG, "stl_adam_step: bad arguments");
    if (n == 0) return STL_OK;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, w16, n, lr, b1,
                       b2, eps, c1, c2);
    return launched("stl_adam_step");
}

extern "C" stl_status stl_ascent_update(float* x, const float* dx, const int32_t* active, int64_t N, int32_t T,
                                        int32_t D, int32_t t0, int32_t d_upd, float lr, void* stream)
{
    if (N < 0 || T < 0 || D < 1 || (N > 0 && (!x || !dx))) return mfail(STL_E_ARG, "stl_ascent_update: bad arguments");
    const int64_t total = N * (int64_t)T * D;
    if (total == 0) return STL_OK;
    hipLaunchKernelGGL(ascent_kernel, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, x, dx, active, N, T,
                       D, t0, d_upd, lr);
    return launched("stl_ascent_update");
}
