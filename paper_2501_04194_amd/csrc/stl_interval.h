// Interval-vectorised evaluation (Sec. VI, after the smooth-mask equation):
// the robustness at t = 0 of one masked Always / Eventually for many
// (a, b) interval values at once, and its derivatives in a and b.
//
// One work-group holds one trajectory's terms in LDS and one thread takes
// one interval.  With the masking form each interval is an independent
// weighted reduction over the trajectory, so the only sharing is the
// per-trajectory terms E_j = 2^{z_j - R} (FP64, R the trajectory's largest
// exponent, exactly as in the fused kernels); the weights are evaluated per
// (interval, offset) over the offsets where they can be positive.
#pragma once

namespace stlmi {

constexpr int IV_NT = 256;
constexpr int IV_MAXT = 4096;

struct IntervalArgs {
    const float* x;
    const float* a;
    const float* b;
    float* rho;
    float* ga;
    float* gb;
    int64_t B, N;
    int T, D;
    int op_sg;          // +1 Eventually (max), -1 Always (min)
    int smooth;
    float beta, mc, meps, c, rho_pad;
    float w[16];
};

// offsets outside [lo, hi] have w_k <= 0 for eps > 0: sig(c(k-a)) < eps below
// a + ln(eps)/c, and sig(c(k-b)) > 1 - eps above b - ln(eps)/c (one step of
// margin for rounding); eps = 0 leaves every offset
DEV void iv_range(float a, float b, float c, float eps, int T, int& lo, int& hi)
{
    lo = 0;
    hi = T - 1;
    if (eps > 0.f) {
        const float r = logf(eps) / c;                 // < 0
        const float fl = floorf(a + r) - 1.f, fh = ceilf(b - r) + 1.f;
        lo = fl > 0.f ? (fl < (float)T ? (int)fl : T) : 0;
        hi = fh < (float)(T - 1) ? (fh > -1.f ? (int)fh : -1) : T - 1;
    }
}

__global__ void __launch_bounds__(IV_NT) stl_interval_kernel(IntervalArgs A)
{
    __shared__ double E[IV_MAXT];
    __shared__ float U[IV_MAXT];
    __shared__ int red[IV_NT / 64];
    const int T = A.T, D = A.D;
    const float bl = A.beta * LOG2E, sg = (float)A.op_sg;
    const int64_t n = (int64_t)blockIdx.x * IV_NT + threadIdx.x;
  for (int64_t bi = blockIdx.y; bi < A.B; bi += gridDim.y) {
    const float* xb = A.x + bi * (int64_t)T * D;
    __syncthreads();                       // the previous trajectory's terms are no longer read
    // predicate trace and the trajectory's reference exponent
    int zmax = INT_MIN;
    for (int j = threadIdx.x; j < T; j += IV_NT) {
        float u = 0.f;
        for (int d = 0; d < D; ++d) u = fmaf(A.w[d], xb[(int64_t)j * D + d], u);
        u -= A.c;
        U[j] = u;
        if (A.smooth) zmax = max(zmax, (int)ceilf(fminf(fmaxf(sg * bl * u, -1e9f), 1e9f)));
    }
    for (int d = 32; d > 0; d >>= 1) zmax = max(zmax, __shfl_xor(zmax, d));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = zmax;
    __syncthreads();
    int R = red[0];
    for (int k = 1; k < IV_NT / 64; ++k) R = max(R, red[k]);
    if (A.smooth)
        for (int j = threadIdx.x; j < T; j += IV_NT) E[j] = exp2d_neg(sg * bl * U[j] - (float)R);
    __syncthreads();
    if (n >= A.N) continue;
    MaskP mp;
    mp.a = A.a[n];
    mp.b = A.b[n];
    mp.c = A.mc;
    mp.eps = A.meps;
    mp.unb = false;
    mp.band = 1.f - expf(-mp.c * (mp.b - mp.a));
    int lo, hi;
    iv_range(mp.a, mp.b, mp.c, mp.eps, T, lo, hi);
    float rho = -sg * A.rho_pad, ga = 0.f, gb = 0.f;
    if (!A.smooth) {
        // max (Eventually) / min (Always) over the support
        bool any = false;
        float best = 0.f;
        for (int k = lo; k <= hi; ++k) {
            if (!(mask_wk(mp, k) > 0.f)) continue;
            const float v = sg * U[k];
            if (!any || v > best) best = v;
            any = true;
        }
        if (any) rho = sg * best;
    } else {
        double S = 0.0, Sa = 0.0, Sb = 0.0;
        for (int k = lo; k <= hi; ++k) {
            float da, db;
            const float w = mask_wk(mp, k, &da, &db);
            if (!(w > 0.f)) continue;
            const double e = E[k];
            S = fma((double)w, e, S);
            Sa = fma((double)da, e, Sa);
            Sb = fma((double)db, e, Sb);
        }
        if (S > 0.0) {
            rho = sg * ((float)R + log2d(S)) / bl;
            ga = (float)((double)(sg / A.beta) * (Sa / S));
            gb = (float)((double)(sg / A.beta) * (Sb / S));
        } else {
            // every support term underflowed against the trajectory's reference:
            // this interval again against its own largest exponent
            int zm = INT_MIN;
            bool any = false;
            for (int k = lo; k <= hi; ++k)
                if (mask_wk(mp, k) > 0.f) {
                    zm = max(zm, (int)ceilf(fminf(fmaxf(sg * bl * U[k], -1e9f), 1e9f)));
                    any = true;
                }
            if (any) {
                S = Sa = Sb = 0.0;
                for (int k = lo; k <= hi; ++k) {
                    float da, db;
                    const float w = mask_wk(mp, k, &da, &db);
                    if (!(w > 0.f)) continue;
                    const double e = exp2d_neg(sg * bl * U[k] - (float)zm);
                    S = fma((double)w, e, S);
                    Sa = fma((double)da, e, Sa);
                    Sb = fma((double)db, e, Sb);
                }
                rho = sg * ((float)zm + log2d(S)) / bl;
                ga = (float)((double)(sg / A.beta) * (Sa / S));
                gb = (float)((double)(sg / A.beta) * (Sb / S));
            }
        }
    }
    const int64_t o = bi * A.N + n;
    A.rho[o] = rho;
    if (A.ga) {
        A.ga[o] = ga;
        A.gb[o] = gb;
    }
  }
}

int interval_max_T() { return IV_MAXT; }

hipError_t launch_interval_sweep(int op_sg, int smooth, float beta, float mc, float meps, int D, const float* w,
                                 float c, float rho_pad, const float* x, int64_t B, int T, const float* a,
                                 const float* b, int64_t N, float* rho, float* ga, float* gb, hipStream_t s)
{
    IntervalArgs A;
    A.x = x;
    A.a = a;
    A.b = b;
    A.rho = rho;
    A.ga = ga;
    A.gb = gb;
    A.B = B;
    A.N = N;
    A.T = T;
    A.D = D;
    A.op_sg = op_sg;
    A.smooth = smooth;
    A.beta = smooth ? beta : 1.f;
    A.mc = mc;
    A.meps = meps;
    A.c = c;
    A.rho_pad = rho_pad;
    for (int d = 0; d < 16; ++d) A.w[d] = d < D ? w[d] : 0.f;
    const dim3 grid((unsigned)((N + IV_NT - 1) / IV_NT), (unsigned)std::min<int64_t>(B, 65535)), block(IV_NT);
    hipLaunchKernelGGL(stl_interval_kernel, grid, block, 0, s, A);
    return hipGetLastError();
}

}  // namespace stlmi
