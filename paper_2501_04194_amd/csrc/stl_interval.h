// Interval-vectorised evaluation (Sec. VI, after the smooth-mask equation):
// the robustness at t = 0 of one masked Always / Eventually for many
// (a, b) interval values at once, and its derivatives in a and b.
//
// One work-group takes 256 intervals (one per thread) and a group of up to
// IV_TB trajectories.  With the masking form each interval is an independent
// weighted reduction over a trajectory; the weights depend on the interval
// only, so a thread evaluates w_k, dw_k/da, dw_k/db once per offset and
// applies them to every trajectory of the group, whose terms
// E_j = 2^{z_j - R} (FP64, R the trajectory's largest exponent, as in the
// fused kernels) sit in LDS.
#pragma once

namespace stlmi {

constexpr int IV_NT = 256;
constexpr int IV_MAXT = 4096;
constexpr int IV_TB = 8;          // trajectories per work-group (IV_TB * T <= IV_MAXT)

struct IntervalArgs {
    const float* x;
    const float* a;
    const float* b;
    float* rho;
    float* ga;
    float* gb;
    int64_t B, N;
    int T, D, tb;       // tb: trajectories per work-group
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

// smooth value and derivatives of one interval on one trajectory, summed
// against the interval's own largest exponent (when every support term
// underflows against the trajectory's)
DEV void iv_own_ref(const MaskP& mp, const float* U, int lo, int hi, float sg, float bl, float beta, float& rho,
                    float& ga, float& gb)
{
    int zm = INT_MIN;
    bool any = false;
    for (int k = lo; k <= hi; ++k)
        if (mask_wk(mp, k) > 0.f) {
            zm = max(zm, (int)ceilf(fminf(fmaxf(sg * bl * U[k], -1e9f), 1e9f)));
            any = true;
        }
    if (!any) return;
    double S = 0.0, Sa = 0.0, Sb = 0.0;
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
    ga = (float)((double)(sg / beta) * (Sa / S));
    gb = (float)((double)(sg / beta) * (Sb / S));
}

template <int TB>
__global__ void __launch_bounds__(IV_NT) stl_interval_kernel(IntervalArgs A)
{
    __shared__ double E[IV_MAXT];     // [tb][T] terms
    __shared__ float U[IV_MAXT];      // [tb][T] predicate trace
    __shared__ int red[TB][IV_NT / 64];
    const int T = A.T, D = A.D, tb = A.tb;
    const float bl = A.beta * LOG2E, sg = (float)A.op_sg;
    const int64_t n = (int64_t)blockIdx.x * IV_NT + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t b0 = (int64_t)blockIdx.y * tb; b0 < A.B; b0 += (int64_t)gridDim.y * tb) {
        const int nb = (int)min<int64_t>(tb, A.B - b0);
        __syncthreads();                   // the previous group's terms are no longer read
        // predicate traces and each trajectory's reference exponent
        for (int t = 0; t < nb; ++t) {
            const float* xb = A.x + (b0 + t) * (int64_t)T * D;
            int zmax = INT_MIN;
            for (int j = threadIdx.x; j < T; j += IV_NT) {
                float u = 0.f;
                for (int d = 0; d < D; ++d) u = fmaf(A.w[d], xb[(int64_t)j * D + d], u);
                u -= A.c;
                U[t * T + j] = u;
                zmax = max(zmax, (int)ceilf(fminf(fmaxf(sg * bl * u, -1e9f), 1e9f)));
            }
            for (int d = 32; d > 0; d >>= 1) zmax = max(zmax, __shfl_xor(zmax, d));
            if (lane == 0) red[t][wv] = zmax;
        }
        __syncthreads();
        int R[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            int r = INT_MIN;
            if (t < nb)
                for (int k = 0; k < IV_NT / 64; ++k) r = max(r, red[t][k]);
            R[t] = r;
        }
        if (A.smooth)
            for (int i = threadIdx.x; i < nb * T; i += IV_NT) {
                int r = R[0];
#pragma unroll
                for (int t = 1; t < TB; ++t) r = i / T == t ? R[t] : r;
                E[i] = exp2d_neg(sg * bl * U[i] - (float)r);
            }
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
        float rho[TB], ga[TB], gb[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            rho[t] = -sg * A.rho_pad;
            ga[t] = 0.f;
            gb[t] = 0.f;
        }
        if (!A.smooth) {
            // max (Eventually) / min (Always) over the support
            bool any = false;
            float best[TB];
#pragma unroll
            for (int t = 0; t < TB; ++t) best[t] = 0.f;
            for (int k = lo; k <= hi; ++k) {
                if (!(mask_wk(mp, k) > 0.f)) continue;
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const float v = t < nb ? sg * U[t * T + k] : 0.f;
                    best[t] = (!any || v > best[t]) ? v : best[t];
                }
                any = true;
            }
            if (any)
#pragma unroll
                for (int t = 0; t < TB; ++t) rho[t] = sg * best[t];
        } else {
            double S[TB], Sa[TB], Sb[TB];
#pragma unroll
            for (int t = 0; t < TB; ++t) S[t] = Sa[t] = Sb[t] = 0.0;
            for (int k = lo; k <= hi; ++k) {
                float da, db;
                const float w = mask_wk(mp, k, &da, &db);
                if (!(w > 0.f)) continue;
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    const double e = t < nb ? E[t * T + k] : 0.0;
                    S[t] = fma((double)w, e, S[t]);
                    Sa[t] = fma((double)da, e, Sa[t]);
                    Sb[t] = fma((double)db, e, Sb[t]);
                }
            }
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                if (t >= nb) continue;
                if (S[t] > 0.0) {
                    rho[t] = sg * ((float)R[t] + log2d(S[t])) / bl;
                    ga[t] = (float)((double)(sg / A.beta) * (Sa[t] / S[t]));
                    gb[t] = (float)((double)(sg / A.beta) * (Sb[t] / S[t]));
                } else {
                    iv_own_ref(mp, U + t * T, lo, hi, sg, bl, A.beta, rho[t], ga[t], gb[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (t >= nb) continue;
            const int64_t o = (b0 + t) * A.N + n;
            A.rho[o] = rho[t];
            if (A.ga) {
                A.ga[o] = ga[t];
                A.gb[o] = gb[t];
            }
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
    const bool group = B > 2;             // one trajectory per work-group for tiny batches
    A.tb = group ? std::max(1, std::min(IV_TB, IV_MAXT / T)) : 1;
    A.op_sg = op_sg;
    A.smooth = smooth;
    A.beta = smooth ? beta : 1.f;
    A.mc = mc;
    A.meps = meps;
    A.c = c;
    A.rho_pad = rho_pad;
    for (int d = 0; d < 16; ++d) A.w[d] = d < D ? w[d] : 0.f;
    const int64_t groups = (B + A.tb - 1) / A.tb;
    const dim3 grid((unsigned)((N + IV_NT - 1) / IV_NT), (unsigned)std::min<int64_t>(groups, 65535)), block(IV_NT);
    if (group)
        hipLaunchKernelGGL(stl_interval_kernel<IV_TB>, grid, block, 0, s, A);
    else
        hipLaunchKernelGGL(stl_interval_kernel<1>, grid, block, 0, s, A);
    return hipGetLastError();
}

}  // namespace stlmi
