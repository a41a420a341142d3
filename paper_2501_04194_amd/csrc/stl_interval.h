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
            bool pos = false;                 // some offset has a positive weight
            for (int k = lo; k <= hi; ++k) {
                float da, db;
                const float w = mask_wk(mp, k, &da, &db);
                if (!(w > 0.f)) continue;
                pos = true;
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
                    const double iS = (double)(sg / A.beta) / S[t];   // one division for both ratios
                    ga[t] = (float)(iS * Sa[t]);
                    gb[t] = (float)(iS * Sb[t]);
                } else if (pos) {
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

// Smooth sweep of one or two trajectories: with one thread per interval the
// launch holds too few waves to cover the latency of each thread's serial
// walk over its offsets, so IVS_LPI consecutive lanes share an interval (lane
// r takes offsets lo + r, lo + r + IVS_LPI, ...) and add their partial sums
// with lane exchanges; the first lane of the group writes the outputs.
constexpr int IVS_LPI = 4;

__global__ void __launch_bounds__(IV_NT) stl_interval_split_kernel(IntervalArgs A)
{
    __shared__ double E[IV_MAXT];
    __shared__ float U[IV_MAXT];
    __shared__ int red[IV_NT / 64];
    const int T = A.T, D = A.D;
    const float bl = A.beta * LOG2E, sg = (float)A.op_sg;
    const int64_t gi = (int64_t)blockIdx.x * IV_NT + threadIdx.x;
    const int64_t n = gi / IVS_LPI;
    const int r = (int)(gi % IVS_LPI);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool nok = n < A.N;
    MaskP mp;
    mp.a = nok ? A.a[n] : 0.f;
    mp.b = nok ? A.b[n] : 1.f;
    mp.c = A.mc;
    mp.eps = A.meps;
    mp.unb = false;
    mp.band = 1.f - expf(-mp.c * (mp.b - mp.a));
    int lo, hi;
    iv_range(mp.a, mp.b, mp.c, mp.eps, T, lo, hi);
    for (int64_t b = blockIdx.y; b < A.B; b += gridDim.y) {
        __syncthreads();                   // the previous trajectory's terms are no longer read
        const float* xb = A.x + b * (int64_t)T * D;
        int zmax = INT_MIN;
        for (int j = threadIdx.x; j < T; j += IV_NT) {
            float u = 0.f;
            for (int d = 0; d < D; ++d) u = fmaf(A.w[d], xb[(int64_t)j * D + d], u);
            u -= A.c;
            U[j] = u;
            zmax = max(zmax, (int)ceilf(fminf(fmaxf(sg * bl * u, -1e9f), 1e9f)));
        }
        for (int d = 32; d > 0; d >>= 1) zmax = max(zmax, __shfl_xor(zmax, d));
        if (lane == 0) red[wv] = zmax;
        __syncthreads();
        int R = INT_MIN;
        for (int k = 0; k < IV_NT / 64; ++k) R = max(R, red[k]);
        for (int j = threadIdx.x; j < T; j += IV_NT) E[j] = exp2d_neg(sg * bl * U[j] - (float)R);
        __syncthreads();
        double S = 0.0, Sa = 0.0, Sb = 0.0;
        int pos = 0;
        if (nok)
            for (int k = lo + r; k <= hi; k += IVS_LPI) {
                float da, db;
                const float w = mask_wk(mp, k, &da, &db);
                if (!(w > 0.f)) continue;
                pos = 1;
                const double e = E[k];
                S = fma((double)w, e, S);
                Sa = fma((double)da, e, Sa);
                Sb = fma((double)db, e, Sb);
            }
#pragma unroll
        for (int d = 1; d < IVS_LPI; d <<= 1) {
            S += __shfl_xor(S, d);
            Sa += __shfl_xor(Sa, d);
            Sb += __shfl_xor(Sb, d);
            pos |= __shfl_xor(pos, d);
        }
        if (!nok || r != 0) continue;
        float rho = -sg * A.rho_pad, ga = 0.f, gb = 0.f;
        if (S > 0.0) {
            rho = sg * ((float)R + log2d(S)) / bl;
            const double iS = (double)(sg / A.beta) / S;
            ga = (float)(iS * Sa);
            gb = (float)(iS * Sb);
        } else if (pos) {
            iv_own_ref(mp, U, lo, hi, sg, bl, A.beta, rho, ga, gb);
        }
        const int64_t o = b * A.N + n;
        A.rho[o] = rho;
        if (A.ga) {
            A.ga[o] = ga;
            A.gb[o] = gb;
        }
    }
}

// ------------------------------------------------------------------ batched sweep on the matrix cores

// For many trajectories the smooth sweep is a dense contraction: with
// E_bk = 2^{z_bk - R_b} (z = +-beta log2(e) u, R_b the trajectory's largest
// exponent), S_bn = sum_k w_nk E_bk and the same sums with dw/da, dw/db are
// three products of the [B, T] term matrix with the [T, N] weight matrices,
// which v_mfma_f32_16x16x4f32 computes 16 x 16 outputs at a time (K = 4 per
// instruction).  A wave owns IVM_NT tiles of 16 intervals: it evaluates their
// weights once, as B operands (lane l: interval n0 + 16j + l%16, offsets
// 4s + l/16), then walks tiles of 16 trajectories, whose terms are the A
// operands (lane l: trajectory b0 + l%16, offsets 4s + l/16) shared by all
// its interval tiles.  Result lane l, register q of tile j holds trajectory
// b0 + 4(l/16) + q, interval n0 + 16j + l%16.  The terms are fp32 in
// (0, 1]; an output whose sum falls below 2^-100 (its support only reaches
// terms near or under the fp32 range) is redone by iv_own_ref from the
// predicate trace kept in LDS.
constexpr int IVM_MAXT = 64;
constexpr int IVM_NT = 2;          // 16-interval tiles per wave (the terms of a trajectory tile serve them all)

typedef float iv_f4 __attribute__((ext_vector_type(4)));

template <int KS>
__global__ void __launch_bounds__(IV_NT) stl_interval_mfma_kernel(IntervalArgs A)
{
    __shared__ float Ush[IV_NT / 64][16 * IVM_MAXT];   // per wave: 16 predicate traces
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, row4 = lane >> 4;
    const int T = A.T, D = A.D;
    const float bl = A.beta * LOG2E, sg = (float)A.op_sg;
    // this wave's IVM_NT interval tiles: intervals n0 + 16 j + col
    const int64_t n0 = ((int64_t)blockIdx.x * (IV_NT / 64) + wv) * (16 * IVM_NT);
    MaskP mp[IVM_NT];
    bool nok[IVM_NT];
    int lo[IVM_NT], hi[IVM_NT], pos[IVM_NT];
    float W[IVM_NT][KS], Wa[IVM_NT][KS], Wb[IVM_NT][KS];
#pragma unroll
    for (int j = 0; j < IVM_NT; ++j) {
        const int64_t n = n0 + 16 * j + col;
        nok[j] = n < A.N;
        mp[j].a = nok[j] ? A.a[n] : 0.f;
        mp[j].b = nok[j] ? A.b[n] : 1.f;
        mp[j].c = A.mc;
        mp[j].eps = A.meps;
        mp[j].unb = false;
        mp[j].band = 1.f - expf(-mp[j].c * (mp[j].b - mp[j].a));
        int p = 0;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + row4;
            float da = 0.f, db = 0.f, w = 0.f;
            if (nok[j] && k < T) w = mask_wk(mp[j], k, &da, &db);
            W[j][s] = w;
            Wa[j][s] = da;
            Wb[j][s] = db;
            p |= w > 0.f;
        }
        // an interval whose support misses [0, T) has the empty-window value on
        // every trajectory: no sum and no fallback for it
        p |= __shfl_xor(p, 16);
        p |= __shfl_xor(p, 32);
        pos[j] = p;
        iv_range(mp[j].a, mp[j].b, mp[j].c, mp[j].eps, T, lo[j], hi[j]);
    }
    float* Uw = Ush[wv];
    const float ib = sg / A.beta;
    for (int64_t b0 = (int64_t)blockIdx.y * 16; b0 < A.B; b0 += (int64_t)gridDim.y * 16) {
        const int64_t bt = b0 + col;                  // this lane's A-operand trajectory
        const bool bok = bt < A.B;
        const float* xb = A.x + (bok ? bt : 0) * (int64_t)T * D;
        float z[KS];
        int zm = INT_MIN;
        __syncthreads();                              // the previous tile's traces are no longer read
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + row4;
            float u = 0.f;
            if (bok && k < T) {
                for (int d = 0; d < D; ++d) u = fmaf(A.w[d], xb[(int64_t)k * D + d], u);
                u -= A.c;
                zm = max(zm, (int)ceilf(fminf(fmaxf(sg * bl * u, -1e9f), 1e9f)));
            }
            z[s] = sg * bl * u;
            Uw[col * IVM_MAXT + k] = u;               // k < 4 KS <= IVM_MAXT
        }
        zm = max(zm, __shfl_xor(zm, 16));
        zm = max(zm, __shfl_xor(zm, 32));
        iv_f4 s0[IVM_NT], sa[IVM_NT], sb[IVM_NT];
#pragma unroll
        for (int j = 0; j < IVM_NT; ++j) s0[j] = sa[j] = sb[j] = iv_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + row4;
            const float e = (bok && k < T) ? exp2f(z[s] - (float)zm) : 0.f;
#pragma unroll
            for (int j = 0; j < IVM_NT; ++j) {
                s0[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(e, W[j][s], s0[j], 0, 0, 0);
                sa[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(e, Wa[j][s], sa[j], 0, 0, 0);
                sb[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(e, Wb[j][s], sb[j], 0, 0, 0);
            }
        }
        __syncthreads();                              // traces visible to every lane of the wave
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * row4 + q;               // trajectory b0 + r
            const int Rb = __shfl(zm, r);
            const int64_t b = b0 + r;
            if (b >= A.B) continue;
#pragma unroll
            for (int j = 0; j < IVM_NT; ++j) {
                if (!nok[j]) continue;
                float rho = -sg * A.rho_pad, ga = 0.f, gb = 0.f;
                const float S = s0[j][q];
                if (S >= 0x1p-100f) {
                    rho = sg * ((float)Rb + log2f(S)) / bl;
                    const float iS = 1.f / S;
                    ga = ib * (sa[j][q] * iS);
                    gb = ib * (sb[j][q] * iS);
                } else if (pos[j]) {
                    iv_own_ref(mp[j], Uw + r * IVM_MAXT, lo[j], hi[j], sg, bl, A.beta, rho, ga, gb);
                }
                const int64_t o = b * A.N + n0 + 16 * j + col;
                A.rho[o] = rho;
                if (A.ga) {
                    A.ga[o] = ga;
                    A.gb[o] = gb;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ pSTL descent

// Gradient descent on the parametric-STL mining loss (Sec. VII-B)
//   L(a, b) = mean_i max(-rho_i, 0) + gamma (a - b),
//   rho_i = robustness at t = 0 of op_[aT, bT](w . x_i - c) with a smooth mask,
// over a = sig(p_a), b = sig(p_b) (fractions of the horizon), the mask
// steepness and beta annealed from (c0, beta0) to (c1, beta1) along a sigmoid
// schedule.  The whole loop runs in one work-group: the dataset's predicate
// traces stay in LDS, each step evaluates the mask weights once (one thread
// per offset) and every signal's rho, d rho/da, d rho/db (threads over
// signals), reduces the hinge gradient in a fixed order and updates (p_a, p_b)
// in LDS; no launch per step.
constexpr int PD_MAXBT = 12288;

struct DescentArgs {
    const float* x;
    float* p;            // [2] logits of (a, b), read and written
    float* loss;         // [steps] or NULL
    int B, T, D, steps, op_sg;
    float eps, c0, c1, beta0, beta1, lr, gamma, c;
    float w[16];
};

DEV float sched(int k, int steps, float lo, float hi)
{
    const float u = (float)k / (float)max(1, steps - 1) - 0.5f;
    return lo + (hi - lo) / (1.f + expf(-12.f * u));
}

__global__ void __launch_bounds__(IV_NT) stl_pstl_descent_kernel(DescentArgs A)
{
    __shared__ float U[PD_MAXBT];
    __shared__ float Wt[IV_MAXT / 4][3];     // w_j, dw_j/da, dw_j/db for the current step
    __shared__ double red[3][IV_NT / 64];
    __shared__ float pab[2];
    const int B = A.B, T = A.T, D = A.D;
    const float sg = (float)A.op_sg;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < B * T; i += IV_NT) {
        float u = 0.f;
        for (int d = 0; d < D; ++d) u = fmaf(A.w[d], A.x[(int64_t)i * D + d], u);
        U[i] = u - A.c;
    }
    if (threadIdx.x < 2) pab[threadIdx.x] = A.p[threadIdx.x];
    __syncthreads();
    for (int k = 0; k < A.steps; ++k) {
        const float c = sched(k, A.steps, A.c0, A.c1), beta = sched(k, A.steps, A.beta0, A.beta1);
        const float bl = beta * LOG2E;
        const float af = 1.f / (1.f + expf(-pab[0])), bf = 1.f / (1.f + expf(-pab[1]));
        MaskP mp;
        mp.a = af * (float)T;
        mp.b = bf * (float)T;
        mp.c = c;
        mp.eps = A.eps;
        mp.unb = false;
        mp.band = 1.f - expf(-c * (mp.b - mp.a));
        for (int j = threadIdx.x; j < T; j += IV_NT) {
            float da, db;
            Wt[j][0] = mask_wk(mp, j, &da, &db);
            Wt[j][1] = da;
            Wt[j][2] = db;
        }
        __syncthreads();
        double ha = 0.0, hb = 0.0, hl = 0.0;      // this thread's hinge sums
        for (int i = threadIdx.x; i < B; i += IV_NT) {
            const float* u = U + i * T;
            int R = INT_MIN;
            bool any = false;
            for (int j = 0; j < T; ++j)
                if (Wt[j][0] > 0.f) {
                    R = max(R, (int)ceilf(fminf(fmaxf(sg * bl * u[j], -1e9f), 1e9f)));
                    any = true;
                }
            float rho = -sg * 1e6f, ga = 0.f, gb = 0.f;
            if (any) {
                double S = 0.0, Sa = 0.0, Sb = 0.0;
                for (int j = 0; j < T; ++j) {
                    const float wj = Wt[j][0];
                    if (!(wj > 0.f)) continue;
                    const double e = exp2d_neg(sg * bl * u[j] - (float)R);
                    S = fma((double)wj, e, S);
                    Sa = fma((double)Wt[j][1], e, Sa);
                    Sb = fma((double)Wt[j][2], e, Sb);
                }
                rho = sg * ((float)R + log2d(S)) / bl;
                ga = (float)((double)(sg / beta) * (Sa / S));
                gb = (float)((double)(sg / beta) * (Sb / S));
            }
            if (rho < 0.f) {
                ha -= ga;
                hb -= gb;
                hl -= rho;
            }
        }
        for (int d = 32; d > 0; d >>= 1) {
            ha += __shfl_xor(ha, d);
            hb += __shfl_xor(hb, d);
            hl += __shfl_xor(hl, d);
        }
        if (lane == 0) {
            red[0][wv] = ha;
            red[1][wv] = hb;
            red[2][wv] = hl;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double sa = 0.0, sb = 0.0, sl = 0.0;
            for (int q = 0; q < IV_NT / 64; ++q) {
                sa += red[0][q];
                sb += red[1][q];
                sl += red[2][q];
            }
            // d L / d a_frac = T mean(-[rho < 0] d rho / d a_steps) + gamma (b: - gamma)
            const float dla = (float)(T * sa / B) + A.gamma, dlb = (float)(T * sb / B) - A.gamma;
            if (A.loss) A.loss[k] = (float)(sl / B) + A.gamma * (af - bf);
            pab[0] -= A.lr * dla * af * (1.f - af);
            pab[1] -= A.lr * dlb * bf * (1.f - bf);
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) A.p[threadIdx.x] = pab[threadIdx.x];
}

int pstl_max_BT() { return PD_MAXBT; }

hipError_t launch_pstl_descent(const float* x, int B, int T, int D, const float* w, float c, int op_sg, float eps,
                               float c0, float c1, float beta0, float beta1, int steps, float lr, float gamma,
                               float* p, float* loss, hipStream_t s)
{
    DescentArgs A;
    A.x = x;
    A.p = p;
    A.loss = loss;
    A.B = B;
    A.T = T;
    A.D = D;
    A.steps = steps;
    A.op_sg = op_sg;
    A.eps = eps;
    A.c0 = c0;
    A.c1 = c1;
    A.beta0 = beta0;
    A.beta1 = beta1;
    A.lr = lr;
    A.gamma = gamma;
    A.c = c;
    for (int d = 0; d < 16; ++d) A.w[d] = d < D ? w[d] : 0.f;
    hipLaunchKernelGGL(stl_pstl_descent_kernel, dim3(1), dim3(IV_NT), 0, s, A);
    return hipGetLastError();
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
    if (smooth && T <= IVM_MAXT && B >= 16) {
        // batched smooth sweep: matrix cores, 64 IVM_NT intervals per work-group; enough
        // trajectory-tile groups for about 8192 work-groups
        const int64_t nx = (N + 64 * IVM_NT - 1) / (64 * IVM_NT), tiles = (B + 15) / 16;
        const int64_t ny = std::max<int64_t>(1, std::min<int64_t>(tiles, std::min<int64_t>(65535, (8192 + nx - 1) / nx)));
        const dim3 g((unsigned)nx, (unsigned)ny), blk(IV_NT);
        if (T <= 20)
            hipLaunchKernelGGL(stl_interval_mfma_kernel<5>, g, blk, 0, s, A);
        else if (T <= 32)
            hipLaunchKernelGGL(stl_interval_mfma_kernel<8>, g, blk, 0, s, A);
        else
            hipLaunchKernelGGL(stl_interval_mfma_kernel<16>, g, blk, 0, s, A);
        return hipGetLastError();
    }
    if (smooth && !group) {
        const dim3 g((unsigned)((N * IVS_LPI + IV_NT - 1) / IV_NT), (unsigned)std::min<int64_t>(B, 65535)),
            blk(IV_NT);
        hipLaunchKernelGGL(stl_interval_split_kernel, g, blk, 0, s, A);
        return hipGetLastError();
    }
    const int64_t groups = (B + A.tb - 1) / A.tb;
    const dim3 grid((unsigned)((N + IV_NT - 1) / IV_NT), (unsigned)std::min<int64_t>(groups, 65535)), block(IV_NT);
    if (group)
        hipLaunchKernelGGL(stl_interval_kernel<IV_TB>, grid, block, 0, s, A);
    else
        hipLaunchKernelGGL(stl_interval_kernel<1>, grid, block, 0, s, A);
    return hipGetLastError();
}

}  // namespace stlmi
