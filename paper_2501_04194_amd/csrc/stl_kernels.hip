// HIP kernels for STL robustness traces on gfx950 (MI355X).
//
// One work-group owns one trajectory at a time (a persistent grid pulls
// trajectory indices from a counter).  Every node trace of the formula lives
// in an on-chip slot (LDS, or a per-work-group region of the workspace when
// the trajectory is too long for LDS) and the plan's instructions run in
// topological order, each one a work-group-cooperative parallel pass over the
// timesteps.  Only x is read and only the root trace (forward) or dx and the
// mask-bound partial sums (backward) are written to HBM.
//
// Operators (arXiv 2501.04194):
//   windows over [a,b] (Sec. IV-B) are evaluated by van Herk / Gil-Werman
//   block decomposition: blocks of K = b-a+1 positions, block-prefix and
//   block-suffix reductions, and every window is suffix(start) (+) prefix(end)
//   of two adjacent blocks.  The masked (T+K) x T array of the paper is never
//   formed.  Unbounded windows are suffix scans.
//   Smooth windows (Sec. III-C) use the same decomposition on "scaled pairs"
//   (s, r) = s * 2^r, so sums of exp(beta u) never overflow whatever the
//   signal range; beta is folded into base-2 exponents.
//   The smooth time mask (Sec. VI) splits into a constant-weight core (a van
//   Herk window) plus two sigmoid bands summed term by term.
//   Until (Sec. IV-C) runs the running min over the inner index once per
//   output (no 3-D array): hard with compare-selects, smooth with running
//   scaled sums; its adjoint uses checkpointed recomputation.
//   Hard min/max carry the element index so ties resolve to the lowest time
//   index, matching the gradient routing rule.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <algorithm>
#include "stl_plan.h"

namespace stlmi {

#define DEV static __device__ __forceinline__

constexpr float LOG2E = 1.4426950408889634f;
constexpr int MAX_NT = 512;
constexpr int PAD_NEUTRAL = 0, PAD_LAST = 1, PAD_CONST = 2;

// ------------------------------------------------------------------ types

// scaled pair: value = s * 2^r
struct SP {
    float s;
    int r;
};
constexpr int SP_NEG = -(1 << 29);

DEV SP sp_zero() { return SP{0.f, SP_NEG}; }

DEV SP sp_leaf(float z)  // 2^z
{
    float c = ceilf(fminf(fmaxf(z, -1e9f), 1e9f));
    return SP{exp2f(z - c), (int)c};
}

DEV SP sp_add(SP a, SP b)
{
    int m = max(a.r, b.r);
    return SP{ldexpf(a.s, a.r - m) + ldexpf(b.s, b.r - m), m};
}

DEV float sp_log2(SP a) { return (float)a.r + log2f(a.s); }

DEV int clampe(long long e) { return (int)(e < -100000 ? -100000 : (e > 100000 ? 100000 : e)); }

// value of a * 2^z as a float (exact exponent bookkeeping, no intermediate overflow)
DEV float sp_times_exp2(SP a, float z)
{
    float c = ceilf(fminf(fmaxf(z, -1e9f), 1e9f));
    return ldexpf(a.s * exp2f(z - c), clampe((long long)a.r + (long long)c));
}

// scaled pair with a double mantissa: signed sums of many terms (adjoints)
struct SPD {
    double s;
    int r;
};

DEV SPD spd_add(SPD a, SP b)
{
    int m = max(a.r, b.r);
    return SPD{ldexp(a.s, a.r - m) + ldexp((double)b.s, b.r - m), m};
}

// renormalised float scaled pair of a double-mantissa pair
DEV SP spd_to_sp(SPD a)
{
    int e;
    const double mant = frexp(a.s, &e);
    return SP{(float)mant, clampe((long long)a.r + e)};
}

// value with index: hard max with ties to the lowest index
struct VI {
    float v;
    int i;
};

DEV VI vi_best(VI a, VI b)
{
    return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}

struct OpSP {
    __device__ __forceinline__ SP operator()(SP a, SP b) const { return sp_add(a, b); }
};
struct OpVI {
    __device__ __forceinline__ VI operator()(VI a, VI b) const { return vi_best(a, b); }
};
struct OpD {
    __device__ __forceinline__ double operator()(double a, double b) const { return a + b; }
};
struct OpF {
    __device__ __forceinline__ float operator()(float a, float b) const { return a + b; }
};

// ------------------------------------------------------------------ scans

struct Shared {
    double scan[MAX_NT];
    int flag[MAX_NT];
    int ints[8];
    float f[8];
    int scan_pos, scan_min;      // flag-scan fix-up: next row index of this work-group, first set flag
};

// storage index maps for scanned arrays: identity, or one pad element after
// every 8 (conflict-free LDS access when each lane owns 8 consecutive elements)
struct IdxId {
    __device__ __forceinline__ int operator()(int p) const { return p; }
};
struct IdxPad {
    __device__ __forceinline__ int operator()(int p) const { return p + (p >> 3); }
};

// In-place inclusive scan of x[0..n) within segments.  Forward scans have
// segment heads at positions with (p + off) % K == 0; reverse scans at
// (p + off) % K == K-1 and at n-1.  K <= 0 means one segment.  Each thread
// scans a contiguous chunk sequentially; chunk aggregates are combined with a
// segmented Hillis-Steele pass; the carry is then applied to each chunk's
// head part.  Must be called by every thread of the work-group.
template <class T, class Op, class SH, class IX = IdxId>
DEV void seg_scan(T* x, int n, int K, bool rev, T ident, Op op, SH& sh, int off = 0, IX ix = IX())
{
    const int tid = threadIdx.x, nt = blockDim.x;
    T* shv = reinterpret_cast<T*>(sh.scan);
    const int C = (n + nt - 1) / nt;
    const int c0 = min(n, tid * C), c1 = min(n, c0 + C);
    T acc = ident;
    int head = 0;
    if (c0 < c1) {
        if (!rev) {
            int rem = K > 0 ? (c0 + off) % K : c0;
            for (int p = c0; p < c1; ++p) {
                bool h = K > 0 ? (rem == 0) : (p == 0);
                T v = x[ix(p)];
                acc = h ? v : op(acc, v);
                head |= h;
                x[ix(p)] = acc;
                if (K > 0 && ++rem == K) rem = 0;
            }
        } else {
            int rem = K > 0 ? (c1 - 1 + off) % K : 0;
            for (int p = c1 - 1; p >= c0; --p) {
                bool h = (p == n - 1) || (K > 0 && rem == K - 1);
                T v = x[ix(p)];
                acc = h ? v : op(v, acc);
                head |= h;
                x[ix(p)] = acc;
                if (K > 0) rem = rem == 0 ? K - 1 : rem - 1;
            }
        }
    }
    shv[tid] = acc;
    sh.flag[tid] = head;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {
        T a = shv[tid];
        int f = sh.flag[tid];
        int src = rev ? tid + d : tid - d;
        if (!f && (rev ? src < nt : src >= 0)) {
            T b = shv[src];
            a = rev ? op(a, b) : op(b, a);
            f = sh.flag[src];
        }
        __syncthreads();
        shv[tid] = a;
        sh.flag[tid] = f;
        __syncthreads();
    }
    const int nb = rev ? tid + 1 : tid - 1;
    if (c0 < c1 && nb >= 0 && nb < nt) {
        T carry = shv[nb];
        if (!rev) {
            int rem = K > 0 ? (c0 + off) % K : c0;
            for (int p = c0; p < c1; ++p) {
                bool h = K > 0 ? (rem == 0) : (p == 0);
                if (h) break;
                x[ix(p)] = op(carry, x[ix(p)]);
                if (K > 0 && ++rem == K) rem = 0;
            }
        } else {
            int rem = K > 0 ? (c1 - 1 + off) % K : 0;
            for (int p = c1 - 1; p >= c0; --p) {
                bool h = (p == n - 1) || (K > 0 && rem == K - 1);
                if (h) break;
                x[ix(p)] = op(x[ix(p)], carry);
                if (K > 0) rem = rem == 0 ? K - 1 : rem - 1;
            }
        }
    }
    __syncthreads();
}

// deterministic work-group sum of one float per thread
DEV float wg_sum(float v, Shared& sh)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    float* f = reinterpret_cast<float*>(sh.scan);
    f[tid] = v;
    __syncthreads();
    for (int s = nt >> 1; s > 0; s >>= 1) {
        if (tid < s) f[tid] += f[tid + s];
        __syncthreads();
    }
    float r = f[0];
    __syncthreads();
    return r;
}

DEV int lower_bound_i(const int* a, int n, int key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ context


struct Env {
    const DevPlan* P;
    const float* x;    // this trajectory, [L, D]
    const float* params;
    int L, Lc, D;
    float* arena;      // slots
    float* scr;        // op scratch (SCR_FLOATS(Lc) floats)
    Shared* sh;
};

// scratch layout (floats): everything an operator needs, in units of Lc
#define SCR_UNITS 16
DEV float* S(const Env& e, int unit) { return e.scr + (size_t)unit * e.Lc; }

DEV float* slot(const Env& e, int s) { return e.arena + (size_t)s * e.Lc; }

DEV float pbeta(const Env& e, const Instr& I) { return I.beta >= 0 ? e.params[I.beta] : 1.f; }

// ------------------------------------------------------------------ pointwise ops

DEV void op_pred_fwd(const Env& e, const Instr& I, float* out)
{
    const float* cf = e.P->coef + I.coef;
    const int D = e.D;
    if (I.kind == K_LIN) {
        const float c = cf[0];
        for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
            const float* xr = e.x + (size_t)t * D;
            float s = 0.f;
            for (int d = 0; d < D; ++d) s = fmaf(cf[1 + d], xr[d], s);
            out[t] = s - c;
        }
    } else {
        const int m = (int)cf[0];
        const float r = cf[1], sg = cf[2];
        for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
            const float* xr = e.x + (size_t)t * D;
            float q = 0.f;
            for (int i = 0; i < m; ++i) {
                float z = -cf[3 + i];
                for (int d = 0; d < D; ++d) z = fmaf(cf[7 + i * D + d], xr[d], z);
                q = fmaf(z, z, q);
            }
            out[t] = sg * (sqrtf(q) - r);
        }
    }
}

// d/dx of all predicates: dx[t, d] = sum_p dmu_p/dx_d * g_p[t]
DEV void op_dx(const Env& e, float* dx)
{
    const DevPlan& P = *e.P;
    const int D = e.D;
    for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
        const float* xr = e.x + (size_t)t * D;
        float acc[MAX_D];
        for (int d = 0; d < D; ++d) acc[d] = 0.f;
        for (int p = 0; p < P.n_pred; ++p) {
            const Instr& I = P.ins[P.pred_ins[p]];
            const float g = slot(e, I.g_out)[t];
            const float* cf = P.coef + I.coef;
            if (I.kind == K_LIN) {
                for (int d = 0; d < D; ++d) acc[d] = fmaf(cf[1 + d], g, acc[d]);
            } else {
                const int m = (int)cf[0];
                const float sg = cf[2];
                float z[4];
                float q = 0.f;
                for (int i = 0; i < m; ++i) {
                    z[i] = -cf[3 + i];
                    for (int d = 0; d < D; ++d) z[i] = fmaf(cf[7 + i * D + d], xr[d], z[i]);
                    q = fmaf(z[i], z[i], q);
                }
                if (q > 0.f) {
                    const float k = sg * g / sqrtf(q);
                    for (int d = 0; d < D; ++d) {
                        float s = 0.f;
                        for (int i = 0; i < m; ++i) s = fmaf(cf[7 + i * D + d], z[i], s);
                        acc[d] = fmaf(k, s, acc[d]);
                    }
                }
            }
        }
        for (int d = 0; d < D; ++d) dx[(size_t)t * D + d] = acc[d];
    }
}

DEV void op_nary_fwd(const Env& e, const Instr& I, const int8_t* ch, float* out)
{
    const float sg = (I.flags & F_MIN) ? -1.f : 1.f;
    const int n = I.nch;
    const float* c[MAX_NCH];
    for (int k = 0; k < MAX_NCH; ++k) c[k] = slot(e, ch[k < n ? k : 0]);
    if (!(I.flags & F_SMOOTH)) {
        for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
            float best = sg * c[0][t];
            for (int k = 1; k < n; ++k) {
                float v = sg * c[k][t];
                if (v > best) best = v;
            }
            out[t] = sg * best;
        }
    } else if (I.flags & F_SOFT) {
        // softmax-weighted mean of the oriented values (Sec. III-C)
        const float bl = pbeta(e, I) * LOG2E;
        for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
            float v[MAX_NCH];
            float m = -INFINITY;
            for (int k = 0; k < n; ++k) { v[k] = sg * c[k][t]; m = fmaxf(m, v[k]); }
            float s0 = 0.f, s1 = 0.f;
            for (int k = 0; k < n; ++k) {
                const float q = exp2f((v[k] - m) * bl);
                s0 += q;
                s1 = fmaf(q, v[k], s1);
            }
            out[t] = sg * (s1 / s0);
        }
    } else {
        const float bl = pbeta(e, I) * LOG2E;
        for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
            float v[MAX_NCH];
            float m = -INFINITY;
            for (int k = 0; k < n; ++k) { v[k] = sg * c[k][t]; m = fmaxf(m, v[k]); }
            float s = 0.f;
            for (int k = 0; k < n; ++k) s += exp2f((v[k] - m) * bl);
            out[t] = sg * (m + log2f(s) / bl);
        }
    }
}

DEV void op_nary_bwd(const Env& e, const Instr& I)
{
    const float sg = (I.flags & F_MIN) ? -1.f : 1.f;
    const int n = I.nch;
    const float* g = slot(e, I.g_out);
    const float* out = slot(e, I.b_out);
    const float* c[MAX_NCH];
    float* gc[MAX_NCH];
    for (int k = 0; k < MAX_NCH; ++k) {
        c[k] = slot(e, I.b_ch[k < n ? k : 0]);
        gc[k] = slot(e, I.g_ch[k < n ? k : 0]);
    }
    const bool smooth = I.flags & F_SMOOTH;
    const float bl = pbeta(e, I) * LOG2E;
    for (int t = threadIdx.x; t < e.L; t += blockDim.x) {
        const float gt = g[t];
        if (!smooth) {
            int kb = 0;
            float best = sg * c[0][t];
            for (int k = 1; k < n; ++k) {
                float v = sg * c[k][t];
                if (v > best) { best = v; kb = k; }
            }
            for (int k = 0; k < n; ++k) gc[k][t] = (k == kb) ? gt : 0.f;
        } else if (I.flags & F_SOFT) {
            // d r / d v_k = p_k (1 + beta (v_k - r)), r = sg out
            const float r = sg * out[t], beta = bl / LOG2E;
            float v[MAX_NCH];
            float m = -INFINITY;
            for (int k = 0; k < n; ++k) { v[k] = sg * c[k][t]; m = fmaxf(m, v[k]); }
            float s0 = 0.f;
            for (int k = 0; k < n; ++k) s0 += exp2f((v[k] - m) * bl);
            for (int k = 0; k < n; ++k)
                gc[k][t] = gt * (exp2f((v[k] - m) * bl) / s0) * (1.f + beta * (v[k] - r));
        } else {
            const float o = sg * out[t];
            for (int k = 0; k < n; ++k) gc[k][t] = gt * exp2f((sg * c[k][t] - o) * bl);
        }
    }
}

// ------------------------------------------------------------------ hard windows

// Hard max (sg=+1) / min (sg=-1) of u over [t+klo, t+khi] (khi<0: to the end)
// with the pad policy.  Writes out[t]; if jstar != NULL also the index of the
// selected element (L when none / a constant pad).
DEV void win_hard(const Env& e, const float* u, float* out, int* jstar, float sg, int klo, int khi,
                  int pad, float padv, VI* Pre, VI* Suf)
{
    const int L = e.L;
    const bool unb = khi < 0;
    const int n = L - klo;
    const int K = unb ? n : khi - klo + 1;
    if (n > 0) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            VI v{sg * u[klo + i], klo + i};
            Suf[i] = v;
            if (!unb) Pre[i] = v;
        }
        __syncthreads();
        const VI id{-INFINITY, 0x7fffffff};
        seg_scan(Suf, n, unb ? 0 : K, true, id, OpVI(), *e.sh);
        if (!unb) seg_scan(Pre, n, K, false, id, OpVI(), *e.sh);
    }
    const float rho_pad = e.P->rho_pad;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        VI r{-INFINITY, L};
        bool any = false;
        if (t < n) {
            int e2 = min(t + K - 1, n - 1);
            r = (unb || t / K == e2 / K) ? Suf[t] : vi_best(Suf[t], Pre[e2]);
            any = true;
        }
        if (!unb && pad != PAD_NEUTRAL && t + khi > L - 1) {
            if (pad == PAD_LAST) {
                if (!any) r = VI{sg * u[L - 1], L - 1};
            } else {
                VI pv{sg * padv, L};
                r = any ? vi_best(r, pv) : pv;
            }
            any = true;
        }
        out[t] = any ? sg * r.v : -sg * rho_pad;
        if (jstar) jstar[t] = any ? r.i : L;
    }
    __syncthreads();
}

// adjoint of a hard window: gu[j] = sum of g[t] over the t whose selected
// index is j.  The selected index is non-decreasing in t, so each j owns a
// contiguous run of t, found by binary search; the run sum comes from an
// fp64 prefix sum of g (exact to fp32 rounding, deterministic).
DEV void win_hard_adj(const Env& e, const float* g, float* gu, const int* jstar, double* P)
{
    const int L = e.L;
    for (int t = threadIdx.x; t < L; t += blockDim.x) P[t + 1] = jstar[t] < L ? (double)g[t] : 0.0;
    if (threadIdx.x == 0) P[0] = 0.0;
    __syncthreads();
    seg_scan(P + 1, L, 0, false, 0.0, OpD(), *e.sh);
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        int lo = lower_bound_i(jstar, L, j);
        int hi = lower_bound_i(jstar, L, j + 1);
        gu[j] = (float)(P[hi] - P[lo]);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ smooth windows

// Smooth max (sg=+1) / min of u over the integer window [t+klo, t+khi]
// (khi<0: to the end), scaled by a constant weight 2^lw, as scaled pairs:
// acc[t] = sum_j w 2^{z_j}, z = sg*beta*log2(e)*u.  Pads add their copies.
// any[t] (byte flag) tells whether the window is non-empty.
DEV void win_smooth_sum(const Env& e, const float* u, SP* acc, float sgz, int klo, int khi, int pad,
                        float padv, SP* Pre, SP* Suf)
{
    const int L = e.L;
    const bool unb = khi < 0;
    const int n = L - klo;
    const int K = unb ? n : khi - klo + 1;
    if (n > 0) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            SP v = sp_leaf(sgz * u[klo + i]);
            Suf[i] = v;
            if (!unb) Pre[i] = v;
        }
        __syncthreads();
        seg_scan(Suf, n, unb ? 0 : K, true, sp_zero(), OpSP(), *e.sh);
        if (!unb) seg_scan(Pre, n, K, false, sp_zero(), OpSP(), *e.sh);
    }
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        SP a = sp_zero();
        if (t < n) {
            int e2 = min(t + K - 1, n - 1);
            a = (unb || t / K == e2 / K) ? Suf[t] : sp_add(Suf[t], Pre[e2]);
        }
        if (!unb && pad != PAD_NEUTRAL && t + khi > L - 1) {
            int np = min(K, t + khi - (L - 1));
            SP pv = sp_leaf(pad == PAD_LAST ? sgz * u[L - 1] : sgz * padv);
            pv.s *= (float)np;
            a = sp_add(a, pv);
        }
        acc[t] = a;
    }
    __syncthreads();
}

// Transposed window sum for adjoints: for each position j,
// out[j] = sum over t in [j-khi, j-klo] (clipped to [0, nt_valid)) of h[t].
// h (scaled pairs) is consumed (overwritten by the scans).
// Window sums of u_j 2^{sgz u_j} (signed scaled pairs) over [t+klo, t+khi]
// (khi < 0: to the end), NEUTRAL pad: the numerator of the softmax-weighted
// mean whose denominator win_smooth_sum gives.
DEV void win_smooth_sum_w(const Env& e, const float* u, SP* acc, float sgz, int klo, int khi, SP* Pre, SP* Suf)
{
    const int L = e.L;
    const bool unb = khi < 0;
    const int n = L - klo;
    const int K = unb ? n : khi - klo + 1;
    if (n > 0) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            SP v = sp_leaf(sgz * u[klo + i]);
            v.s *= u[klo + i];
            Suf[i] = v;
            if (!unb) Pre[i] = v;
        }
        __syncthreads();
        seg_scan(Suf, n, unb ? 0 : K, true, sp_zero(), OpSP(), *e.sh);
        if (!unb) seg_scan(Pre, n, K, false, sp_zero(), OpSP(), *e.sh);
    }
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        SP a = sp_zero();
        if (t < n) {
            int e2 = min(t + K - 1, n - 1);
            a = (unb || t / K == e2 / K) ? Suf[t] : sp_add(Suf[t], Pre[e2]);
        }
        acc[t] = a;
    }
    __syncthreads();
}

// ratio of two scaled pairs as a float (den > 0)
DEV float sp_ratio(SP num, SP den)
{
    return ldexpf(num.s / den.s, clampe((long long)num.r - den.r));
}

DEV void win_smooth_adj_sum(const Env& e, SP* h, SP* hPre, SP* res, int klo, int khi, int n_valid)
{
    const int L = e.L;
    const bool unb = khi < 0;
    const int K = unb ? L : khi - klo + 1;
    for (int t = threadIdx.x; t < L; t += blockDim.x) hPre[t] = h[t];
    __syncthreads();
    seg_scan(hPre, L, unb ? 0 : K, false, sp_zero(), OpSP(), *e.sh);
    if (!unb) seg_scan(h, L, K, true, sp_zero(), OpSP(), *e.sh);
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        SP a = sp_zero();
        int en = min(j - klo, n_valid - 1);
        int st = unb ? 0 : max(0, j - khi);
        if (st <= en) {
            if (unb) a = hPre[en];
            else if (st / K == en / K) a = (st % K == 0) ? hPre[en] : h[st];
            else a = sp_add(h[st], hPre[en]);
        }
        res[j] = a;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ masks

struct MaskInfo {
    int klo, khi;      // support {w > 0}; khi = L-1 .. for unbounded
    int clo, chi;      // constant core (clo > chi: none)
    float wc;          // core weight
    bool any;
};

// Smooth-mask weight of offset k (Sec. VI):
//   w_k = max(sig(c(k-a)) - sig(c(k-b)) - eps, 0)
// using sig(x) - sig(y) = sig(x) sig(-y) (1 - exp(-(x-y))), which has no
// cancellation, and its derivatives d w/da = -c sig'(c(k-a)),
// d w/db = c sig'(c(k-b)) (zero where the clamp is active).
struct MaskP {
    float a, b, c, eps, band;
    bool unb;
};

DEV MaskP mask_params(const float* pm, bool unb)
{
    MaskP m;
    m.a = pm[0];
    m.b = pm[1];
    m.c = pm[2];
    m.eps = pm[3];
    m.unb = unb;
    m.band = unb ? 1.f : 1.f - expf(-m.c * (m.b - m.a));
    return m;
}

DEV float mask_wk(const MaskP& m, int k, float* dwa = nullptr, float* dwb = nullptr)
{
    const float x1 = m.c * ((float)k - m.a);
    const float s1 = 1.f / (1.f + expf(-x1));
    float wk;
    if (m.unb) {
        wk = s1 - m.eps;
    } else {
        const float y1 = m.c * ((float)k - m.b);
        const float sny = 1.f / (1.f + expf(y1));
        wk = s1 * sny * m.band - m.eps;
    }
    wk = wk > 0.f ? wk : 0.f;
    if (dwa) {
        // sig'(x) = e^{-|x|} / (1 + e^{-|x|})^2: accurate in both tails (the
        // form s (1 - s) loses all digits where s rounds to 1)
        const float t1 = expf(-fabsf(x1));
        *dwa = wk > 0.f ? -m.c * (t1 / ((1.f + t1) * (1.f + t1))) : 0.f;
        if (wk > 0.f && !m.unb) {
            const float t2 = expf(-fabsf(m.c * ((float)k - m.b)));
            *dwb = m.c * (t2 / ((1.f + t2) * (1.f + t2)));
        } else {
            *dwb = 0.f;
        }
    }
    return wk;
}

// Offsets that can hold the support {w > 0}: it lies inside [a - 89/c,
// b + 89/c], beyond which a sigmoid's exponential overflows in fp32 (e^x is
// inf for x > 88.73), the factor is exactly 0 and w_k = max(-eps, 0).
DEV void mask_window(const MaskP& mp, int L, int& k0, int& k1)
{
    k0 = 0;
    k1 = L - 1;
    const double a = mp.a, b = mp.b, c = mp.c;
    if (c > 0.0 && isfinite(a) && isfinite(c) && (mp.unb || isfinite(b))) {
        k0 = (int)fmax(0.0, fmin((double)L, floor(a - 89.0 / c) - 2.0));
        if (!mp.unb) k1 = (int)fmin((double)(L - 1), fmax(-1.0, ceil(b + 89.0 / c) + 2.0));
    }
}

// the core where both sigmoid derivatives are below 2^-24 (|c(k-a)|,
// |c(k-b)| > 17), over which w is constant to fp32 rounding, given the
// support [klo, khi]
DEV MaskInfo mask_core(const MaskP& mp, int klo, int khi, int mid_known = INT_MIN, float w_known = 0.f)
{
    MaskInfo mi;
    mi.klo = klo;
    mi.khi = khi;
    mi.any = mi.klo <= mi.khi;
    const float a = mp.a, b = mp.b, c = mp.c;
    if (c > 0.f && mi.any) {
        mi.clo = max(mi.klo, (int)fminf(ceilf(a + 17.f / c), 2e9f));
        mi.chi = mp.unb ? mi.khi : min(mi.khi, (int)fmaxf(floorf(b - 17.f / c), -2e9f));
    } else {
        mi.clo = 1;
        mi.chi = 0;
    }
    // (w at the midpoint, unless the caller has it already)
    if (mi.clo > mi.chi) { mi.clo = 1; mi.chi = 0; mi.wc = 0.f; }
    else mi.wc = (mi.clo + mi.chi) / 2 == mid_known ? w_known : mask_wk(mp, (mi.clo + mi.chi) / 2);
    return mi;
}

// min / max over the wave (an atomic with a value per lane becomes a scalar
// loop over the lanes, which the work-group's waves share: reduce first)
DEV int wave_imin(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
DEV int wave_imax(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Weights for k in [0, L) (stored when w != NULL), the support {w > 0} and
// the core.  Without stored weights only the support's window is searched.
template <class SH>
DEV MaskInfo mask_info(const float* params, const Instr& I, int L, SH& sh, float* w, float* dwa, float* dwb)
{
    const MaskP mp = mask_params(params + I.mask, I.flags & F_MASK_UNB);
    int* si = sh.ints;
    if (threadIdx.x == 0) { si[0] = L; si[1] = -1; }
    __syncthreads();
    int lo = L, hi = -1;
    int k0 = 0, k1 = L - 1;
    if (!w && !dwa) mask_window(mp, L, k0, k1);
    for (int k = k0 + (int)threadIdx.x; k <= k1; k += blockDim.x) {
        float da, db;
        const float wk = mask_wk(mp, k, dwa ? &da : nullptr, &db);
        if (w) w[k] = wk;
        if (dwa) { dwa[k] = da; dwb[k] = db; }
        if (wk > 0.f) { lo = min(lo, k); hi = max(hi, k); }
    }
    lo = wave_imin(lo);
    hi = wave_imax(hi);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&si[0], lo);
        atomicMax(&si[1], hi);
    }
    __syncthreads();
    const MaskInfo mi = mask_core(mp, si[0], si[1]);
    __syncthreads();
    return mi;
}

// pad value of a smooth-mask node (carried in the instruction: kernels read
// it without indexing the plan's coefficient table)
DEV float mask_padv(const Instr& I) { return __int_as_float(I.a); }

DEV MaskInfo mask_weights(const Env& e, const Instr& I, float* w, float* dwa, float* dwb)
{
    return mask_info(e.params, I, e.L, *e.sh, w, dwa, dwb);
}

// deterministic work-group sum of one double per thread
DEV double wg_sum_d(double v, Shared& sh)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    sh.scan[tid] = v;
    __syncthreads();
    for (int s = nt >> 1; s > 0; s >>= 1) {
        if (tid < s) sh.scan[tid] += sh.scan[tid + s];
        __syncthreads();
    }
    const double r = sh.scan[0];
    __syncthreads();
    return r;
}

// Offsets past the signal end, for the LAST / CONST pads of a bounded smooth
// mask: each offset k >= L of the support contributes one pad copy with
// weight w_k.  Past b, w_k <= sig(-c(k - b)) < e^{-c(k - b)}, which is below
// eps (and w_k clamps to 0) from k = b + ln(1/eps)/c on; in fp32 the sigmoid
// itself is 0 once c(k - b) > 89.  The walk stops there, and never runs more
// than MASK_TAIL_MAX offsets past the end.
constexpr int MASK_TAIL_MAX = 65536;

struct MaskTail {
    int lo, hi;          // support offsets >= L (lo > hi: none)
    double s, sa, sb;    // sums of w_k, d w_k/da, d w_k/db over them
};

DEV MaskTail mask_tail(const Env& e, const Instr& I, bool grads)
{
    const int L = e.L;
    const MaskP mp = mask_params(e.params + I.mask, false);
    int kend = -1;
    if (mp.c > 0.f && mp.b == mp.b) {
        const float span = fminf(logf(1.f / fmaxf(mp.eps, 1e-38f)), 89.f) / mp.c + 2.f;
        const float ke = fminf(mp.b + span, (float)L + (float)MASK_TAIL_MAX);
        kend = ke >= (float)L ? (int)ke : -1;
    }
    int* si = e.sh->ints;
    if (threadIdx.x == 0) { si[5] = INT_MAX; si[6] = -1; }
    __syncthreads();
    int lo = INT_MAX, hi = -1;
    double s = 0.0, sa = 0.0, sb = 0.0;
    for (int k = L + (int)threadIdx.x; k <= kend; k += blockDim.x) {
        float da = 0.f, db = 0.f;
        const float wk = mask_wk(mp, k, grads ? &da : nullptr, &db);
        if (wk > 0.f) {
            lo = min(lo, k);
            hi = max(hi, k);
            s += wk;
            sa += da;
            sb += db;
        }
    }
    atomicMin(&si[5], lo);
    atomicMax(&si[6], hi);
    __syncthreads();
    MaskTail mt;
    mt.lo = si[5];
    mt.hi = si[6];
    mt.s = wg_sum_d(s, *e.sh);
    mt.sa = grads ? wg_sum_d(sa, *e.sh) : 0.0;
    mt.sb = grads ? wg_sum_d(sb, *e.sh) : 0.0;
    return mt;
}

// out[t] = tail + sum_{k=L-t}^{L-1} v[k] for t in [0, L): the part of an
// offset table v (zero outside the mask support) that lies past the signal
// end for the output at t, plus the tail beyond the table.  fp64 sums: one
// contiguous chunk per thread, an exclusive suffix scan over the lanes and
// the totals of the later waves.
DEV void tail_weights(const float* v, float* out, int L, double tail, Shared& sh)
{
    const int nt = blockDim.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nw = (nt + 63) >> 6;
    const int ch = (L + nt - 1) / nt;
    const int k0 = min(L, tid * ch), k1 = min(L, k0 + ch);
    double c = 0.0;
    for (int k = k0; k < k1; ++k) c += (double)v[k];
    double r = c;                               // inclusive suffix over the lanes
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_down(r, d);
        if (lane + d < 64) r += o;
    }
    double ex = __shfl_down(r, 1);              // lanes after this one
    if (lane == 63) ex = 0.0;
    if (lane == 0) sh.scan[wv] = r;
    __syncthreads();
    double acc = tail + ex;
    for (int q = wv + 1; q < nw; ++q) acc += sh.scan[q];
    for (int k = k1 - 1; k >= k0; --k) {
        acc += (double)v[k];
        if (k >= 1) out[L - k] = (float)acc;
    }
    if (tid == 0) out[0] = (float)tail;
    __syncthreads();
}

// ------------------------------------------------------------------ until

// Hard Until, one thread per output t: running min of phi over [t, t+i],
// max over i in [a, b] of min(running min, psi_{t+i}); phi wins ties.
// Adjoint (g != null): every output sends g_t to the one phi or psi sample
// that decides it.  The target of each t goes to `code` (phi index k as k,
// psi index k as -k-1, none as INT_MIN); then each position sums the g_t
// that target it in increasing t, so the result does not depend on the
// order in which threads finish.
DEV void until_hard(const Env& e, int a, int b, const float* phi, const float* psi, float* out,
                    const float* g, float* gphi, float* gpsi, int* code)
{
    const int L = e.L;
    const float rho_pad = e.P->rho_pad;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const int imax = b < 0 ? L - 1 - t : min(b, L - 1 - t);
        if (a > imax) {
            if (out) out[t] = -rho_pad;
            if (g) code[t] = INT_MIN;
            continue;
        }
        float R = phi[t], best = -INFINITY;
        int kR = t, tgt = -1;
        bool tphi = false;
        for (int i = 0; i <= imax; ++i) {
            const float f = phi[t + i];
            if (f < R) { R = f; kR = t + i; }
            if (i >= a) {
                const float p = psi[t + i];
                const bool pw = R <= p;
                const float v = pw ? R : p;
                if (tgt < 0 || v > best) { best = v; tphi = pw; tgt = pw ? kR : t + i; }
            }
        }
        if (out) out[t] = best;
        if (g) code[t] = tphi ? tgt : -tgt - 1;
    }
    if (!g) return;
    __syncthreads();
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        float sp = 0.f, sq = 0.f;
        for (int t = b < 0 ? 0 : max(0, j - b); t <= j; ++t) {
            const int c = code[t];
            if (c == j) sp += g[t];
            else if (c == -j - 1) sq += g[t];
        }
        gphi[j] += sp;
        gpsi[j] += sq;
    }
}

// Hard Until with an unbounded interval [a, inf), O(L) per trajectory.
// With m_a(t) = min of phi over [t, t+a-1] (a > 0) and the a = 0 form
//   U(s) = max_{j >= 0} min(min_{k <= j} phi_{s+k}, psi_{s+j}),
// out(t) = min(m_a(t), U(t+a)).  U satisfies U(s) = f_s(U(s+1)), U(L) = -inf,
// for the clamp map f_s(u) = min(phi_s, max(psi_s, u)) = clamp of u to
// [min(psi_s, phi_s), phi_s]; clamp maps compose into clamp maps, so U is a
// suffix scan of compositions.  The adjoint follows the same ties as the
// walk of until_hard (lowest index, phi wins): output s decides at phi_s
// (phi_s <= psi_s, or psi_s < phi_s <= U(s+1)), at psi_s (U(s+1) <= psi_s
// < phi_s), or passes its adjoint to output s+1 (psi_s < U(s+1) < phi_s); an
// output t goes to the window argmin of m_a when m_a(t) <= U(t+a).  The
// passed-on sums F(s) = h(s) + [s-1 passes] F(s-1) are a scan of affine
// maps; the window part is the hard window's adjoint.  Scratch units 0..15.
struct ClampMap {
    float lo, hi;   // u -> min(hi, max(lo, u)), lo <= hi
};
struct OpClamp {    // a after b
    __device__ __forceinline__ ClampMap operator()(ClampMap a, ClampMap b) const
    {
        auto f = [&](float x) { return x < a.lo ? a.lo : (x > a.hi ? a.hi : x); };
        return ClampMap{f(b.lo), f(b.hi)};
    }
};
struct Affine {
    float h;        // x -> h + c x, c in {0, 1}
    int c;
};
struct OpAffine {   // l then r
    __device__ __forceinline__ Affine operator()(Affine l, Affine r) const
    {
        return Affine{r.c ? r.h + l.h : r.h, l.c & r.c};
    }
};
enum { UH_PHI = 0, UH_PSI = 1, UH_PASS = 2 };

DEV void until_hard_unb(const Env& e, int a, const float* phi, const float* psi, float* out, const float* g,
                        float* gphi, float* gpsi)
{
    const int L = e.L;
    const float rho_pad = e.P->rho_pad;
    float* mA = S(e, 4);
    int* jA = (int*)S(e, 5);
    ClampMap* cm = (ClampMap*)S(e, 6);      // units 6, 7
    if (a > 0) win_hard(e, phi, mA, jA, -1.f, 0, a - 1, PAD_NEUTRAL, 0.f, (VI*)S(e, 0), (VI*)S(e, 2));
    for (int s = threadIdx.x; s < L; s += blockDim.x) cm[s] = ClampMap{phi[s] <= psi[s] ? phi[s] : psi[s], phi[s]};
    __syncthreads();
    seg_scan(cm, L, 0, true, ClampMap{-INFINITY, INFINITY}, OpClamp(), *e.sh);     // cm[s].lo = U(s)
    if (!g) {
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            float v = -rho_pad;
            if (t + a <= L - 1) {
                const float u = cm[t + a].lo;
                v = (a > 0 && mA[t] <= u) ? mA[t] : u;
            }
            out[t] = v;
        }
        __syncthreads();
        return;
    }
    int* code = (int*)S(e, 8);
    Affine* fa = (Affine*)S(e, 9);          // units 9, 10
    float* gw = S(e, 11);                   // adjoint sent to the window argmin of m_a
    for (int s = threadIdx.x; s < L; s += blockDim.x) {
        const float un = s + 1 < L ? cm[s + 1].lo : -INFINITY;
        int c = UH_PHI;
        if (!(phi[s] <= psi[s])) {
            const float w = phi[s] <= un ? phi[s] : un;
            c = w > psi[s] ? (phi[s] <= un ? UH_PHI : UH_PASS) : UH_PSI;
        }
        code[s] = c;
        // output t = s: to the window argmin, or to U(s + a)
        float gt = 0.f;
        bool win = false;
        if (s + a <= L - 1) {
            gt = g[s];
            win = a > 0 && mA[s] <= cm[s + a].lo;
        }
        gw[s] = win ? gt : 0.f;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < L; s += blockDim.x) {
        const int t = s - a;
        const float h = (t >= 0 && !(a > 0 && mA[t] <= cm[s].lo)) ? g[t] : 0.f;
        fa[s] = Affine{h, s > 0 && code[s - 1] == UH_PASS ? 1 : 0};
    }
    __syncthreads();
    seg_scan(fa, L, 0, false, Affine{0.f, 1}, OpAffine(), *e.sh);                 // fa[s].h = F(s)
    for (int s = threadIdx.x; s < L; s += blockDim.x) {
        if (code[s] == UH_PHI) gphi[s] += fa[s].h;
        else if (code[s] == UH_PSI) gpsi[s] += fa[s].h;
    }
    __syncthreads();
    if (a > 0) {
        float* gu = S(e, 15);
        win_hard_adj(e, gw, gu, jA, (double*)S(e, 12));                          // units 12..14
        for (int j = threadIdx.x; j < L; j += blockDim.x) gphi[j] += gu[j];
        __syncthreads();
    }
}

// Smooth Until forward, one thread per output t:
//   P_i = sum_{k<=i} 2^{-z_phi(t+k)}   (running scaled sum: smooth min of phi)
//   Y_i = 1 / (P_i + 2^{-z_psi(t+i)})  (= exp(beta * smin(R_i, psi_{t+i})))
//   out = log2(sum_{i in [a,b]} w_i Y_i) / (beta log2 e)
// Ephi / Epsi hold the leaves 2^{-z}; w (smooth mask weights by offset i,
// Sec. VI) is null for the 0/1 interval.
DEV void until_smooth_fwd(const Env& e, int a, int b, const float* w, const SP* Ephi, const SP* Epsi,
                          float* out, float bl)
{
    const int L = e.L;
    const float rho_pad = e.P->rho_pad;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const int imax = b < 0 ? L - 1 - t : min(b, L - 1 - t);
        if (a > imax) { out[t] = -rho_pad; continue; }
        SP P = sp_zero(), Z = sp_zero();
        for (int i = 0; i <= imax; ++i) {
            P = sp_add(P, Ephi[t + i]);
            if (i >= a) {
                SP Dn = sp_add(P, Epsi[t + i]);
                Z = sp_add(Z, SP{(w ? w[i] : 1.f) / Dn.s, -Dn.r});
            }
        }
        out[t] = sp_log2(Z) / bl;
    }
}

constexpr int UCK = 16;   // checkpoint spacing of the smooth Until adjoint
constexpr int UCK_UNIT = 7;   // scratch unit where its checkpoints start (units 4-6: mask tables)

// Smooth Until adjoint (checkpointed reverse sweep per output t):
//   d out / d psi_{t+i} = w_i Y_i^2 Q_i / Z,  Q_i = 2^{-z_psi(t+i)}
//   d out / d phi_{t+k} = e_k / Z * sum_{i >= max(k,a)} w_i Y_i^2,  e_k = 2^{-z_phi(t+k)}
//   d out / d w_i = Y_i / (beta Z)   (summed against d w/da, d w/db into pa, pb)
// Pass 1 recomputes Z and stores P every UCK steps; pass 2 walks the
// checkpoint blocks backward, recomputing P inside each block.  The float
// contributions go through the lane-shifted accumulators of lane_stage
// (defined below), in the same fixed order as the fp64 adjoint.
DEV void lane_stage_f(int i, int tb, int lane, int L, float& accp, float& accq, float& stp, float& stq,
                      float* gphi, float* gpsi);

DEV void until_smooth_adj(const Env& e, int a, int b, const float* w, const float* dwa, const float* dwb,
                          const SP* Ephi, const SP* Epsi, const float* g, float* gphi, float* gpsi, SP* ck,
                          int ncks, float& pa, float& pb)
{
    const int L = e.L;
    const int lane = threadIdx.x & 63;
    for (int base = 0; base < L; base += blockDim.x) {
        const int tb = base + (int)threadIdx.x - lane;
        const int t = tb + lane;
        const int imax = t >= L ? -1 : (b < 0 ? L - 1 - t : min(b, L - 1 - t));
        const float gt = t < L ? g[t] : 0.f;
        const bool act = a <= imax && gt != 0.f;
        SP* myck = ck + (size_t)threadIdx.x * ncks;
        SP Z = sp_zero();
        if (act) {
            SP P = sp_zero();
            for (int i = 0; i <= imax; ++i) {
                if (i % UCK == 0) myck[i / UCK] = P;
                P = sp_add(P, Ephi[t + i]);
                if (i >= a) {
                    SP Dn = sp_add(P, Epsi[t + i]);
                    Z = sp_add(Z, SP{(w ? w[i] : 1.f) / Dn.s, -Dn.r});
                }
            }
        }
        const float gz = act ? gt / Z.s : 0.f;      // G / Z = gz * 2^{-Z.r}
        const int imax0 = b < 0 ? L - 1 - base : min(b, L - 1 - base);     // t = base: the longest chain
        const int wblk = a <= imax0 ? imax0 / UCK + 1 : 0;
        float accp = 0.f, accq = 0.f, stp = 0.f, stq = 0.f;
        SP A = sp_zero();                   // suffix sum of w_i Y_i^2
        for (int blk = wblk - 1; blk >= 0; --blk) {
            const int i0 = blk * UCK;
            const int i1 = act ? min(imax, i0 + UCK - 1) : i0 - 1;      // this lane's last step in the block
            SP Ps[UCK];
            SP Pc = i0 <= i1 ? myck[blk] : sp_zero();
#pragma unroll
            for (int q = 0; q < UCK; ++q) {
                if (i0 + q <= i1) Pc = sp_add(Pc, Ephi[t + i0 + q]);
                Ps[q] = Pc;
            }
#pragma unroll
            for (int q = UCK - 1; q >= 0; --q) {
                const int i = i0 + q;
                if (i <= i1) {
                    if (i >= a) {
                        const SP Q = Epsi[t + i];
                        const SP Dn = sp_add(Ps[q], Q);
                        const float y = 1.f / Dn.s;       // Y = y * 2^{-Dn.r}
                        const SP Y2{(w ? w[i] : 1.f) * y * y, -2 * Dn.r};
                        A = sp_add(A, Y2);
                        // psi: gz * w Y^2 * Q  (exponent -Z.r - 2 Dn.r + Q.r)
                        accq += ldexpf(gz * Y2.s * Q.s, clampe((long long)Y2.r + Q.r - Z.r));
                        if (w) {
                            const int ex = clampe(-(long long)Dn.r - Z.r);
                            pa += ldexpf(gz * dwa[i] * y, ex);
                            pb += ldexpf(gz * dwb[i] * y, ex);
                        }
                    }
                    const SP E = Ephi[t + i];
                    accp += ldexpf(gz * A.s * E.s, clampe((long long)A.r + E.r - Z.r));
                }
                if (i > 0) lane_stage_f(i, tb, lane, L, accp, accq, stp, stq, gphi, gpsi);
            }
        }
        if (wblk > 0 && t < L) {
            gphi[t] += accp;
            gpsi[t] += accq;
        }
        __syncthreads();
    }
}

// Smooth Until in fp64 against one reference exponent per trajectory.  The
// leaf terms 2^u, u = -beta log2(e) (phi or psi), are kept as the doubles
// 2^{u - M} with M = ceil(max u) over both inputs: every term is <= 1, so the
// running sums, their reciprocals and the outer sums stay inside the fp64
// range while the exponent range max u - min u is below UF_RANGE.  Beyond it
// (or with a non-finite value) the scaled-pair routines above take over.
constexpr int UF_RANGE = 1000;

// 2^{u - M} with exact exponent bookkeeping (u - ceil(u) is exact)
DEV double uterm(float u, int M)
{
    const float c = ceilf(u);
    return ldexp((double)__builtin_amdgcn_exp2f(u - c), (int)c - M);
}

// 1/d for a positive normal d: the hardware estimate alone.  Its relative
// error is at the float32 level (measured on gfx950: at most 4.6e-8 over 4M
// samples spanning 2^-1010 .. 2^31), which is all the float32 outputs need:
// the fp64 form is there for its exponent range, and every sum it feeds
// (Z, the suffix sums of Y^2) adds positive terms, so relative errors do not
// grow.  A Newton step would cost two more fp64 FMAs per term.
DEV double rcpd(double d)
{
    return __builtin_amdgcn_rcp(d);
}

// log2 of a positive double, as the double (exponent - M) + log2(mantissa)
DEV double log2_minus(double z, int M)
{
    int ez;
    const double mz = frexp(z, &ez);
    return (double)(ez - M) + (double)__builtin_amdgcn_logf((float)mz);
}

// Reference exponent M of the two leaf traces; false when the fp64 form
// cannot hold them.
DEV bool until_ref(const float* phi, const float* psi, int L, float bl, Shared& sh, int& M)
{
    int hi = INT_MIN, lo = INT_MAX, bad = 0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const float u1 = -bl * phi[j], u2 = -bl * psi[j];
        if (!(fabsf(u1) < 1e9f) || !(fabsf(u2) < 1e9f)) {
            bad = 1;                                 // also catches NaN
        } else {
            hi = max(hi, (int)ceilf(fmaxf(u1, u2)));
            lo = min(lo, (int)floorf(fminf(u1, u2)));
        }
    }
    if (threadIdx.x == 0) {
        sh.ints[2] = INT_MIN;
        sh.ints[3] = INT_MAX;
        sh.ints[4] = 0;
    }
    __syncthreads();
    atomicMax(&sh.ints[2], hi);
    atomicMin(&sh.ints[3], lo);
    if (bad) atomicOr(&sh.ints[4], 1);
    __syncthreads();
    M = sh.ints[2];
    const bool ok = sh.ints[4] == 0 && (long long)M - (long long)sh.ints[3] <= UF_RANGE;
    __syncthreads();
    return ok;
}

// leaf terms of both inputs as doubles 2^{u - M} (Ep, Eq)
DEV void until_terms(const float* phi, const float* psi, int L, float bl, int M, double* Ep, double* Eq)
{
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        Ep[j] = uterm(-bl * phi[j], M);
        Eq[j] = uterm(-bl * psi[j], M);
    }
    __syncthreads();
}

typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) float lds_float;

// true when p points into the work-group's LDS (the arena placement is chosen per launch)
DEV bool in_lds(const void* p)
{
    return __builtin_amdgcn_is_shared((const __attribute__((address_space(0))) void*)p);
}

// Z = sum_{i=a}^{imax} 1 / (P_i + q_i), P_i = sum_{k<=i} p_k, over the terms of
// one output.  The terms are read eight at a time (independent loads ahead of
// the dependent sums); the additions keep the plain sequential order.
template <bool MW, class DP>
DEV double until_z(DP ep, DP eq, int a, int imax, const float* w)
{
    double P = 0.0, Z = 0.0;
    int i = 0;
    for (; i + 8 <= a; i += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = ep[i + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) P += v[k];
    }
    for (; i < a; ++i) P += ep[i];
    for (; i + 8 <= imax + 1; i += 8) {
        double v[8], q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = ep[i + k];
            q[k] = eq[i + k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            P += v[k];
            const double y = rcpd(P + q[k]);
            Z += MW ? (double)w[i + k] * y : y;
        }
    }
    for (; i <= imax; ++i) {
        P += ep[i];
        const double y = rcpd(P + eq[i]);
        Z += MW ? (double)w[i] * y : y;
    }
    return Z;
}

// Forward on the fp64 terms: the same sums as until_smooth_fwd, with
// Y_i = 2^{-M} / (P_i + Q_i) in true units, so log2 Z_true = log2 Z - M.
template <bool MW, class DP>
DEV void until_fwd_d(const Env& e, int a, int b, const float* w, DP Ep, DP Eq, float* out, double* zs, float bl,
                     int M)
{
    const int L = e.L;
    const float rho_pad = e.P->rho_pad;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const int imax = b < 0 ? L - 1 - t : min(b, L - 1 - t);
        if (a > imax) { out[t] = -rho_pad; continue; }
        const double Z = until_z<MW>(Ep + t, Eq + t, a, imax, w);
        out[t] = (float)(log2_minus(Z, M) / (double)bl);
        if (zs) zs[t] = Z;
    }
}

// value of the lane below (lane 0 receives 0): one DPP wave shift
DEV float lane_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// One step of the lane-shifted adjoint accumulators of the Until adjoints
// (step i > 0, walked downwards, the same i in every wave of the
// work-group): lane 63 holds the finished sum of position tb + 64 + s,
// s = i - 1; it is parked in lane s % 64 of the staging pair, and a full
// stage (s a multiple of 64: positions tb + 64 + s + lane) is added to the
// adjoint slots, followed by a barrier.  Then the accumulators move up a lane.
template <class FP>
DEV void lane_stage(int i, int tb, int lane, int L, float& accp, float& accq, float& stp, float& stq, FP gphi,
                    FP gpsi)
{
    const int s_ = i - 1, j = s_ & 63;
    const float dp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(accp), 63));
    const float dq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(accq), 63));
    if (lane == j) {
        stp = dp;
        stq = dq;
    }
    if (j == 0) {
        const int pos = tb + 64 + s_ + lane;
        if (pos < L) {
            gphi[pos] += stp;
            gpsi[pos] += stq;
        }
        stp = 0.f;
        stq = 0.f;
        __syncthreads();
    }
    accp = lane_shr1(accp);
    accq = lane_shr1(accq);
}

DEV void lane_stage_f(int i, int tb, int lane, int L, float& accp, float& accq, float& stp, float& stq,
                      float* gphi, float* gpsi)
{
    lane_stage<float*>(i, tb, lane, L, accp, accq, stp, stq, gphi, gpsi);
}

// Adjoint on the fp64 terms (the derivatives are ratios of terms, so the
// reference cancels).  Z_t comes from the forward recompute (zs); a forward
// sweep of additions keeps P every UCK steps; the reverse sweep rebuilds each
// block's P from its checkpoint and carries the suffix sum A of Y_i^2:
//   d out / d psi_{t+i} = Y_i^2 q_i / Z,  d out / d phi_{t+k} = p_k A_k / Z.
// The lanes of a wave hold consecutive t and walk i downwards in step, so at
// each step lane l adds to position t_0 + l + i: the wave keeps one register
// accumulator per lane for these positions and moves them up one lane per
// step.  The position leaving lane 63 is complete for this wave; it is parked
// in one lane of a staging register, and every 64 steps the stage is added to
// the adjoint slots.  The rest are added at the end.  All waves of the
// work-group walk the same steps (those of the longest chain of the pass), so
// the stages are added at the same points in every wave: at one point the
// waves' stages cover disjoint positions, and a barrier separates the points,
// which fixes the order of every addition (results are bitwise reproducible).
// With smooth mask weights (MW) each term carries w_i: Z = sum w_i Y_i, A
// sums w_i Y_i^2, and d out / d w_i = Y_i / (beta Z) is summed against
// d w/da, d w/db into pa, pb (per thread, before the division by beta).
template <bool MW, class DP, class CP, class FP>
DEV void until_adj_d(const Env& e, int a, int b, const float* w, const float* dwa, const float* dwb, DP Ep,
                     DP Eq, const double* zs, const float* g, FP gphi, FP gpsi, CP ck, int ncks, float& pa,
                     float& pb)
{
    const int L = e.L;
    const int lane = threadIdx.x & 63;
    for (int base = 0; base < L; base += blockDim.x) {
        const int tb = base + (int)threadIdx.x - lane;
        const int t = tb + lane;
        const int imax = t >= L ? -1 : (b < 0 ? L - 1 - t : min(b, L - 1 - t));
        const float gt = t < L ? g[t] : 0.f;
        const bool act = a <= imax && gt != 0.f;
        const int nblk = act ? imax / UCK + 1 : 0;
        const DP ep = Ep + t;
        const DP eq = Eq + t;
        const CP myck = ck + (size_t)threadIdx.x * ncks;
        double Z = 1.0;
        if (act) {
            // Z comes from the forward recompute: only the block-start prefixes of P
            Z = zs[t];
            double P = 0.0;
            for (int blk = 0; blk < nblk; ++blk) {
                myck[blk] = P;
                if (blk + 1 < nblk) {                  // blocks before the last are full
                    const int i0 = blk * UCK;
                    double v[UCK];
#pragma unroll
                    for (int k = 0; k < UCK; ++k) v[k] = ep[i0 + k];
#pragma unroll
                    for (int k = 0; k < UCK; ++k) P += v[k];
                }
            }
        }
        const double wz = act ? (double)gt / Z : 0.0;
        const int imax0 = b < 0 ? L - 1 - base : min(b, L - 1 - base);     // t = base: the longest chain
        const int wblk = a <= imax0 ? imax0 / UCK + 1 : 0;
        float accp = 0.f, accq = 0.f;
        float stp = 0.f, stq = 0.f;         // staged finished sums (see the shift below)
        double A = 0.0;                     // G/Z times the suffix sum of w_i Y_i^2
        double da = 0.0, db = 0.0;          // sum of dw_i Y_i (MW)
        for (int blk = wblk - 1; blk >= 0; --blk) {
            const int i0 = blk * UCK;
            const int n = blk < nblk ? min(UCK, imax - i0 + 1) : 0;
            double v[UCK], q[UCK], Ps[UCK];
            double Pc = n > 0 ? myck[blk] : 0.0;
#pragma unroll
            for (int k = 0; k < UCK; ++k) {
                v[k] = k < n ? ep[i0 + k] : 0.0;
                q[k] = k < n ? eq[i0 + k] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < UCK; ++k) {
                Pc += v[k];
                Ps[k] = Pc;
            }
#pragma unroll
            for (int k = UCK - 1; k >= 0; --k) {
                const int i = i0 + k;
                if (k < n) {
                    if (i >= a) {
                        const double y = rcpd(Ps[k] + q[k]);
                        const double y2 = (MW ? wz * (double)w[i] : wz) * y * y;   // G/Z w_i Y_i^2
                        A += y2;
                        accq += (float)(y2 * q[k]);
                        if (MW) {
                            da += (double)dwa[i] * y;
                            db += (double)dwb[i] * y;
                        }
                    }
                    accp += (float)(A * v[k]);
                }
                if (i > 0) lane_stage(i, tb, lane, L, accp, accq, stp, stq, gphi, gpsi);
            }
        }
        if (wblk > 0 && t < L) {
            gphi[t] += accp;
            gpsi[t] += accq;
        }
        __syncthreads();
        if (MW) {
            pa += (float)(wz * da);
            pb += (float)(wz * db);
        }
    }
}

DEV void until_smooth_fwd_d(const Env& e, int a, int b, const float* w, double* Ep, double* Eq, float* out,
                            double* zs, float bl, int M)
{
    if (w) {
        if (in_lds(Ep))
            until_fwd_d<true>(e, a, b, w, (const lds_double*)Ep, (const lds_double*)Eq, out, zs, bl, M);
        else
            until_fwd_d<true>(e, a, b, w, (const double*)Ep, (const double*)Eq, out, zs, bl, M);
    } else if (in_lds(Ep)) {
        until_fwd_d<false>(e, a, b, w, (const lds_double*)Ep, (const lds_double*)Eq, out, zs, bl, M);
    } else {
        until_fwd_d<false>(e, a, b, w, (const double*)Ep, (const double*)Eq, out, zs, bl, M);
    }
}

DEV void until_smooth_adj_d(const Env& e, int a, int b, const float* w, const float* dwa, const float* dwb,
                            double* Ep, double* Eq, const double* zs, const float* g, float* gphi, float* gpsi,
                            double* ck, int ncks, float& pa, float& pb)
{
    if (w) {
        if (in_lds(Ep))
            until_adj_d<true>(e, a, b, w, dwa, dwb, (const lds_double*)Ep, (const lds_double*)Eq, zs, g,
                              (lds_float*)gphi, (lds_float*)gpsi, (lds_double*)ck, ncks, pa, pb);
        else
            until_adj_d<true>(e, a, b, w, dwa, dwb, (const double*)Ep, (const double*)Eq, zs, g, gphi, gpsi, ck,
                              ncks, pa, pb);
    } else if (in_lds(Ep)) {
        until_adj_d<false>(e, a, b, w, dwa, dwb, (const lds_double*)Ep, (const lds_double*)Eq, zs, g,
                           (lds_float*)gphi, (lds_float*)gpsi, (lds_double*)ck, ncks, pa, pb);
    } else {
        until_adj_d<false>(e, a, b, w, dwa, dwb, (const double*)Ep, (const double*)Eq, zs, g, gphi, gpsi, ck, ncks,
                           pa, pb);
    }
}

// ------------------------------------------------------------------ instructions

DEV bool is_smooth(const Instr& I) { return I.flags & F_SMOOTH; }

// Run one instruction forward with the given slot map (fwd or bwd).
DEV void exec_fwd(const Env& e, const Instr& I, bool bwdmap)
{
    const int o = bwdmap ? I.b_out : I.f_out;
    const int i0 = bwdmap ? I.b_in0 : I.f_in0;
    const int i1 = bwdmap ? I.b_in1 : I.f_in1;
    float* out = slot(e, o);
    const int L = e.L;
    const float sg = (I.flags & F_MIN) ? -1.f : 1.f;
    switch (I.kind) {
    case K_TRUE:
        for (int t = threadIdx.x; t < L; t += blockDim.x) out[t] = e.P->rho_max;
        break;
    case K_LIN:
    case K_NORM:
        op_pred_fwd(e, I, out);
        break;
    case K_NOT: {
        const float* u = slot(e, i0);
        for (int t = threadIdx.x; t < L; t += blockDim.x) out[t] = -u[t];
        break;
    }
    case K_NARY:
        op_nary_fwd(e, I, bwdmap ? I.b_ch : I.f_ch, out);
        break;
    case K_WIN: {
        const float* u = slot(e, i0);
        const int khi = (I.flags & F_UNB) ? -1 : I.b;
        const float padv = e.P->coef[I.coef];
        if (!is_smooth(I)) {
            win_hard(e, u, out, nullptr, sg, I.a, khi, I.pad, padv, (VI*)S(e, 0), (VI*)S(e, 2));
        } else if (I.flags & F_SOFT) {
            // softmax-weighted mean over the window: out = sum u 2^{z} / sum 2^{z};
            // LAST / CONST add np copies of the pad value v to both sums
            const float bl = pbeta(e, I) * LOG2E;
            SP* den = (SP*)S(e, 4);
            SP* num = (SP*)S(e, 6);
            win_smooth_sum(e, u, den, sg * bl, I.a, khi, I.pad, padv, (SP*)S(e, 0), (SP*)S(e, 2));
            win_smooth_sum_w(e, u, num, sg * bl, I.a, khi, (SP*)S(e, 0), (SP*)S(e, 2));
            const float v = I.pad == PAD_LAST ? u[L - 1] : padv;
            for (int t = threadIdx.x; t < L; t += blockDim.x) {
                SP nm = num[t];
                const bool padded = khi >= 0 && I.pad != PAD_NEUTRAL && t + khi > L - 1;
                if (padded) {
                    const int np = min(khi - I.a + 1, t + khi - (L - 1));
                    SP pv = sp_leaf(sg * bl * v);
                    pv.s *= (float)np * v;
                    nm = sp_add(nm, pv);
                }
                out[t] = (t + I.a <= L - 1 || padded) ? sp_ratio(nm, den[t]) : -sg * e.P->rho_pad;
            }
        } else {
            const float bl = pbeta(e, I) * LOG2E;
            SP* acc = (SP*)S(e, 4);
            win_smooth_sum(e, u, acc, sg * bl, I.a, khi, I.pad, padv, (SP*)S(e, 0), (SP*)S(e, 2));
            const bool unb = khi < 0;
            for (int t = threadIdx.x; t < L; t += blockDim.x) {
                const bool any = (t + I.a <= L - 1) || (!unb && I.pad != PAD_NEUTRAL && t + khi > L - 1);
                out[t] = any ? sg * sp_log2(acc[t]) / bl : -sg * e.P->rho_pad;
            }
        }
        break;
    }
    case K_MASK: {
        const float* u = slot(e, i0);
        float* w = S(e, 6);
        MaskInfo mi = mask_weights(e, I, w, nullptr, nullptr);
        // LAST / CONST pads of a bounded mask: support offsets past the end
        const bool padm = I.pad != PAD_NEUTRAL && !(I.flags & F_MASK_UNB);
        MaskTail mt{INT_MAX, -1, 0.0, 0.0, 0.0};
        if (padm) mt = mask_tail(e, I, false);
        const int klo = mi.any ? mi.klo : mt.lo;             // whole support
        const int khi = mt.hi >= 0 ? mt.hi : mi.khi;
        const bool anyk = mi.any || mt.hi >= 0;
        const float padv = mask_padv(I);
        if (!is_smooth(I)) {
            if (!anyk) {
                for (int t = threadIdx.x; t < L; t += blockDim.x) out[t] = -sg * e.P->rho_pad;
            } else {
                const int kh = ((I.flags & F_MASK_UNB) && khi == L - 1) ? -1 : khi;
                win_hard(e, u, out, nullptr, sg, klo, kh, padm ? I.pad : PAD_NEUTRAL, padv, (VI*)S(e, 0),
                         (VI*)S(e, 2));
            }
            break;
        }
        const float bl = pbeta(e, I) * LOG2E;
        SP* acc = (SP*)S(e, 4);
        SP* E = (SP*)S(e, 8);
        float* TW = S(e, 7);
        const bool core = mi.clo <= mi.chi;
        if (core) {
            const int kh = ((I.flags & F_MASK_UNB) && mi.chi == L - 1) ? -1 : mi.chi;
            win_smooth_sum(e, u, acc, sg * bl, mi.clo, kh, PAD_NEUTRAL, 0.f, (SP*)S(e, 0), (SP*)S(e, 2));
        }
        for (int j = threadIdx.x; j < L; j += blockDim.x) E[j] = sp_leaf(sg * bl * u[j]);
        if (padm) tail_weights(w, TW, L, mt.s, *e.sh);
        __syncthreads();
        const SP Ev = sp_leaf(sg * bl * (I.pad == PAD_LAST ? u[L - 1] : padv));
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            // band terms are summed one by one (up to a few hundred of them):
            // accumulate with a double mantissa so the error does not grow with the count
            SPD a{0.0, SP_NEG};
            if (core) a = spd_add(a, SP{acc[t].s * mi.wc, acc[t].r});
            const int b0 = mi.klo, b1 = core ? mi.clo - 1 : mi.khi;
            for (int k = b0; k <= b1 && t + k < L; ++k) a = spd_add(a, SP{w[k] * E[t + k].s, E[t + k].r});
            if (core)
                for (int k = mi.chi + 1; k <= mi.khi && t + k < L; ++k)
                    a = spd_add(a, SP{w[k] * E[t + k].s, E[t + k].r});
            const bool pt = padm && anyk && t + khi > L - 1;   // pad copies for this output
            if (pt) a = spd_add(a, SP{TW[t] * Ev.s, Ev.r});
            const bool any = (mi.any && t + mi.klo <= L - 1) || pt;
            out[t] = any ? sg * sp_log2(spd_to_sp(a)) / bl : -sg * e.P->rho_pad;
        }
        break;
    }
    case K_UNTIL: {
        const float* phi = slot(e, i0);
        const float* psi = slot(e, i1);
        // outer index range [ua, ub]; a smooth mask (Sec. VI) replaces it by
        // its support {w > 0} and weights the terms
        int ua = I.a, ub = I.b;
        const float* w = nullptr;
        if (I.mask >= 0) {
            float* wt = S(e, 4);
            const MaskInfo mi = mask_weights(e, I, wt, nullptr, nullptr);
            if (!mi.any) {
                for (int t = threadIdx.x; t < L; t += blockDim.x) out[t] = -e.P->rho_pad;
                break;
            }
            ua = mi.klo;
            ub = mi.khi;
            w = wt;
        }
        if (!is_smooth(I)) {
            if (ub < 0 && I.mask < 0) until_hard_unb(e, ua, phi, psi, out, nullptr, nullptr, nullptr);
            else until_hard(e, ua, ub, phi, psi, out, nullptr, nullptr, nullptr, nullptr);
        } else {
            const float bl = pbeta(e, I) * LOG2E;
            int M;
            if (until_ref(phi, psi, L, bl, *e.sh, M)) {
                double* Ep = (double*)S(e, 0);
                double* Eq = (double*)S(e, 2);
                until_terms(phi, psi, L, bl, M, Ep, Eq);
                // the backward's recompute keeps Z in the instruction's slot pair for the adjoint
                double* zs = bwdmap ? (double*)slot(e, I.coef) : nullptr;
                until_smooth_fwd_d(e, ua, ub, w, Ep, Eq, out, zs, bl, M);
                break;
            }
            SP* Ephi = (SP*)S(e, 0);
            SP* Epsi = (SP*)S(e, 2);
            for (int j = threadIdx.x; j < L; j += blockDim.x) {
                Ephi[j] = sp_leaf(-bl * phi[j]);
                Epsi[j] = sp_leaf(-bl * psi[j]);
            }
            __syncthreads();
            until_smooth_fwd(e, ua, ub, w, Ephi, Epsi, out, bl);
        }
        break;
    }
    default:
        break;
    }
    __syncthreads();
}

// Adjoint of one instruction (backward slot map).  Children adjoints are
// written (not accumulated): every node has exactly one parent.
DEV void exec_adj(const Env& e, const Instr& I, float* mask_part)
{
    const int L = e.L;
    const float sg = (I.flags & F_MIN) ? -1.f : 1.f;
    const float* g = slot(e, I.g_out);
    switch (I.kind) {
    case K_TRUE:
    case K_LIN:
    case K_NORM:
        break;
    case K_NOT: {
        float* gu = slot(e, I.g_in0);
        for (int t = threadIdx.x; t < L; t += blockDim.x) gu[t] = -g[t];
        break;
    }
    case K_NARY:
        op_nary_bwd(e, I);
        break;
    case K_WIN: {
        const float* u = slot(e, I.b_in0);
        float* gu = slot(e, I.g_in0);
        const int khi = (I.flags & F_UNB) ? -1 : I.b;
        const float padv = e.P->coef[I.coef];
        if (!is_smooth(I)) {
            int* js = (int*)S(e, 4);
            win_hard(e, u, S(e, 5), js, sg, I.a, khi, I.pad, padv, (VI*)S(e, 0), (VI*)S(e, 2));
            win_hard_adj(e, g, gu, js, (double*)S(e, 6));
            break;
        }
        if (I.flags & F_SOFT) {
            // d out_t / d u_j = p_j(t) (1 + k (u_j - out_t)), p_j(t) = 2^{z_j} / S0(t), k = sg beta:
            // gu_j = 2^{z_j} [(1 + k u_j) sum_t G_t / S0(t) - k sum_t G_t out_t / S0(t)]
            // over the t whose window holds j (transposed window sums)
            // A LAST pad adds, per output, np copies of u_{L-1}: p_v(t) np (1 + k (u_{L-1} - out_t)).
            const float bl = pbeta(e, I) * LOG2E, kap = sg * bl / LOG2E;
            const float* out = slot(e, I.b_out);
            const int n = L - I.a;
            SP* den = (SP*)S(e, 6);
            win_smooth_sum(e, u, den, sg * bl, I.a, khi, I.pad, padv, (SP*)S(e, 0), (SP*)S(e, 2));
            SP* h = (SP*)S(e, 0);
            SP* h2 = (SP*)S(e, 8);
            float lastpad = 0.f;
            const SP zv = sp_leaf(sg * bl * u[L - 1]);
            for (int t = threadIdx.x; t < L; t += blockDim.x) {
                SP a = sp_zero(), b2 = sp_zero();
                if (t < n) {
                    const SP d = den[t];
                    a = SP{g[t] / d.s, -d.r};
                    b2 = SP{g[t] * out[t] / d.s, -d.r};
                }
                h[t] = a;
                h2[t] = b2;
                if (khi >= 0 && I.pad == PAD_LAST && t + khi > L - 1) {
                    const int np = min(khi - I.a + 1, t + khi - (L - 1));
                    const float pv = sp_ratio(zv, den[t]);
                    lastpad += g[t] * (float)np * pv * (1.f + kap * (u[L - 1] - out[t]));
                }
            }
            if (I.pad == PAD_LAST) lastpad = wg_sum(lastpad, *e.sh);
            __syncthreads();
            SP* res = (SP*)S(e, 4);
            SP* res2 = (SP*)S(e, 10);
            win_smooth_adj_sum(e, h, (SP*)S(e, 2), res, I.a, khi, n);
            win_smooth_adj_sum(e, h2, (SP*)S(e, 2), res2, I.a, khi, n);
            for (int j = threadIdx.x; j < L; j += blockDim.x) {
                const SP r1 = res[j], r2 = res2[j];
                const SP c = sp_add(SP{r1.s * (1.f + kap * u[j]), r1.r}, SP{-kap * r2.s, r2.r});
                float vj = sp_times_exp2(c, sg * bl * u[j]);
                if (j == L - 1) vj += lastpad;
                gu[j] = vj;
            }
            break;
        }
        const float bl = pbeta(e, I) * LOG2E;
        const float* out = slot(e, I.b_out);
        const bool unb = khi < 0;
        const int n = L - I.a;
        SP* h = (SP*)S(e, 0);
        float lastpad = 0.f;
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            const float O = sg * bl * out[t];
            const bool real = t < n;
            const bool padded = !unb && I.pad != PAD_NEUTRAL && t + khi > L - 1;
            SP hv = sp_zero();
            if (real || padded) {
                SP q = sp_leaf(-O);
                hv = SP{g[t] * q.s, q.r};
            }
            h[t] = real ? hv : sp_zero();
            if (padded && I.pad == PAD_LAST) {
                const int np = min(unb ? 0 : khi - I.a + 1, t + khi - (L - 1));
                lastpad += (float)np * sp_times_exp2(hv, sg * bl * u[L - 1]);
            }
        }
        lastpad = wg_sum(lastpad, *e.sh);
        SP* res = (SP*)S(e, 4);
        win_smooth_adj_sum(e, h, (SP*)S(e, 2), res, I.a, khi, n);
        for (int j = threadIdx.x; j < L; j += blockDim.x) {
            float v = sp_times_exp2(res[j], sg * bl * u[j]);
            if (j == L - 1) v += lastpad;
            gu[j] = v;
        }
        break;
    }
    case K_MASK: {
        const float* u = slot(e, I.b_in0);
        float* gu = slot(e, I.g_in0);
        float* w = S(e, 6);
        float* dwa = S(e, 7);
        float* dwb = S(e, 8);
        MaskInfo mi = mask_weights(e, I, w, dwa, dwb);
        const bool padm = I.pad != PAD_NEUTRAL && !(I.flags & F_MASK_UNB);
        MaskTail mt{INT_MAX, -1, 0.0, 0.0, 0.0};
        if (padm) mt = mask_tail(e, I, true);
        const int kall = mi.any ? mi.klo : mt.lo;            // whole support
        const int khi_all = mt.hi >= 0 ? mt.hi : mi.khi;
        const bool anyk = mi.any || mt.hi >= 0;
        if (!is_smooth(I) || !anyk) {
            if (!anyk) {
                for (int j = threadIdx.x; j < L; j += blockDim.x) gu[j] = 0.f;
            } else {
                const int khi = ((I.flags & F_MASK_UNB) && khi_all == L - 1) ? -1 : khi_all;
                int* js = (int*)S(e, 4);
                win_hard(e, u, S(e, 5), js, sg, kall, khi, padm ? I.pad : PAD_NEUTRAL, mask_padv(I),
                         (VI*)S(e, 0), (VI*)S(e, 2));
                win_hard_adj(e, g, gu, js, (double*)S(e, 10));
            }
            if (I.mslot >= 0 && threadIdx.x == 0) { mask_part[2 * I.mslot] = 0.f; mask_part[2 * I.mslot + 1] = 0.f; }
            break;
        }
        const float bl = pbeta(e, I) * LOG2E;
        const float* out = slot(e, I.b_out);
        const bool core = mi.clo <= mi.chi;
        SP* h = (SP*)S(e, 0);
        SP* hb = (SP*)S(e, 9);      // band copy of h (the scans consume h)
        SP* E = (SP*)S(e, 11);
        const int nvalid = mi.any ? L - mi.klo : 0;
        float pa = 0.f, pb = 0.f;
        float lastpad = 0.f;
        if (padm) {
            // pad copies: out_t gains TW_t 2^{z_v}; its share of the sum is
            // f_t = TW_t 2^{z_v - O_t}, giving d/du_{L-1} (LAST) = f_t and
            // d/da = TWa_t / TW_t * f_t / beta (d/db alike)
            float* TW = S(e, 13);
            float* TWa = S(e, 14);
            float* TWb = S(e, 15);
            tail_weights(w, TW, L, mt.s, *e.sh);
            tail_weights(dwa, TWa, L, mt.sa, *e.sh);
            tail_weights(dwb, TWb, L, mt.sb, *e.sh);
            const float zv = sg * bl * (I.pad == PAD_LAST ? u[L - 1] : mask_padv(I));
            const float ib0 = sg / pbeta(e, I);
            for (int t = threadIdx.x; t < L; t += blockDim.x) {
                if (t + khi_all <= L - 1 || !(TW[t] > 0.f)) continue;
                const float f = exp2f(zv - sg * bl * out[t] + log2f(TW[t]));
                const float gf = g[t] * f;
                pa += ib0 * gf * (TWa[t] / TW[t]);
                pb += ib0 * gf * (TWb[t] / TW[t]);
                lastpad += gf;
            }
            if (I.pad == PAD_LAST) lastpad = wg_sum(lastpad, *e.sh);
        }
        for (int t = threadIdx.x; t < L; t += blockDim.x) {
            E[t] = sp_leaf(sg * bl * u[t]);
            SP hv = sp_zero();
            if (t < nvalid) {
                SP q = sp_leaf(-sg * bl * out[t]);
                hv = SP{g[t] * q.s, q.r};
            }
            h[t] = hv;
            hb[t] = hv;
        }
        __syncthreads();
        // d/da, d/db: per t, sum over the support bands of dw_k 2^{z_{t+k} - O_t}
        for (int t = threadIdx.x; t < nvalid; t += blockDim.x) {
            SPD aa{0.0, SP_NEG}, ab{0.0, SP_NEG};
            const int b0 = mi.klo, b1 = core ? mi.clo - 1 : mi.khi;
            for (int k = b0; k <= b1 && t + k < L; ++k) {
                aa = spd_add(aa, SP{dwa[k] * E[t + k].s, E[t + k].r});
                ab = spd_add(ab, SP{dwb[k] * E[t + k].s, E[t + k].r});
            }
            if (core)
                for (int k = mi.chi + 1; k <= mi.khi && t + k < L; ++k) {
                    aa = spd_add(aa, SP{dwa[k] * E[t + k].s, E[t + k].r});
                    ab = spd_add(ab, SP{dwb[k] * E[t + k].s, E[t + k].r});
                }
            const float O = sg * bl * out[t];
            const float ib = sg * g[t] / pbeta(e, I);
            pa += ib * sp_times_exp2(spd_to_sp(aa), -O);
            pb += ib * sp_times_exp2(spd_to_sp(ab), -O);
        }
        pa = wg_sum(pa, *e.sh);
        pb = wg_sum(pb, *e.sh);
        if (I.mslot >= 0 && threadIdx.x == 0) { mask_part[2 * I.mslot] = pa; mask_part[2 * I.mslot + 1] = pb; }
        // dx: core via the transposed van Herk sum, bands term by term
        SP* res = (SP*)S(e, 4);
        if (core) {
            const int khi = ((I.flags & F_MASK_UNB) && mi.chi == L - 1) ? -1 : mi.chi;
            win_smooth_adj_sum(e, h, (SP*)S(e, 2), res, mi.clo, khi, nvalid);
        }
        for (int j = threadIdx.x; j < L; j += blockDim.x) {
            // signed adjoint terms: accumulate with a double mantissa
            SPD a{0.0, SP_NEG};
            if (core) a = spd_add(a, SP{res[j].s * mi.wc, res[j].r});
            const int b0 = mi.klo, b1 = core ? mi.clo - 1 : mi.khi;
            for (int k = b0; k <= b1 && j - k >= 0; ++k) a = spd_add(a, SP{w[k] * hb[j - k].s, hb[j - k].r});
            if (core)
                for (int k = mi.chi + 1; k <= mi.khi && j - k >= 0; ++k)
                    a = spd_add(a, SP{w[k] * hb[j - k].s, hb[j - k].r});
            float v = sp_times_exp2(spd_to_sp(a), sg * bl * u[j]);
            if (padm && I.pad == PAD_LAST && j == L - 1) v += lastpad;
            gu[j] = v;
        }
        break;
    }
    case K_UNTIL: {
        const float* phi = slot(e, I.b_in0);
        const float* psi = slot(e, I.b_in1);
        float* gphi = slot(e, I.g_in0);
        float* gpsi = slot(e, I.g_in1);
        for (int t = threadIdx.x; t < L; t += blockDim.x) { gphi[t] = 0.f; gpsi[t] = 0.f; }
        __syncthreads();
        int ua = I.a, ub = I.b;
        const float *w = nullptr, *dwa = nullptr, *dwb = nullptr;
        bool none = false;
        if (I.mask >= 0) {
            float* wt = S(e, 4);
            float* wa = S(e, 5);
            float* wb = S(e, 6);
            const MaskInfo mi = mask_weights(e, I, wt, wa, wb);
            none = !mi.any;
            ua = mi.klo;
            ub = mi.khi;
            w = wt;
            dwa = wa;
            dwb = wb;
        }
        float pa = 0.f, pb = 0.f;
        if (none) {
            // empty support: constant output
        } else if (!is_smooth(I)) {
            if (ub < 0 && I.mask < 0) until_hard_unb(e, ua, phi, psi, nullptr, g, gphi, gpsi);
            else until_hard(e, ua, ub, phi, psi, nullptr, g, gphi, gpsi, (int*)S(e, 0));
        } else {
            const float bl = pbeta(e, I) * LOG2E;
            const int bmax = ub < 0 ? L - 1 : min(ub, L - 1);
            int M;
            if (until_ref(phi, psi, L, bl, *e.sh, M)) {
                double* Ep = (double*)S(e, 0);
                double* Eq = (double*)S(e, 2);
                until_terms(phi, psi, L, bl, M, Ep, Eq);
                const double* zs = (const double*)slot(e, I.coef);
                until_smooth_adj_d(e, ua, ub, w, dwa, dwb, Ep, Eq, zs, g, gphi, gpsi, (double*)S(e, UCK_UNIT),
                                   bmax / UCK + 1, pa, pb);
            } else {
                SP* Ephi = (SP*)S(e, 0);
                SP* Epsi = (SP*)S(e, 2);
                for (int j = threadIdx.x; j < L; j += blockDim.x) {
                    Ephi[j] = sp_leaf(-bl * phi[j]);
                    Epsi[j] = sp_leaf(-bl * psi[j]);
                }
                __syncthreads();
                until_smooth_adj(e, ua, ub, w, dwa, dwb, Ephi, Epsi, g, gphi, gpsi, (SP*)S(e, UCK_UNIT),
                                 bmax / UCK + 1, pa, pb);
            }
        }
        if (I.mslot >= 0) {
            // d out / d w_i = Y_i / (beta Z); zero for the hard form
            const float ib = is_smooth(I) ? 1.f / pbeta(e, I) : 0.f;
            const float sa = wg_sum(pa * ib, *e.sh);
            const float sb = wg_sum(pb * ib, *e.sh);
            if (threadIdx.x == 0) { mask_part[2 * I.mslot] = sa; mask_part[2 * I.mslot + 1] = sb; }
        }
        // d phi / d psi are sums of scaled terms: convert the scaled psi/phi sums in place
        break;
    }
    default:
        break;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ kernels

struct MaskTab;


DEV bool next_item(const KArgs& ka, Shared& sh, int64_t& item, bool first, int64_t B)
{
    if (ka.scan) {
        // the rows blockIdx.x + i gridDim.x whose flag is set, in order of i
        // (the flags of up to blockDim.x rows are read at once)
        __syncthreads();
        const int64_t nrow = B > (int64_t)blockIdx.x ? (B - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
        for (int64_t i0 = first ? 0 : (int64_t)sh.scan_pos; i0 < nrow; i0 += blockDim.x) {
            if (threadIdx.x == 0) sh.scan_min = INT_MAX;
            __syncthreads();
            const int64_t i = i0 + threadIdx.x;
            if (i < nrow && ka.scan[blockIdx.x + i * gridDim.x] != 0) atomicMin(&sh.scan_min, (int)i);
            __syncthreads();
            const int f = sh.scan_min;
            __syncthreads();
            if (f != INT_MAX) {
                item = (int64_t)blockIdx.x + (int64_t)f * gridDim.x;
                if (threadIdx.x == 0) sh.scan_pos = f + 1;
                return true;
            }
        }
        return false;
    }
    if (!ka.persistent) {
        item = blockIdx.x;
        return first;
    }
    __syncthreads();
    if (threadIdx.x == 0) sh.ints[7] = atomicAdd(ka.counter, 1);
    __syncthreads();
    item = sh.ints[7];
    return true;
}

template <bool BWD>
__global__ void __launch_bounds__(MAX_NT) stl_exec_kernel(DevPlan plan, Batch bt, KArgs ka)
{
    extern __shared__ float smem[];
    __shared__ Shared sh;
    // The plan is the first kernel argument, at offset 0 of the kernarg
    // segment: read it there.  (Taking the address of the by-value parameter
    // lets the compiler copy all of it into per-lane private memory, which it
    // does once the kernel body grows past some size.)
    const DevPlan* P = (const DevPlan*)__builtin_amdgcn_kernarg_segment_ptr();
    (void)plan;
    float* arena = ka.garena ? ka.garena + (size_t)blockIdx.x * ka.arena_floats : smem;
    const int nslots = BWD ? P->n_slots_bwd : P->n_slots_fwd;
    const int Lc = bt.Lcap;
    int64_t item = 0;
    bool first = true;
    // an empty fix-up list: nothing to do and no counter to clear
    if (ka.list_mode && *ka.list_count <= 0) return;
    while (next_item(ka, sh, item, first, bt.B)) {
        first = false;
        const int64_t nitems = ka.list_mode ? min(max((int64_t)*ka.list_count, (int64_t)0), bt.B) : bt.B;
        if (item >= nitems) break;
        const int64_t b = ka.list_mode ? (int64_t)ka.list[item] : (bt.order ? (int64_t)bt.order[item] : item);
        const int64_t off = bt.offsets ? bt.offsets[b] : b * bt.T;
        const int64_t len = bt.offsets ? bt.offsets[b + 1] - off : bt.T;
        if (len <= 0) {
            // an empty trajectory adds nothing to d/da, d/db: its partials
            // are still read by the reduction
            if (BWD)
                for (int q = threadIdx.x; q < ka.part_stride * P->n_masks * 2; q += blockDim.x)
                    ka.mask_part[b * ka.part_stride * P->n_masks * 2 + q] = 0.f;
            continue;
        }
        if (len > Lc) {
            // trajectory longer than the launch's capacity: report NaN
            for (int64_t t = threadIdx.x; t < len; t += blockDim.x) {
                if (!BWD) ka.root[off + t] = NAN;
                else for (int d = 0; d < bt.D; ++d) ka.dx[(off + t) * bt.D + d] = NAN;
            }
            if (BWD)
                for (int q = threadIdx.x; q < ka.part_stride * P->n_masks * 2; q += blockDim.x)
                    ka.mask_part[b * ka.part_stride * P->n_masks * 2 + q] = NAN;
            continue;
        }
        Env e;
        e.P = P;
        e.x = bt.x + off * bt.D;
        e.params = ka.params;
        e.L = (int)len;
        e.Lc = Lc;
        e.D = bt.D;
        e.arena = arena;
        e.scr = arena + (size_t)nslots * Lc;
        e.sh = &sh;
        for (int k = 0; k < P->n_ins; ++k) exec_fwd(e, P->ins[k], BWD);
        if (!BWD) {
            const float* r = slot(e, P->ins[P->root].f_out);
            for (int t = threadIdx.x; t < e.L; t += blockDim.x) ka.root[off + t] = r[t];
            if (ka.nodes) {
                // every node trace (debug): rerun with all slots kept is not
                // needed because the forward map keeps node outputs until
                // overwritten; the host gives every node its own slot when
                // traces are requested.
                // [n_nodes][N_total]: a ragged batch's N_total is offsets[B], read
                // here on the device so the host never waits for it
                const int64_t ntot = bt.offsets ? bt.offsets[bt.B] : ka.n_total;
                for (int k = 0; k < P->n_ins; ++k) {
                    const Instr& I = P->ins[k];
                    if (I.node < 0) continue;
                    const float* s = slot(e, I.f_out);
                    for (int t = threadIdx.x; t < e.L; t += blockDim.x)
                        ka.nodes[(int64_t)I.node * ntot + off + t] = s[t];
                }
            }
            __syncthreads();
        } else {
            float* gr = slot(e, P->ins[P->root].g_out);
            for (int t = threadIdx.x; t < e.L; t += blockDim.x) gr[t] = ka.G[off + t];
            __syncthreads();
            // one partial row per trajectory; with part_stride > 1 (rows per
            // chunk of the matrix-core path) the trajectory's other rows are cleared
            float* mp = ka.mask_part + b * ka.part_stride * P->n_masks * 2;
            for (int q = threadIdx.x; q < (ka.part_stride - 1) * P->n_masks * 2; q += blockDim.x)
                mp[P->n_masks * 2 + q] = 0.f;
            for (int k = P->n_ins - 1; k >= 0; --k) exec_adj(e, P->ins[k], mp);
            op_dx(e, ka.dx + off * bt.D);
            __syncthreads();
        }
    }
    if (ka.list_mode) {
        // the last work-group out clears the item counter, the list count and
        // this ticket, so that the next call through the same counters starts
        // from zero without a clearing kernel
        __syncthreads();
        if (threadIdx.x == 0 && atomicAdd(ka.counter + 2, 1) == (int)gridDim.x - 1) {
            ka.counter[0] = 0;
            ka.counter[1] = 0;
            ka.counter[2] = 0;
        }
    }
}

// One work-group per parameter p: d/dp is the sum, over the per-trajectory
// rows and in a fixed order, of every (mask, bound) column of the partials
// whose parameter index is p (two mask nodes may share a, b); parameters no
// mask bound names get 0.  The kernels overwrite gp, they never accumulate.
__global__ void __launch_bounds__(1024) stl_reduce_params(const float* part, int64_t rows, int n_masks, DevPlan plan,
                                                          float* gp)
{
    __shared__ float red[1024];
    const int tid = threadIdx.x;
    const int p = blockIdx.x;
    int cols[2 * MAX_MASKS];
    int nc = 0;
    for (int q = 0; q < 2 * n_masks; ++q)
        if (plan.mask_param[q >> 1] + (q & 1) == p) cols[nc++] = q;
    if (nc == 0) {
        if (tid == 0) gp[p] = 0.f;
        return;
    }
    // each thread: rows tid, tid + 1024, ... (four independent sums, added in a fixed order)
    float s4[4] = {0.f, 0.f, 0.f, 0.f};
    const int64_t stride = (int64_t)blockDim.x;
    for (int64_t r0 = tid; r0 < rows; r0 += 4 * stride) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t r = r0 + u * stride;
            if (r < rows)
                for (int k = 0; k < nc; ++k) s4[u] += part[r * 2 * n_masks + cols[k]];
        }
    }
    red[tid] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    __syncthreads();
    for (int k = blockDim.x >> 1; k > 0; k >>= 1) {
        if (tid < k) red[tid] += red[tid + k];
        __syncthreads();
    }
    if (tid == 0) gp[p] = red[0];
}

__global__ void stl_zero_counter(int* c) { if (threadIdx.x < 3) c[threadIdx.x] = 0; }

__global__ void stl_fill_int(int* p, int64_t n, int v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace stlmi

#include "stl_fused.h"
#include "stl_interval.h"
#include "stl_mx.h"

namespace stlmi {

}  // namespace stlmi

// ------------------------------------------------------------------ launch helpers (host)

namespace stlmi {

size_t scratch_floats(int Lc, int nt, int max_until_b)
{
    size_t s = (size_t)SCR_UNITS * Lc + 64;
    // smooth Until checkpoints: nt * (b/UCK + 1) scaled pairs, placed at unit UCK_UNIT
    size_t ck = (size_t)nt * (size_t)(max_until_b / UCK + 1) * 2;
    if ((size_t)UCK_UNIT * Lc + ck + 64 > s) s = (size_t)UCK_UNIT * Lc + ck + 64;
    return s;
}

hipError_t launch_exec(bool bwd, const DevPlan& plan, const Batch& bt, const KArgs& ka, int grid, int nt,
                       size_t lds_bytes, hipStream_t s)
{
    if (bwd) {
        hipLaunchKernelGGL(stl_exec_kernel<true>, dim3(grid), dim3(nt), lds_bytes, s, plan, bt, ka);
    } else {
        hipLaunchKernelGGL(stl_exec_kernel<false>, dim3(grid), dim3(nt), lds_bytes, s, plan, bt, ka);
    }
    return hipGetLastError();
}

hipError_t set_max_lds(size_t bytes)
{
    hipError_t e1 = hipFuncSetAttribute((const void*)stl_exec_kernel<false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipError_t e2 = hipFuncSetAttribute((const void*)stl_exec_kernel<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e1 != hipSuccess ? e1 : e2;
}

size_t fused_lds(int Lc, int n, int D, bool bwd)
{
    (void)n;
    (void)D;
    (void)bwd;
    return fused_lds_bytes(Lc);
}

int fused_max_T() { return FNT * FNO; }

size_t mask_tab_bytes() { return sizeof(MaskTab); }

hipError_t launch_fused(bool bwd, const DevPlan& plan, const Batch& bt, const KArgs& ka, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(stl_mask_tables, dim3(plan.fused.n), dim3(256), 0, s, plan, ka.params, (int)bt.T,
                       (MaskTab*)ka.tabs, ka.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)bt.B), block(FNT);
    const bool full = bt.T == FNT * FNO && bt.Lcap == FNT * FNO;
#define STLMI_FUSED_CASE(NN)                                                                            \
    case NN:                                                                                            \
        if (bwd && full)                                                                                \
            hipLaunchKernelGGL((stl_fused_bwd<NN, true>), grid, block, lds, s, plan, bt, ka);           \
        else if (bwd)                                                                                   \
            hipLaunchKernelGGL((stl_fused_bwd<NN, false>), grid, block, lds, s, plan, bt, ka);          \
        else if (full)                                                                                  \
            hipLaunchKernelGGL((stl_fused_fwd<NN, true>), grid, block, lds, s, plan, bt, ka);           \
        else                                                                                            \
            hipLaunchKernelGGL((stl_fused_fwd<NN, false>), grid, block, lds, s, plan, bt, ka);          \
        break;
    switch (plan.fused.n) {
        STLMI_FUSED_CASE(1)
        STLMI_FUSED_CASE(2)
        STLMI_FUSED_CASE(3)
        STLMI_FUSED_CASE(4)
    default:
        return hipErrorInvalidValue;
    }
#undef STLMI_FUSED_CASE
    return hipGetLastError();
}

hipError_t set_max_lds_fused(size_t bytes)
{
    const void* fns[] = {
        (const void*)stl_fused_fwd<1, false>, (const void*)stl_fused_fwd<2, false>, (const void*)stl_fused_fwd<3, false>,
        (const void*)stl_fused_fwd<4, false>, (const void*)stl_fused_bwd<1, false>, (const void*)stl_fused_bwd<2, false>,
        (const void*)stl_fused_bwd<3, false>, (const void*)stl_fused_bwd<4, false>, (const void*)stl_fused_fwd<1, true>,
        (const void*)stl_fused_fwd<2, true>, (const void*)stl_fused_fwd<3, true>, (const void*)stl_fused_fwd<4, true>,
        (const void*)stl_fused_bwd<1, true>, (const void*)stl_fused_bwd<2, true>, (const void*)stl_fused_bwd<3, true>,
        (const void*)stl_fused_bwd<4, true>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero_counter(int* c, hipStream_t s)
{
    hipLaunchKernelGGL(stl_zero_counter, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(stl_fill_int, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_reduce_params(const float* part, int64_t B, const DevPlan& plan, float* gp, hipStream_t s)
{
    if (plan.n_params < 1) return hipSuccess;
    hipLaunchKernelGGL(stl_reduce_params, dim3(plan.n_params), dim3(1024), 0, s, part, B, plan.n_masks, plan, gp);
    return hipGetLastError();
}

// ------------------------------------------------------------------ matrix-core path

// dynamic LDS of the matrix-core kernels: the rings (n masks x 16 rows), the
// result buffers, and the backward's derivative tiles
size_t mx_lds_bytes(int n, int D, bool bwd)
{
    return (size_t)n * MXG * MXRS + mx_xch_bytes(n, D, bwd) + (bwd ? (size_t)n * NDMAX * 2 * 64 * 16 : 0);
}
size_t mx_static_lds() { return sizeof(MxShared); }

hipError_t set_max_lds_mx(size_t bytes)
{
    hipError_t e = hipSuccess;
#define STLMI_MX_ATTR(KK)                                                                                   \
    {                                                                                                     \
        const hipError_t e2 = hipFuncSetAttribute((const void*)KK, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                                  (int)bytes);                                            \
        if (e2 != hipSuccess) e = e2;                                                                     \
    }
#define STLMI_MX_ATTR2(NN, DD)                                                                            \
    STLMI_MX_ATTR((stl_mx_fwd<NN, DD, false>)) STLMI_MX_ATTR((stl_mx_fwd<NN, DD, true>))                  \
    STLMI_MX_ATTR((stl_mx_bwd<NN, DD, false>)) STLMI_MX_ATTR((stl_mx_bwd<NN, DD, true>))
    STLMI_MX_ATTR2(1, 1) STLMI_MX_ATTR2(1, 2) STLMI_MX_ATTR2(2, 1) STLMI_MX_ATTR2(2, 2)
#undef STLMI_MX_ATTR2
#undef STLMI_MX_ATTR
    return e;
}

static bool al16(const void* p) { return (((uintptr_t)p) & 15) == 0; }

// the forward or backward kernel over groups of 16 trajectories.  The
// 16-byte load / store variants need T a multiple of 4 and 16-byte aligned
// arrays (x; forward: root and saved values; backward: G, saved values, dx).
hipError_t launch_mx(bool bwd, const DevPlan& plan, const Batch& bt, const KArgs& ka, const MxArgs& mx, size_t lds,
                     hipStream_t s)
{
    // (forward: 2n matrix and 4n staging waves; backward: 2n of each)
    const dim3 grid((unsigned)((bt.B + MXG - 1) / MXG)), block((bwd ? 256 : 384) * plan.fused.n);
    const bool d2 = bt.D == 2;
    const bool vec = bt.T % 4 == 0 && bt.T >= 4 && al16(bt.x) &&
                     (bwd ? al16(ka.G) && al16(ka.saved_in) && al16(ka.dx) : al16(ka.root) && al16(ka.saved));
#define STLMI_MX_K(NN, DD, VV)                                                                            \
    if (bwd) hipLaunchKernelGGL((stl_mx_bwd<NN, DD, VV>), grid, block, lds, s, plan, bt, ka, mx);          \
    else hipLaunchKernelGGL((stl_mx_fwd<NN, DD, VV>), grid, block, lds, s, plan, bt, ka, mx);
#define STLMI_MX_CASE(NN)                                                                                 \
    case NN:                                                                                              \
        if (d2 && vec) { STLMI_MX_K(NN, 2, true) }                                                        \
        else if (d2) { STLMI_MX_K(NN, 2, false) }                                                         \
        else if (vec) { STLMI_MX_K(NN, 1, true) }                                                         \
        else { STLMI_MX_K(NN, 1, false) }                                                                 \
        break;
    switch (plan.fused.n) {
        STLMI_MX_CASE(1)
        STLMI_MX_CASE(2)
    default:
        return hipErrorInvalidValue;
    }
#undef STLMI_MX_CASE
#undef STLMI_MX_K
    return hipGetLastError();
}

}  // namespace stlmi
