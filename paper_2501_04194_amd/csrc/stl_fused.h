// Fused fast path for formulas of the shape
//     root = smooth And/Or over up to 4 smooth-mask Eventually/Always nodes,
//            each over a linear predicate (or a single such mask node),
// e.g. Eventually~[a,b](x0 > 0) and~ Always~[a,b](x1 < 0.5) with the smooth
// time mask of arXiv 2501.04194 Sec. VI.  Included by stl_kernels.hip.
//
// One work-group (FNT threads) computes the whole formula for one trajectory
// of length L <= FNT * FNO; thread i owns timesteps [FNO*i, FNO*i + FNO) and
// keeps their mask traces in registers.  For each mask node the terms
// 2^{z_j}, z = sign * beta * log2(e) * u, are held in fp64 relative to one
// per-trajectory reference exponent (fp64's exponent range makes per-window
// rescaling unnecessary; fp64 FMA runs at the non-packed fp32 FMA rate on
// CDNA4).  The constant-weight core of the mask is a van Herk window: block
// prefix and block suffix sums (segmented scans done in registers and wave
// shuffles), every window is suffix(start) + prefix(end), no subtraction.
// The two sigmoid bands are register-blocked FMA loops over LDS with fp64
// weights read as scalars from a per-call table.  Two LDS arrays suffice:
// the terms (later the adjoint terms, later the block prefixes) and the
// block suffixes, so four work-groups fit in one compute unit.  LDS arrays
// hold one pad element per 8 so that lanes owning 8 consecutive elements hit
// distinct banks.
//
// Trajectories whose signal range exceeds fp64's exponent range, and masks
// whose bands are wider than FMAXB, are handed to the generic executor.
#pragma once

namespace stlmi {

constexpr int FNT = 256;          // threads per work-group
constexpr int FNO = 8;            // consecutive timesteps per thread
constexpr int FNW = FNT / 64;     // waves per work-group
constexpr int FMAXB = 512;        // max padded width of one band weight array
constexpr int FHOFF = 32;         // room for the shift of the term / adjoint copies (elements)
constexpr int FTAIL = 16;         // high-side zero padding (elements)
constexpr int FMAXN = 4;          // mask nodes under the root
// waves per SIMD the kernels are compiled for (VGPR budget 512 / waves); LDS
// allows four work-groups (of one wave per SIMD) per compute unit
constexpr int FWAVES_FWD = 3;
constexpr int FWAVES_BWD = 2;
// more mask nodes keep more per-mask state in registers: fewer waves
constexpr int fused_waves(int n, int w) { return n <= 2 ? w : (n == 3 ? (w > 2 ? 2 : w) : 1); }

// Per-mask tables, computed once per call by stl_mask_tables.
struct MaskTab {
    int ok;                     // 0: bands too wide for the fused path
    int any;                    // support {w > 0} is non-empty
    int klo, khi, clo, chi;     // support and constant core (clo > chi: no core)
    int core, K, off;           // van Herk block length and head offset (core only)
    unsigned kmag;              // div_magic(K)
    int kl0, nWl, kr0, nWr;     // bands: first offset and width (a multiple of 8; zero weights pad it)
    int nz_al, nz_bl;           // left band: d/da, d/db weights not all zero
    int nz_ar, nz_br;           // right band: same
    float wc;                   // core weight
    double Wl[FMAXB], Wr[FMAXB];                          // band weights
    // reversed d w / d a and d w / d b (D[nW-1-s]), for the transposed sums of the backward
    double Dalr[FMAXB + 8], Darr[FMAXB + 8], Dblr[FMAXB + 8], Dbrr[FMAXB + 8];
    double Wlr[FMAXB + 8], Wrr[FMAXB + 8];                // reversed (W[nW-1-s]), for transposed sums
};

struct FShared {
    double wv[FNW];
    int wf[FNW];
    double wv2[FNW];
    int wf2[FNW];
    int wi[FNW];
    int wn[FMAXN][FNW];
    int wq[FMAXN][FNW];
    double wp[2 * FMAXN][FNW];
    // per mask node (filled by fused_enter): sign, beta, predicate coefficient
    // offset, gradient slot; read with a runtime mask index from LDS rather
    // than from the kernel argument
    float m_sg[FMAXN], m_beta[FMAXN];
    int m_slot[FMAXN];
    float m_coef[FMAXN][1 + MAX_D];     // linear predicate: c, w[0..D)
    int ints[8];
    int fragile;
};

DEV int PX(int j) { return j + (j >> 3); }
__host__ __device__ constexpr int px_len(int n) { return n + (n >> 3) + 16; }
DEV int round8(int v) { return (v + 7) & ~7; }

// n / K for 0 <= n, n * K < 2^32, with mag = floor(2^32 / K) + 1 (exact in
// that range); K = 1 is coded as mag = 0
DEV int div_mag(int n, unsigned mag) { return mag ? (int)__umulhi((unsigned)n, mag) : n; }
__host__ __device__ inline unsigned div_magic(int K) { return K > 1 ? (unsigned)(0x100000000ull / (unsigned)K) + 1u : 0u; }

// Wave reductions: xor butterflies over each 32-lane half with ds_swizzle
// (the lane pattern is an immediate, so no per-lane address registers stay
// live), then the two halves combined from lanes 0 and 32.  The result is
// wave-uniform; sums use a fixed order.
template <int XM>
DEV int swz_xor(int v)
{
    return __builtin_amdgcn_ds_swizzle(v, (XM << 10) | 0x1F);
}

template <int XM>
DEV double swz_xor(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = swz_xor<XM>((int)b), hi = swz_xor<XM>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

DEV int wave_max_i(int v)
{
    v = max(v, swz_xor<1>(v));
    v = max(v, swz_xor<2>(v));
    v = max(v, swz_xor<4>(v));
    v = max(v, swz_xor<8>(v));
    v = max(v, swz_xor<16>(v));
    return max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 32));
}

DEV double wave_sum_d(double v)
{
    v += swz_xor<1>(v);
    v += swz_xor<2>(v);
    v += swz_xor<4>(v);
    v += swz_xor<8>(v);
    v += swz_xor<16>(v);
    const long long b = __double_as_longlong(v);
    const long long b0 = ((long long)__builtin_amdgcn_readlane((int)(b >> 32), 0) << 32) |
                         (unsigned)__builtin_amdgcn_readlane((int)b, 0);
    const long long b1 = ((long long)__builtin_amdgcn_readlane((int)(b >> 32), 32) << 32) |
                         (unsigned)__builtin_amdgcn_readlane((int)b, 32);
    return __longlong_as_double(b0) + __longlong_as_double(b1);
}

DEV int wg_max_i(int v, FShared& sh)
{
    v = wave_max_i(v);
    if ((threadIdx.x & 63) == 0) sh.wi[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = sh.wi[0];
    for (int w = 1; w < FNW; ++w) r = max(r, sh.wi[w]);
    __syncthreads();
    return r;
}

// deterministic work-group sum (fixed shuffle tree, waves in order)
DEV double wg_sum_d(double v, FShared& sh)
{
    v = wave_sum_d(v);
    if ((threadIdx.x & 63) == 0) sh.wv[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh.wv[0];
    for (int w = 1; w < FNW; ++w) r += sh.wv[w];
    __syncthreads();
    return r;
}

// hardware 2^x and log2(x) (one instruction each, about 1 ulp); used only
// where the argument keeps the result a normal float
DEV float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
DEV float lg2(float x) { return __builtin_amdgcn_logf(x); }

DEV float log2d(double s)
{
    int e;
    double m = frexp(s, &e);                    // m in [0.5, 1)
    return (float)e + lg2((float)m);
}

// 2^d as a double for d <= 0 (log2 units): exact exponent split
DEV double exp2d_neg(float d)
{
    float fl = floorf(d);
    int ip = (int)fmaxf(fl, -1100.f);
    return ldexp((double)ex2(d - fl), ip);      // d - fl in [0, 1)
}

// DPP lane moves (bound_ctrl: lanes with no source read 0): 0x101 + k row_shl,
// 0x111 + k row_shr (within rows of 16), 0x130 wave_shl:1, 0x138 wave_shr:1
template <int CTRL>
DEV int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
DEV double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

DEV double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    return __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(b >> 32), l) << 32) |
                                (unsigned)__builtin_amdgcn_readlane((int)b, l));
}

// one level of both segmented scans inside the rows: up from the lane SHR
// below, down from the lane SHL above
template <int SHR, int SHL>
DEV void scan_row_step(double& a, int& f, double& r, int& g)
{
    const double ao = dpp_d<SHR>(a), ro = dpp_d<SHL>(r);
    const int fo = dpp_i<SHR>(f), go = dpp_i<SHL>(g);
    if (!f) a = ao + a;
    f |= fo;
    if (!g) r = r + ro;
    g |= go;
}

// Both block scans of the same values in one pass (two barriers in all):
// pre = segmented inclusive prefix with heads where (p + off) % K == 0, suf =
// segmented inclusive suffix with tails where (p + off) % K == K-1 and at n-1
// (the van Herk block prefixes and suffixes), written to the padded LDS
// arrays pre[0..n) and suf[0..n).  Values past n must be 0.
DEV void fscan2(const double* vin, double* pre, double* suf, int n, int K, unsigned kmag, int off, FShared& sh,
                int tid)
{
    const int lane = tid & 63, w = tid >> 6;
    const int c0 = FNO * tid;
    double vf[FNO], vr[FNO];
    int hf = 0, hr = 0;
    int rem = c0 + off - div_mag(c0 + off, kmag) * K;
#pragma unroll
    for (int i = 0; i < FNO; ++i) {
        const int p = c0 + i;
        const bool in = p < n;
        hf |= (in && rem == 0) ? (1 << i) : 0;
        hr |= (in && (p == n - 1 || rem == K - 1)) ? (1 << i) : 0;
        rem = rem + 1 == K ? 0 : rem + 1;
    }
    double af = 0.0, ar = 0.0;
#pragma unroll
    for (int i = 0; i < FNO; ++i) { af = ((hf >> i) & 1) ? vin[i] : af + vin[i]; vf[i] = af; }
#pragma unroll
    for (int i = FNO - 1; i >= 0; --i) { ar = ((hr >> i) & 1) ? vin[i] : vin[i] + ar; vr[i] = ar; }
    // wave-level segmented scans of the per-thread totals (forward: up; reverse:
    // down): DPP row shifts within each row of 16 lanes (lanes shifted in from
    // outside the row read the identity (0, no head)), then the row totals
    // (read with readlane) carried into the later (earlier) rows
    double a = af, r = ar;
    int f = hf != 0, g = hr != 0;
    scan_row_step<0x111, 0x101>(a, f, r, g);
    scan_row_step<0x112, 0x102>(a, f, r, g);
    scan_row_step<0x114, 0x104>(a, f, r, g);
    scan_row_step<0x118, 0x108>(a, f, r, g);
    {
        const int row = lane >> 4;
        // up: carries C1 = T0, C2 = C1 (+) T1, C3 = C2 (+) T2 (T_q = row q's total, at lane 16q + 15)
        const double t0 = readlane_d(a, 15), t1 = readlane_d(a, 31), t2 = readlane_d(a, 47);
        const int u0 = __builtin_amdgcn_readlane(f, 15), u1 = __builtin_amdgcn_readlane(f, 31),
                  u2 = __builtin_amdgcn_readlane(f, 47);
        const double c2 = u1 ? t1 : t0 + t1, c3 = u2 ? t2 : c2 + t2;
        const int h2 = u0 | u1, h3 = h2 | u2;
        const double cu = row == 1 ? t0 : (row == 2 ? c2 : c3);
        const int hu = row == 1 ? u0 : (row == 2 ? h2 : h3);
        if (row > 0) {
            if (!f) a = cu + a;
            f |= hu;
        }
        // down: carries D2 = T3, D1 = T2 (+) D2, D0 = T1 (+) D1 (T_q at lane 16q)
        const double s1 = readlane_d(r, 16), s2 = readlane_d(r, 32), s3 = readlane_d(r, 48);
        const int v1 = __builtin_amdgcn_readlane(g, 16), v2 = __builtin_amdgcn_readlane(g, 32),
                  v3 = __builtin_amdgcn_readlane(g, 48);
        const double d1 = v2 ? s2 : s2 + s3, d0 = v1 ? s1 : s1 + d1;
        const int k1 = v2 | v3, k0 = v1 | k1;
        const double cd = row == 2 ? s3 : (row == 1 ? d1 : d0);
        const int hd = row == 2 ? v3 : (row == 1 ? k1 : k0);
        if (row < 3) {
            if (!g) r = r + cd;
            g |= hd;
        }
    }
    // the previous lane's inclusive value (up) and the next lane's (down)
    const double exf = dpp_d<0x138>(a), exr = dpp_d<0x130>(r);
    const int eff = dpp_i<0x138>(f), efr = dpp_i<0x130>(g);
    if (lane == 63) { sh.wv[w] = a; sh.wf[w] = f; }
    if (lane == 0) { sh.wv2[w] = r; sh.wf2[w] = g; }
    __syncthreads();
    double cf = 0.0, cr = 0.0;
    for (int w2 = 0; w2 < w; ++w2) cf = sh.wf[w2] ? sh.wv[w2] : cf + sh.wv[w2];
    for (int w2 = FNW - 1; w2 > w; --w2) cr = sh.wf2[w2] ? sh.wv2[w2] : cr + sh.wv2[w2];
    const double carf = eff ? exf : cf + exf;
    const double carr = efr ? exr : cr + exr;
    bool gf = true, gr = true;
#pragma unroll
    for (int i = 0; i < FNO; ++i) { gf = gf && !((hf >> i) & 1); if (gf) vf[i] += carf; }
#pragma unroll
    for (int i = FNO - 1; i >= 0; --i) { gr = gr && !((hr >> i) & 1); if (gr) vr[i] += carr; }
#pragma unroll
    for (int i = 0; i < FNO; ++i)
        if (c0 + i < n) {
            pre[PX(c0 + i)] = vf[i];
            suf[PX(c0 + i)] = vr[i];
        }
    __syncthreads();
}

// ------------------------------------------------------------------ band sums

// The weight tables are written by an earlier launch and only read here:
// reading them through the constant address space lets uniform reads become
// scalar loads (weights as scalar FMA operands, no vector memory traffic).
typedef const __attribute__((address_space(4))) double* cdptr;

// S[i] += sum_{dk<8} W[dk] * window[i + dk], window = (a[0..7], b[0..7])
DEV void fma_block(double* S, const double* __restrict__ W, const double* a, const double* b)
{
    const cdptr Wc = (cdptr)W;
#pragma unroll
    for (int dk = 0; dk < 8; ++dk) {
        const double w = Wc[dk];
#pragma unroll
        for (int i = 0; i < FNO; ++i) {
            const int p = i + dk;
            S[i] = fma(w, p < 8 ? a[p] : b[p - 8], S[i]);
        }
    }
}

// element index of the zero block (8 zeros) at the end of each LDS array
__host__ __device__ constexpr int fused_zero_at(int Lc) { return (Lc + FHOFF + FTAIL + 7) & ~7; }
// padded length of each LDS array (doubles)
__host__ __device__ constexpr int fused_arr_len(int Lc) { return px_len(fused_zero_at(Lc) + 8); }

// The 8 elements starting at element p (a multiple of 8) of the padded array
// A, or the zero block at element zp when [p, p+8) is not inside the written
// range [0, hi).
DEV void load8z(double* r, const double* A, int p, int hi, int zp)
{
    const int pp = (p >= 0 && p + 8 <= hi) ? p : zp;
    const double* a = A + PX(pp);
#pragma unroll
    for (int c = 0; c < 8; ++c) r[c] = a[c];
}

// S[i] += sum_{s=s0}^{nW-1} W[s] * A[PX(base + i + s)], i in [0, FNO).  base is
// this lane's window start (a multiple of 8); s0 and nW are the same for the
// whole wave (multiples of 8), so the loop is uniform and W (a uniform
// pointer) is read with scalar loads.  Blocks outside the written range [0, hi)
// of A read as the zero block at zp: windows of lanes near either end of the
// trajectory need no lane-dependent trip count.  The two 8-element halves of
// the window alternate roles, so nothing is moved.
DEV void band_acc(const double* A, int base, const double* __restrict__ W, int s0, int nW, int hi, int zp, double* S)
{
    if (s0 >= nW) return;
    int p = base + s0;
    double x[8], y[8];
    load8z(x, A, p, hi, zp);
    load8z(y, A, p + 8, hi, zp);
    int s = s0;
    for (;;) {
        fma_block(S, W + s, x, y);
        s += 8;
        if (s >= nW) break;
        p += 8;
        load8z(x, A, p + 8, hi, zp);
        fma_block(S, W + s, y, x);
        s += 8;
        if (s >= nW) break;
        p += 8;
        load8z(y, A, p + 8, hi, zp);
    }
}

// timestep of the first lane of this thread's wave (uniform)
DEV int wave_c0(int tid) { return __builtin_amdgcn_readfirstlane(FNO * tid); }

// ------------------------------------------------------------------ tables

struct TabShared {
    int ints[8];
};

// One work-group per mask node: support, core and band weight tables.  Work-group
// 0 also resets the two counters of the fused launch (the generic executor's work
// counter and the hand-off list length).
__global__ void __launch_bounds__(256) stl_mask_tables(DevPlan plan, const float* params, int L, MaskTab* tabs,
                                                       int* counters)
{
    __shared__ TabShared sh;
    if (blockIdx.x == 0 && threadIdx.x < 3) counters[threadIdx.x] = 0;
    const DevPlan& P = plan;
    const int m = blockIdx.x;
    const Instr& I = P.ins[P.fused.ins[m]];
    MaskTab& T = tabs[m];
    const MaskInfo mi = mask_info(params, I, L, sh, nullptr, nullptr, nullptr);
    const bool core = mi.any && mi.clo <= mi.chi;
    const int le = core ? mi.clo : mi.khi + 1;
    const int kl0 = mi.any ? mi.klo : 0;
    const int nWl = mi.any ? round8(le - kl0) : 0;
    const int rs = mi.chi + 1, re = mi.khi + 1;
    const int kr0 = core ? rs : 0;
    const int nWr = core ? round8(re - kr0) : 0;
    const bool ok = nWl <= FMAXB && nWr <= FMAXB;
    if (threadIdx.x == 0) {
        T.ok = ok;
        T.any = mi.any;
        T.klo = mi.klo;
        T.khi = mi.khi;
        T.clo = mi.clo;
        T.chi = mi.chi;
        T.core = core;
        T.K = core ? mi.chi - mi.clo + 1 : 1;
        T.off = core ? (T.K - mi.clo % T.K) % T.K : 0;
        T.kmag = div_magic(T.K);
        T.kl0 = kl0;
        T.nWl = nWl;
        T.kr0 = kr0;
        T.nWr = nWr;
        T.wc = core ? mi.wc : 0.f;
        sh.ints[4] = 0;
    }
    __syncthreads();
    if (!ok) return;
    const MaskP mp = mask_params(params + I.mask, I.flags & F_MASK_UNB);
    for (int s = threadIdx.x; s < FMAXB + 8; s += blockDim.x) {
        float wl = 0.f, wr = 0.f;
        if (s < nWl) {
            const int k = kl0 + s;
            if (k >= mi.klo && k < le) wl = mask_wk(mp, k);
        }
        if (s < nWr) {
            const int k = kr0 + s;
            if (k >= rs && k < re) wr = mask_wk(mp, k);
        }
        if (s < FMAXB) {
            T.Wl[s] = wl;
            T.Wr[s] = wr;
        }
        // reversed: Wlr[s] = Wl[nWl - 1 - s] for 0 <= s < nWl, and the same for
        // the derivatives
        float wlr = 0.f, dal = 0.f, dbl = 0.f, wrr = 0.f, dar = 0.f, dbr = 0.f;
        if (s < nWl) {
            const int k = kl0 + nWl - 1 - s;
            if (k >= mi.klo && k < le) wlr = mask_wk(mp, k, &dal, &dbl);
        }
        if (s < nWr) {
            const int k = kr0 + nWr - 1 - s;
            if (k >= rs && k < re) wrr = mask_wk(mp, k, &dar, &dbr);
        }
        T.Wlr[s] = wlr;
        T.Wrr[s] = wrr;
        T.Dalr[s] = dal;
        T.Dblr[s] = dbl;
        T.Darr[s] = dar;
        T.Dbrr[s] = dbr;
        if (dal != 0.f) atomicOr(&sh.ints[4], 1);
        if (dbl != 0.f) atomicOr(&sh.ints[4], 2);
        if (dar != 0.f) atomicOr(&sh.ints[4], 4);
        if (dbr != 0.f) atomicOr(&sh.ints[4], 8);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T.nz_al = (sh.ints[4] & 1) != 0;
        T.nz_bl = (sh.ints[4] & 2) != 0;
        T.nz_ar = (sh.ints[4] & 4) != 0;
        T.nz_br = (sh.ints[4] & 8) != 0;
    }
}

// ------------------------------------------------------------------ forward pieces

struct FOp {
    float sg, bl, beta;
    const float* cf;     // predicate: [0] c, [1..] w
    int R;               // reference exponent
};

DEV void fop_init(const DevPlan& P, int m, const FShared& sh, FOp& op)
{
    op.cf = sh.m_coef[m];
    op.sg = sh.m_sg[m];
    op.beta = sh.m_beta[m];
    op.bl = op.beta * LOG2E;
    op.R = 0;
}

// Shift of the copy of the terms read by a band starting at offset k0:
// term j sits at padded position PX(j + band_shift(k0)), so that every
// thread's band window starts on a multiple of 8 whatever k0 is.
DEV int band_shift(int k0) { return 8 - (k0 & 7); }

// Exponents z = sign * beta * log2(e) * (w . x_j - c) of every mask node for
// this thread's timesteps (-inf past the end).  The thread's FNO state rows are
// FNO*D consecutive floats, read once for all masks (as four 16-byte loads
// when D == 2).
template <int N>
DEV void fused_exponents(const FShared& sh, const float* x, int L, int D, int c0, float (&z)[N][FNO])
{
    const float* xr = x + (size_t)c0 * D;
    if (D == 2 && c0 + FNO <= L && (((uintptr_t)xr) & 15) == 0) {
        float v[2 * FNO];
        const float4* q = (const float4*)xr;
#pragma unroll
        for (int k = 0; k < FNO / 2; ++k) {
            const float4 a = q[k];
            v[4 * k] = a.x;
            v[4 * k + 1] = a.y;
            v[4 * k + 2] = a.z;
            v[4 * k + 3] = a.w;
        }
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const float* cf = sh.m_coef[m];
            const float sg = sh.m_sg[m], bl = sh.m_beta[m] * LOG2E;
#pragma unroll
            for (int i = 0; i < FNO; ++i) {
                float t = 0.f;
                t = fmaf(cf[1], v[2 * i], t);
                t = fmaf(cf[2], v[2 * i + 1], t);
                z[m][i] = sg * bl * (t - cf[0]);
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < FNO; ++i) {
        const int j = c0 + i;
        float t[N];
#pragma unroll
        for (int m = 0; m < N; ++m) t[m] = 0.f;
        if (j < L) {
            for (int d = 0; d < D; ++d) {
                const float xv = xr[(size_t)i * D + d];
#pragma unroll
                for (int m = 0; m < N; ++m) t[m] = fmaf(sh.m_coef[m][1 + d], xv, t[m]);
            }
        }
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const float sg = sh.m_sg[m], bl = sh.m_beta[m] * LOG2E;
            z[m][i] = j < L ? sg * bl * (t[m] - sh.m_coef[m][0]) : -INFINITY;
        }
    }
}

// Per-trajectory reference exponents R_m = ceil(max_j z_m[j]) of every mask,
// one work-group reduction for all of them.
template <int N>
DEV void fused_refs(const float (&z)[N][FNO], int (&R)[N], FShared& sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        float zm = -INFINITY;
#pragma unroll
        for (int i = 0; i < FNO; ++i) zm = fmaxf(zm, z[m][i]);
        int v = (int)ceilf(fminf(fmaxf(zm, -1e9f), 1e9f));
        v = wave_max_i(v);
        if (lane == 0) sh.wn[m][w] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < N; ++m) {
        int r = sh.wn[m][0];
        for (int k = 1; k < FNW; ++k) r = max(r, sh.wn[m][k]);
        R[m] = r;
    }
}

// E[j] = 2^{z_j - R} for this thread's timesteps: registers e[] and two
// padded LDS copies, A shifted by shA and B shifted by shB (one per band),
// with a zero tail.  Starts with a barrier, so earlier reads of A and B by
// other threads are complete, and ends with one.
DEV void fused_terms(const float* z, int R, int L, double* e, double* A, double* B, int shA, int shB, FShared& sh,
                     int tid)
{
    const int c0 = FNO * tid;
    __syncthreads();
    bool frag = false;
#pragma unroll
    for (int i = 0; i < FNO; ++i) {
        const int j = c0 + i;
        if (j < L) {
            const float d = z[i] - (float)R;
            frag |= d < -1000.f;
            e[i] = exp2d_neg(d);
            A[PX(j + shA)] = e[i];
            B[PX(j + shB)] = e[i];
        } else {
            e[i] = 0.0;
            if (j < L + FTAIL) {
                A[PX(j + shA)] = 0.0;
                B[PX(j + shB)] = 0.0;
            }
        }
    }
    for (int j = max(L, FNO * FNT) + tid; j < L + FTAIL; j += FNT) {
        A[PX(j + shA)] = 0.0;
        B[PX(j + shB)] = 0.0;
    }
    if (frag) sh.fragile = 1;
    __syncthreads();
}

// Forward trace of one mask node for this thread's timesteps (out[0..FNO)).
// Uses A (terms, then block prefixes) and Bs (block suffixes).
DEV void mask_trace(const DevPlan& P, const MaskTab& T, FOp& op, const float* z, int L, int Lc, double* A,
                    double* Bs, float* out, FShared& sh, int tid)
{
    const int c0 = FNO * tid;
    double e[FNO];
    const int shA = band_shift(T.kl0), shB = band_shift(T.kr0);
    fused_terms(z, op.R, L, e, A, Bs, shA, shB, sh, tid);
    if (!T.any) {
#pragma unroll
        for (int i = 0; i < FNO; ++i) out[i] = -op.sg * P.rho_pad;
        return;
    }
    double S[FNO];
#pragma unroll
    for (int i = 0; i < FNO; ++i) S[i] = 0.0;
    {
        // the wave's first lane has the longest valid window: its limit serves the wave
        const int lim = L - wave_c0(tid), zp = fused_zero_at(Lc);
        band_acc(A, c0 + T.kl0 + shA, T.Wl, 0, min(T.nWl, max(0, round8(lim - T.kl0))), L + FTAIL + shA, zp, S);
        if (T.core)
            band_acc(Bs, c0 + T.kr0 + shB, T.Wr, 0, min(T.nWr, max(0, round8(lim - T.kr0))), L + FTAIL + shB, zp, S);
    }
    if (T.core) {
        // block prefixes and suffixes of the terms (A and Bs are overwritten only
        // after the scan's own barrier, when every band read is done)
        fscan2(e, A, Bs, L, T.K, T.kmag, T.off, sh, tid);
        if (c0 < L) {
            const int K = T.K, s0 = c0 + T.clo;
            const int qL = div_mag(L - 1 + T.off, T.kmag);
            int q = div_mag(s0 + T.off, T.kmag), rem = s0 + T.off - q * K;
            const double wc = (double)T.wc;
#pragma unroll
            for (int i = 0; i < FNO; ++i) {
                const int s = s0 + i;
                if (s <= L - 1) {
                    const bool clipped = s + K - 1 > L - 1;
                    const int en = clipped ? L - 1 : s + K - 1;
                    const bool same = rem == 0 || (clipped && qL == q);
                    S[i] = fma(wc, same ? Bs[PX(s)] : Bs[PX(s)] + A[PX(en)], S[i]);
                }
                if (++rem == K) { rem = 0; ++q; }
            }
        }
    }
    const float ibl = 1.f / op.bl;
#pragma unroll
    for (int i = 0; i < FNO; ++i) {
        const int t = c0 + i;
        out[i] = -op.sg * P.rho_pad;
        if (t < L && t + T.klo <= L - 1) {
            if (!(S[i] > 0.0)) sh.fragile = 1;
            out[i] = op.sg * ((float)op.R + log2d(S[i])) * ibl;
        }
    }
}

// Opaque copy of the thread index: the per-mask loops take their index
// arithmetic from it, so the compiler does not hoist one copy per mask out of
// the loop and keep them all live.
DEV int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    __builtin_assume(t >= 0 && t < FNT);
    return t;
}

// row m of a per-mask register array, for a runtime (uniform) m
template <int N>
DEV void select_row(const float (&a)[N][FNO], int m, float* r)
{
#pragma unroll
    for (int i = 0; i < FNO; ++i) {
        r[i] = a[0][i];
#pragma unroll
        for (int k = 1; k < N; ++k) r[i] = k == m ? a[k][i] : r[i];
    }
}

template <int N>
DEV int select_int(const int (&a)[N], int m)
{
    int r = a[0];
#pragma unroll
    for (int k = 1; k < N; ++k) r = k == m ? a[k] : r;
    return r;
}

// every mask trace for this thread's timesteps (tr[m][i]); ends with a barrier
template <int N>
DEV void mask_traces(const DevPlan& P, const KArgs& ka, const float (&z)[N][FNO], const int (&R)[N], int L, int Lc,
                     double* A, double* Bs, float (&tr)[N][FNO], FShared& sh)
{
#pragma unroll 1
    for (int m = 0; m < N; ++m) {
        FOp op;
        fop_init(P, m, sh, op);
        op.R = select_int<N>(R, m);
        float zm[FNO], out[FNO];
        select_row<N>(z, m, zm);
        mask_trace(P, ka.tabs[m], op, zm, L, Lc, A, Bs, out, sh, opaque_tid());
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int i = 0; i < FNO; ++i) tr[k][i] = k == m ? out[i] : tr[k][i];
    }
    __syncthreads();
}

// root = smooth n-ary over the mask traces v[0..N) at one timestep (same
// formula as the generic op); wts receives d root / d v_k
template <int N>
DEV float fused_root(const DevPlan& P, const float* params, const float* v, float* wts)
{
    const FusedDesc& F = P.fused;
    if (N == 1 && !F.root_nary) {
        if (wts) wts[0] = 1.f;
        return v[0];
    }
    const float sg = F.nary_min ? -1.f : 1.f;
    const float bl = params[F.nary_beta] * LOG2E, ibl = 1.f / bl;
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < N; ++k) m = fmaxf(m, sg * v[k]);
    float s = 0.f, ek[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ek[k] = ex2((sg * v[k] - m) * bl);      // <= 1; tiny terms may flush to 0
        s += ek[k];
    }
    const float r = sg * (m + lg2(s) * ibl);   // s in [1, N]
    if (wts) {
        // softmax weights e_k / s (s >= 1: the largest term is 1)
        const float is = __builtin_amdgcn_rcpf(s);
#pragma unroll
        for (int k = 0; k < N; ++k) wts[k] = ek[k] * is;
    }
    return r;
}

// LDS: two padded fp64 arrays
__host__ __device__ inline size_t fused_lds_bytes(int Lc)
{
    return (size_t)2 * fused_arr_len(Lc) * sizeof(double);
}

DEV bool fused_enter(const DevPlan& P, const KArgs& ka, FShared& sh, double* A, double* Bs, int Lc)
{
    if (threadIdx.x < 16) (threadIdx.x < 8 ? A : Bs)[(fused_zero_at(Lc) >> 3) * 9 + (threadIdx.x & 7)] = 0.0;
    if (threadIdx.x < FMAXN && (int)threadIdx.x < P.fused.n) {
        const int m = threadIdx.x;
        const Instr& I = P.ins[P.fused.ins[m]];
        sh.m_sg[m] = (I.flags & F_MIN) ? -1.f : 1.f;
        sh.m_beta[m] = ka.params[I.beta];
        sh.m_slot[m] = I.mslot;
    }
    if ((int)threadIdx.x < P.fused.n * (1 + MAX_D)) {
        const int m = threadIdx.x / (1 + MAX_D), k = threadIdx.x % (1 + MAX_D);
        sh.m_coef[m][k] = k <= P.D ? P.coef[P.ins[P.fused.pred[m]].coef + k] : 0.f;
    }
    bool ok = true;
    for (int m = 0; m < P.fused.n; ++m) ok = ok && ka.tabs[m].ok;
    if (threadIdx.x == 0) sh.fragile = 0;
    __syncthreads();
    return ok;
}

DEV void fused_handoff(const KArgs& ka, int64_t b)
{
    if (threadIdx.x == 0) ka.list[atomicAdd(ka.list_count, 1)] = (int)b;
}

// 8 consecutive floats at p[c0 ..] (positions < L only)
DEV void store8(float* p, int c0, int L, const float* v)
{
    if (c0 + FNO <= L && (((uintptr_t)(p + c0)) & 15) == 0) {
        float4* q = (float4*)(p + c0);
        q[0] = make_float4(v[0], v[1], v[2], v[3]);
        q[1] = make_float4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int i = 0; i < FNO; ++i)
            if (c0 + i < L) p[c0 + i] = v[i];
    }
}

DEV void load8f(const float* p, int c0, int L, float* v)
{
    if (c0 + FNO <= L && (((uintptr_t)(p + c0)) & 15) == 0) {
        const float4* q = (const float4*)(p + c0);
        const float4 a = q[0], b = q[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int i = 0; i < FNO; ++i) v[i] = c0 + i < L ? p[c0 + i] : 0.f;
    }
}

// FULL: T == FNT * FNO exactly (every thread owns FNO valid timesteps; the
// bounds checks fold away)
template <int N, bool FULL>
__global__ void __launch_bounds__(FNT, fused_waves(N, FWAVES_FWD)) stl_fused_fwd(DevPlan plan, Batch bt, KArgs ka)
{
    extern __shared__ double fsm[];
    __shared__ FShared sh;
    const DevPlan& P = plan;
    const int L = FULL ? FNT * FNO : (int)bt.T, Lc = FULL ? FNT * FNO : bt.Lcap, D = bt.D;
    __builtin_assume(threadIdx.x < FNT);
    const int64_t b = blockIdx.x;
    const int pl = fused_arr_len(Lc);
    double* A = fsm;
    double* Bs = A + pl;
    if (!fused_enter(P, ka, sh, A, Bs, Lc)) {
        if (ka.saved_flag && threadIdx.x == 0) ka.saved_flag[b] = 0;
        fused_handoff(ka, b);
        return;
    }
    const float* x = bt.x + b * (int64_t)L * D;
    const int c0 = FNO * threadIdx.x;
    float z[N][FNO], tr[N][FNO];
    int R[N];
    fused_exponents<N>(sh, x, L, D, c0, z);
    fused_refs<N>(z, R, sh);
    mask_traces<N>(P, ka, z, R, L, Lc, A, Bs, tr, sh);
    if (sh.fragile) {
        if (ka.saved_flag && threadIdx.x == 0) ka.saved_flag[b] = 0;
        fused_handoff(ka, b);
        return;
    }
    float r[FNO];
#pragma unroll
    for (int i = 0; i < FNO; ++i) {
        float v[N];
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = tr[m][i];
        r[i] = fused_root<N>(P, ka.params, v, nullptr);
    }
    store8(ka.root + b * (int64_t)L, c0, L, r);
    if (ka.saved) {
        // mask-node traces for the backward: [n][B][T], valid when the flag is 1
#pragma unroll
        for (int m = 0; m < N; ++m) store8(ka.saved + ((int64_t)m * bt.B + b) * L, c0, L, tr[m]);
        if (threadIdx.x == 0) ka.saved_flag[b] = 1;
    }
}

// S[i] += sum_{dk<8} W[dk] window[i + dk] and Sd[i] += sum_{dk<8} Wd[dk]
// window[i + dk]: two weight sets over one window
DEV void fma_block2(double* S, double* Sd, const double* __restrict__ W, const double* __restrict__ Wd,
                    const double* a, const double* b)
{
    const cdptr Wc = (cdptr)W, Dc = (cdptr)Wd;
#pragma unroll
    for (int dk = 0; dk < 8; ++dk) {
        const double w = Wc[dk], d = Dc[dk];
#pragma unroll
        for (int i = 0; i < FNO; ++i) {
            const int p = i + dk;
            const double v = p < 8 ? a[p] : b[p - 8];
            S[i] = fma(w, v, S[i]);
            Sd[i] = fma(d, v, Sd[i]);
        }
    }
}

// band_acc with a second weight set Wd summed into Sd over the same windows
DEV void band_acc2(const double* A, int base, const double* __restrict__ W, const double* __restrict__ Wd, int s0,
                   int nW, int hi, int zp, double* S, double* Sd)
{
    if (s0 >= nW) return;
    int p = base + s0;
    double x[8], y[8];
    load8z(x, A, p, hi, zp);
    load8z(y, A, p + 8, hi, zp);
    int s = s0;
    for (;;) {
        fma_block2(S, Sd, W + s, Wd + s, x, y);
        s += 8;
        if (s >= nW) break;
        p += 8;
        load8z(x, A, p + 8, hi, zp);
        fma_block2(S, Sd, W + s, Wd + s, y, x);
        s += 8;
        if (s >= nW) break;
        p += 8;
        load8z(y, A, p + 8, hi, zp);
    }
}

// sum_i E_i v[i] for this thread's timesteps, E_i = 2^{z_i - R} from the exponents
DEV double edot(const float* zm, int R, int c0, int L, const double* v)
{
    double p = 0.0;
#pragma unroll
    for (int i = 0; i < FNO; ++i)
        if (c0 + i < L) p = fma(exp2d_neg(zm[i] - (float)R), v[i], p);
    return p;
}

// Transposed sums of one band over the adjoint terms H (window of output j
// starting at base + s0): Bd += sum_s Wr[s] H, and for the band's derivative
// tables (reversed d/da Dar, d/db Dbr) pa, pb += sum_j E_j sum_s Dr[s] H.
// The first non-zero derivative table shares the pass with Bd; a second one
// (a band that spans both a and b) takes a pass of its own.
DEV void band_bwd(const double* A, int base, const double* Wr, const double* Dar, const double* Dbr, int nza,
                  int nzb, int s0, int nW, int hi, int zp, const float* zm, int R, int c0, int L, double* Bd,
                  double& pa, double& pb)
{
    double Dd[FNO];
#pragma unroll
    for (int i = 0; i < FNO; ++i) Dd[i] = 0.0;
    band_acc2(A, base, Wr, nza ? Dar : Dbr, s0, nW, hi, zp, Bd, Dd);
    const double p1 = edot(zm, R, c0, L, Dd);
    if (nza) pa += p1;
    else pb += p1;
    if (nza && nzb) {
#pragma unroll
        for (int i = 0; i < FNO; ++i) Dd[i] = 0.0;
        band_acc(A, base, Dbr, s0, nW, hi, zp, Dd);
        pb += edot(zm, R, c0, L, Dd);
    }
}

template <int N, bool FULL>
__global__ void __launch_bounds__(FNT, fused_waves(N, FWAVES_BWD)) stl_fused_bwd(DevPlan plan, Batch bt, KArgs ka)
{
    extern __shared__ double fsm[];
    __shared__ FShared sh;
    const DevPlan& P = plan;
    const FusedDesc& F = P.fused;
    const int L = FULL ? FNT * FNO : (int)bt.T, Lc = FULL ? FNT * FNO : bt.Lcap, D = bt.D;
    __builtin_assume(threadIdx.x < FNT);
    const int64_t b = blockIdx.x;
    const int pl = fused_arr_len(Lc);
    double* A = fsm;             // terms E, then adjoint terms H, then block prefixes (shifted copies
    double* Bs = A + pl;         // for the left band in A, the right band in Bs), then block suffixes
    if (!fused_enter(P, ka, sh, A, Bs, Lc)) { fused_handoff(ka, b); return; }
    const float* x = bt.x + b * (int64_t)L * D;
    const int c0 = FNO * threadIdx.x;
    float z[N][FNO], tr[N][FNO];
    int R[N];
    // the loads of G and of the kept mask traces go out first, so that their
    // latency overlaps the exponents of x
    float G8[FNO];
    load8f(ka.G + b * (int64_t)L, c0, L, G8);
    if (ka.saved_in) {
#pragma unroll
        for (int m = 0; m < N; ++m) load8f(ka.saved_in + ((int64_t)m * bt.B + b) * L, c0, L, tr[m]);
    }
    fused_exponents<N>(sh, x, L, D, c0, z);
    fused_refs<N>(z, R, sh);
    if (!(ka.saved_in && ka.saved_flag[b] == 1)) {
        // forward recompute of every mask trace (the n-ary adjoint needs all of them)
        mask_traces<N>(P, ka, z, R, L, Lc, A, Bs, tr, sh);
        if (sh.fragile) { fused_handoff(ka, b); return; }
    }
    // adjoint of each mask trace, G_m = G * d root / d trace_m (gm), and its
    // exponent O_t = sg beta log2(e) trace_m (in place of the trace)
    float gm[N][FNO];
    {
#pragma unroll
        for (int i = 0; i < FNO; ++i) {
            float v[N], wts[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = tr[k][i];
            fused_root<N>(P, ka.params, v, wts);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const Instr& I = P.ins[F.ins[k]];
                const float sg = (I.flags & F_MIN) ? -1.f : 1.f;
                gm[k][i] = c0 + i < L ? G8[i] * wts[k] : 0.f;
                tr[k][i] = sg * ka.params[I.beta] * LOG2E * v[k];
            }
        }
    }
    float* mp = ka.mask_part + b * P.n_masks * 2;
    // Q_m: the per-trajectory exponent of max |G_m 2^{-O}|, all masks in one reduction
    int Qs[N];
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const int klo = ka.tabs[m].klo;
            int qloc = INT_MIN;
#pragma unroll
            for (int i = 0; i < FNO; ++i) {
                const int t = c0 + i;
                if (t < L && t + klo <= L - 1 && gm[m][i] != 0.f) {
                    // frexp exponent of a normal G_m (an upper bound for a subnormal one)
                    const int eg = ((__float_as_int(gm[m][i]) >> 23) & 0xff) - 126;
                    qloc = max(qloc, eg - (int)floorf(tr[m][i]));
                }
            }
            qloc = wave_max_i(qloc);
            if (lane == 0) sh.wq[m][w] = qloc;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < N; ++m) {
            int q = sh.wq[m][0];
            for (int k = 1; k < FNW; ++k) q = max(q, sh.wq[m][k]);
            Qs[m] = q == INT_MIN ? 0 : q;
        }
    }
    float gvs[N][FNO];            // per mask: d root / d (w_m . x_j) for this thread's j
    double pab[2 * N];            // per mask: this thread's d/da, d/db partials
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) pab[k] = 0.0;
#pragma unroll 1
    for (int m = 0; m < N; ++m) {
        const int tid = opaque_tid();
        const int c0 = FNO * tid;
        const MaskTab& T = ka.tabs[m];
        const int mslot = sh.m_slot[m];
        FOp op;
        fop_init(P, m, sh, op);
        op.R = select_int<N>(R, m);
        float g[FNO], om[FNO];        // this mask's G_m and O_t
#pragma unroll
        for (int i = 0; i < FNO; ++i) {
            g[i] = gm[0][i];
            om[i] = tr[0][i];
#pragma unroll
            for (int k = 1; k < N; ++k) {
                g[i] = k == m ? gm[k][i] : g[i];
                om[i] = k == m ? tr[k][i] : om[i];
            }
        }
        float gv[FNO];
        if (!T.any) {
#pragma unroll
            for (int i = 0; i < FNO; ++i) gv[i] = 0.f;
        } else {
            float zm[FNO];
            select_row<N>(z, m, zm);
            // H_t = G_m[t] 2^{-O_t - Q}
            const int Q = select_int<N>(Qs, m);
            double h[FNO];
#pragma unroll
            for (int i = 0; i < FNO; ++i) {
                const int t = c0 + i;
                h[i] = 0.0;
                if (t < L && t + T.klo <= L - 1) {
                    const float fl = floorf(om[i]);
                    h[i] = ldexp((double)(g[i] * ex2(fl - om[i])), -(int)fl - Q);   // fl - om in (-1, 0]
                }
            }
            __syncthreads();              // every read of A and Bs by the previous mask is done
            // adjoint terms H, two shifted copies (A for the left band, Bs for
            // the right) zero padded on both sides: H_t sits at PX(t + hA)
            // with hA = kl0 - 1 (mod 8), so that the transposed window of
            // output j, starting at t = j - kl0 - nWl + 1, starts on a multiple of 8
            const int hA = 24 + ((T.kl0 - 1) & 7), hB = 24 + ((T.kr0 - 1) & 7);
            for (int p = tid; p < 32; p += FNT) {
                if (p < hA) A[PX(p)] = 0.0;
                if (p < hB) Bs[PX(p)] = 0.0;
            }
#pragma unroll
            for (int i = 0; i < FNO; ++i) {
                const int j = c0 + i;
                if (j < L + FTAIL) {
                    const double hv = (j < L) ? h[i] : 0.0;
                    A[PX(j + hA)] = hv;
                    Bs[PX(j + hB)] = hv;
                }
            }
            for (int j = max(L, FNO * FNT) + tid; j < L + FTAIL; j += FNT) {
                A[PX(j + hA)] = 0.0;
                Bs[PX(j + hB)] = 0.0;
            }
            __syncthreads();
            // band sums over H: dx_j += sum_k w_k H_{j-k} = sum_s Wrev[s] H_{j - k0 - nW + 1 + s},
            // and for d/da, d/db the same sums with the derivative weights:
            //   sum_t sg G_m[t]/beta sum_k dw_k 2^{z_{t+k} - O_t} = sg/beta 2^{R+Q} sum_j E_j sum_k dw_k H_{j-k}
            double Bd[FNO];
#pragma unroll
            for (int i = 0; i < FNO; ++i) Bd[i] = 0.0;
            const int zp = fused_zero_at(Lc);
            {
                double pa = 0.0, pb = 0.0;
                // blocks before t = 0 read as zeros; the wave's last lane (base + 8*63)
                // fixes the first block any lane of the wave needs
                const int w0 = wave_c0(tid) + FNO * 63;
                const int base = c0 - T.kl0 - T.nWl + 1 + hA;      // a multiple of 8
                band_bwd(A, base, T.Wlr, T.Dalr, T.Dblr, T.nz_al, T.nz_bl, max(0, -(w0 - T.kl0 - T.nWl + 1 + hA)),
                         T.nWl, L + FTAIL + hA, zp, zm, op.R, c0, L, Bd, pa, pb);
                if (T.core) {
                    const int base2 = c0 - T.kr0 - T.nWr + 1 + hB;
                    band_bwd(Bs, base2, T.Wrr, T.Darr, T.Dbrr, T.nz_ar, T.nz_br,
                             max(0, -(w0 - T.kr0 - T.nWr + 1 + hB)), T.nWr, L + FTAIL + hB, zp, zm, op.R, c0, L, Bd,
                             pa, pb);
                }
                const double k0 = (double)(op.sg / op.beta);
                pa = ldexp(pa, op.R + Q) * k0;
                pb = ldexp(pb, op.R + Q) * k0;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    pab[2 * k] = k == m ? pa : pab[2 * k];
                    pab[2 * k + 1] = k == m ? pb : pab[2 * k + 1];
                }
            }
            // dx core: van Herk over t of H, windows [j - chi, j - clo] (heads at t % K == 0)
            if (T.core) {
                // H again, from this thread's own entries of the copy in A (not
                // kept in registers across the band sums)
                double hr[FNO];
#pragma unroll
                for (int i = 0; i < FNO; ++i) hr[i] = A[PX(c0 + i + hA)];
                // A and Bs receive the block sums after the scan's own barrier
                fscan2(hr, A, Bs, L, T.K, T.kmag, 0, sh, tid);
                const double wc = (double)T.wc;
                const int K = T.K;
                // window of j over t: [j - chi, j - clo]; j - clo <= L - 1 always, so
                // only the start can be clipped (at t = 0, a block start)
                const int stu = c0 - T.chi;
                int rem = stu > 0 ? stu - div_mag(stu, T.kmag) * K : 0;      // (max(0, j - chi)) % K
#pragma unroll
                for (int i = 0; i < FNO; ++i) {
                    const int j = c0 + i;
                    if (j < L) {
                        const int st = max(0, stu + i), en = j - T.clo;
                        if (st <= en) {
                            const bool same = (stu + i < 0) ? en < K : rem == 0;
                            const double c = same ? (rem == 0 ? A[PX(en)] : Bs[PX(st)]) : Bs[PX(st)] + A[PX(en)];
                            Bd[i] = fma(wc, c, Bd[i]);
                        }
                    }
                    if (stu + i >= 0 && ++rem == K) rem = 0;
                }
            }
#pragma unroll
            for (int i = 0; i < FNO; ++i) {
                gv[i] = c0 + i < L ? (float)ldexp(Bd[i] * exp2d_neg(zm[i] - (float)op.R), op.R + Q) : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int i = 0; i < FNO; ++i) gvs[k][i] = k == m ? gv[i] : gvs[k][i];
    }
    // d/da, d/db per mask: deterministic work-group sums (fixed shuffle tree, waves in order)
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < 2 * N; ++k) {
            double v = pab[k];
            v = wave_sum_d(v);
            if (lane == 0) sh.wp[k][w] = v;
        }
        __syncthreads();
        if (threadIdx.x < 2 * N) {
            const int k = threadIdx.x, m = k >> 1;
            double r = sh.wp[k][0];
            for (int ww = 1; ww < FNW; ++ww) r += sh.wp[k][ww];
            if (sh.m_slot[m] >= 0) mp[2 * sh.m_slot[m] + (k & 1)] = (float)r;
        }
    }
    // dx_j = sum_m w_m gv_m[j] (masks in order), this thread's FNO*D consecutive floats
    float* dxr = ka.dx + (b * (int64_t)L + c0) * D;
    if (D == 2 && c0 + FNO <= L && (((uintptr_t)dxr) & 15) == 0) {
        float v[2 * FNO];
#pragma unroll
        for (int i = 0; i < FNO; ++i)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m < N; ++m) acc = acc + sh.m_coef[m][1 + d] * gvs[m][i];
                v[2 * i + d] = acc;
            }
        float4* q = (float4*)dxr;
#pragma unroll
        for (int k = 0; k < FNO / 2; ++k) q[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < FNO; ++i) {
            if (c0 + i >= L) break;
            for (int d = 0; d < D; ++d) {
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m < N; ++m) acc = acc + sh.m_coef[m][1 + d] * gvs[m][i];
                dxr[(size_t)i * D + d] = acc;
            }
        }
    }
}

}  // namespace stlmi
