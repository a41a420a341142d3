// Matrix-core path for formulas of the fused shape
//     root = smooth And/Or over one or two smooth-mask Eventually/Always
//            nodes with bounded masks, each over a linear predicate,
// e.g. Eventually~[a,b](x0 > 0) and~ Always~[a,b](x1 < 0.5) with the smooth
// time mask of arXiv 2501.04194 Sec. VI.  Included by stl_kernels.hip after
// stl_fused.h.
//
// A mask node's trace is out_t = (sg / beta) log sum_k w_k e^{beta sg u_{t+k}}
// (Sec. III-C logsumexp with the Sec. VI weights inside the sum).  With the
// terms E_j = 2^{z_j - R}, z = sg beta log2(e) u, the window sums
// S_t = sum_k w_k E_{t+k} of 16 outputs t and 16 trajectories b are one
// matrix product S = W E: W[t][j] = w_{j - t} (a Toeplitz tile, the same for
// every trajectory and every output tile) and E[j][b] the terms.  The
// product runs on v_mfma_f32_16x16x32_bf16 with each factor split into two
// bf16 parts (x = hi + lo to 2^-18 relative) and three products
// (Wh Eh + Wh El + Wl Eh) accumulated in fp32: every sum has positive terms,
// so its relative error is a few 2^-18 at worst and far smaller on average.
// The weights are divided by the core weight (core offsets have W = 1).
//
// The backward needs, for the adjoint terms H_t = G(t) p_m(t) 2^{-O_t - Q}
// (O_t = sg beta log2(e) out_t, p_m the root's softmax weight of the node),
// the transposed window sums D_j = sum_t w_{j - t} H_t (for d/dx) and
// sum_t dw_{j - t} H_t for the band derivative tables (for d/da, d/db): the
// same products with transposed weight tiles over H.  The forward keeps, per
// mask and output, l = log2 p_m - (O - R) against its own reference R, so the
// backward's adjoint term is one exp2 of l plus a per-trajectory constant.
//
// Tile origins: the forward tiles start at klo rounded down to a multiple
// of 4, the backward tiles at khi rounded up (zero weights in between), so
// that every staged group of 4 positions starts at a multiple of 4; when T is
// a multiple of 4 such a group lies wholly inside or outside the trajectory
// and is loaded with 16-byte loads.
//
// Work decomposition: a work-group takes 16 trajectories from start to end.
// It first derives each mask's support, core and tile geometry from the
// parameters and builds its weight tiles in LDS (no table kernel).  The
// terms (or adjoint terms) of each mask stream through an LDS ring of 640
// positions per trajectory, 128 positions (one block) at a time: in round k
// the matrix waves compute outputs [128 k, 128 k + 128) from blocks
// k .. k+3 (four 16-output tiles per wave, which read the same staged terms
// one K-step apart, so every ring read feeds up to 12 products), while the
// staging waves turn round k-1's sums into outputs and stage block k+4 over
// block k-1.  The reference R of a trajectory's terms is the midpoint of its
// exponents over a strided sample; every staged exponent is checked to lie
// within 100 of it (so that nothing over- or underflows), and a trajectory
// that fails is flagged for the generic executor, which runs after the
// kernel in the same call.  The backward's reference Q comes from the range
// of O the forward recorded.
#pragma once

namespace stlmi {

constexpr int MXG = 16;                 // trajectories per work-group (the MFMA N)
constexpr int NKMAX = 12;               // K-steps (32 offsets each) of a window tile
constexpr int NDMAX = 4;                // derivative tiles per mask (a K-step with d/da and d/db weights has two)
constexpr int MXROUND = 128;            // outputs per round (4 pairs of 16-output tiles)
constexpr int MXBLK = 128;              // positions per staged block
constexpr int MXNBLK = 5;               // blocks in the ring
constexpr int MXRING = MXBLK * MXNBLK;  // ring positions per trajectory
constexpr int MXRS = MXRING / 8 * 32 + 16;   // LDS row stride (bytes): 16 bytes of pad put the 16
                                             // rows a wave reads at once on distinct bank groups
constexpr float MX_HALF = 100.f;       // largest |z - R| (and half the range of O), log2 units
constexpr int MX_MAXN = 2;              // mask nodes under the root

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float mxf4;

// Per-mask quantities of the matrix-core path.  Every work-group of both
// kernels derives them from the mask's parameters at its start (the same
// values everywhere), then builds its weight tiles from per-offset weights
// in LDS.  Tiles are in the lane layout of the MFMA A operand (16 rows x 32
// columns, lane l holds row l % 16, columns 8 (l / 16) .. + 7).
struct MxHead {
    int ok;                    // 0: the window needs more than NKMAX K-steps
    int any;                   // the support {w > 0} is non-empty
    int klo, khi, clo, chi;    // support and constant core (clo > chi: no core)
    int kf, kb;                // tile origins: klo rounded down, khi rounded up to a multiple of 4
    int NK;                    // K-steps of an output tile
    float lscale;              // log2 of the weight scale (the core weight, or 1)
    double scale;
};

// offsets one set of tiles reads: forward tiles w(kf + 32 s + j - t) at
// entry 32 s + j - t + 15; backward tiles w(kb - 32 s + t - j) at entry
// 32 (NKMAX - 1 - s) + t - j + 31 (t < 16 rows, j < 32 columns)
constexpr int MXWT = 32 * NKMAX + 16;

// round to nearest even float -> bf16 bits (finite inputs)
DEV unsigned bf16_bits(float f)
{
    const unsigned u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// hi = bf16(v), lo = bf16(v - hi): v to about 2^-18 relative
DEV void split2(double v, unsigned& hi, unsigned& lo)
{
    const float f = (float)v;
    hi = bf16_bits(f);
    lo = bf16_bits((float)(v - (double)__uint_as_float(hi << 16)));
}

// eight floats -> packed bf16 hi and lo parts (hardware conversion, round to
// nearest even)
DEV void split8(const float* e, bf16x8& h, bf16x8& l)
{
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const __bf16 hh = (__bf16)e[v];
        h[v] = hh;
        l[v] = (__bf16)(e[v] - (float)hh);
    }
}

DEV mxf4 mfma(const bf16x8& a, const bf16x8& b, mxf4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

DEV bf16x8 ld_bf16x8(const void* p) { return *(const bf16x8*)p; }

// max / min over each 32-lane half of the wave
DEV float half_max(float v)
{
    v = fmaxf(v, __int_as_float(swz_xor<1>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(swz_xor<2>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(swz_xor<4>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(swz_xor<8>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(swz_xor<16>(__float_as_int(v))));
    return v;
}

DEV float half_min(float v) { return -half_max(-v); }

// ------------------------------------------------------------------ tables

static_assert(MX_MAXN <= 2, "MxArgs carries the window parameters of two masks");

// (from the launch arguments: one dependent read fewer than through the plan)
DEV MaskP mx_mask_params(const MxArgs& mx, const float* params, int m)
{
    return mask_params(params + mx.moff[m], mx.munb[m] != 0);
}

// support, core and tile geometry of the N masks into sh.hd (collective over
// the work-group; the support search of mask_info over both masks' windows
// at once, one offset per thread)
template <int N, class SH>
DEV void mx_heads(const MxArgs& mx, const float* params, int L, SH& sh)
{
    // (every mask's parameters are requested before any is used)
    MaskP mp[N];
#pragma unroll
    for (int mm = 0; mm < N; ++mm) mp[mm] = mx_mask_params(mx, params, mm);
    int k0[N], k1[N], n[N];
#pragma unroll
    for (int mm = 0; mm < N; ++mm) {
        mask_window(mp[mm], L, k0[mm], k1[mm]);
        n[mm] = max(k1[mm] - k0[mm] + 1, 0);
    }
#pragma unroll
    for (int mm = 0; mm < N; ++mm)
        if (threadIdx.x == mm) sh.mp[mm] = mp[mm];
    if (threadIdx.x < 2 * N) sh.ints[threadIdx.x] = (threadIdx.x & 1) ? -1 : L;
    __syncthreads();
    // the core weight at the core's midpoint, computed beside the search for
    // the usual case of a core that the support does not clip (a bounded
    // mask's core is then [ceil(a + 17/c), floor(b - 17/c)])
    // (by the last wave, which has the fewest offsets to search)
    if (threadIdx.x >= blockDim.x - 64 && threadIdx.x < blockDim.x - 64 + N) {
        const int mm = threadIdx.x - (blockDim.x - 64);
        const MaskP m = sh.mp[mm];
        int mid = INT_MIN;
        if (!m.unb && m.c > 0.f) {
            const int clo = (int)fminf(ceilf(m.a + 17.f / m.c), 2e9f);
            const int chi = (int)fmaxf(floorf(m.b - 17.f / m.c), -2e9f);
            if (clo <= chi) mid = (int)(((int64_t)clo + chi) / 2);
        }
        sh.ints[2 * N + 2 * mm] = mid;
        sh.ints[2 * N + 2 * mm + 1] = __float_as_int(mid != INT_MIN ? mask_wk(m, mid) : 0.f);
    }
    // support bounds: offset k0 + i of the masks' windows laid end to end is
    // thread i's (k grows with the lane, so a wave's bounds are its first and
    // last lane with w > 0)
    int lo[N], hi[N];
#pragma unroll
    for (int mm = 0; mm < N; ++mm) {
        lo[mm] = L;
        hi[mm] = -1;
    }
    const int lane = threadIdx.x & 63;
    for (int i0 = threadIdx.x - lane; i0 < n[0] + (N > 1 ? n[N - 1] : 0); i0 += blockDim.x) {
        const int i = i0 + lane;
        const int mm = (N > 1 && i >= n[0]) ? N - 1 : 0;
        const int k = k0[mm] + (mm ? i - n[0] : i);
        const bool pos = i < n[0] + (N > 1 ? n[N - 1] : 0) && mask_wk(mm ? mp[N - 1] : mp[0], k) > 0.f;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const unsigned long long bq = __ballot(pos && mm == q);
            if (bq) {
                const int fl = __builtin_ctzll(bq), ll = 63 - __builtin_clzll(bq);
                const int base = k0[q] - (q ? n[0] : 0) + i0;
                lo[q] = min(lo[q], base + fl);
                hi[q] = max(hi[q], base + ll);
            }
        }
    }
#pragma unroll
    for (int mm = 0; mm < N; ++mm)
        if (lane == 0) {
            atomicMin(&sh.ints[2 * mm], lo[mm]);
            atomicMax(&sh.ints[2 * mm + 1], hi[mm]);
        }
    __syncthreads();
    if (threadIdx.x < N) {
        const int mm = threadIdx.x;
        const MaskInfo mi = mask_core(sh.mp[mm], sh.ints[2 * mm], sh.ints[2 * mm + 1], sh.ints[2 * N + 2 * mm],
                                      __int_as_float(sh.ints[2 * N + 2 * mm + 1]));
        const bool core = mi.any && mi.clo <= mi.chi;
        MxHead h;
        h.any = mi.any;
        h.klo = mi.klo;
        h.khi = mi.khi;
        h.clo = core ? mi.clo : 1;
        h.chi = core ? mi.chi : 0;
        h.kf = mi.klo & ~3;
        h.kb = (mi.khi + 3) & ~3;
        h.NK = mi.any ? (16 + h.kb - h.kf + 31) / 32 : 0;
        h.ok = h.NK <= NKMAX;
        h.scale = core ? (double)mi.wc : 1.0;
        h.lscale = core ? lg2(mi.wc) : 0.f;
        sh.hd[mm] = h;
    }
    __syncthreads();
}

// weight of offset k divided by the scale (0 outside the support, exactly 1
// in the core), as packed bf16 hi (low half) and lo parts
DEV unsigned mx_wpack(const MxHead& h, const MaskP& mp, int k)
{
    double w = 0.0;
    if (k >= h.klo && k <= h.khi) w = (k >= h.clo && k <= h.chi) ? 1.0 : (double)mask_wk(mp, k) / h.scale;
    unsigned hi, lo;
    split2(w, hi, lo);
    return hi | (lo << 16);
}

// the hi and lo tiles of lane `lane` from packed per-offset weights: entry
// e0 + j - t for row t, column j (zero tiles where !live)
DEV void mx_tile(const unsigned* wt, int e0, int lane, bool live, bf16x8& h, bf16x8& l, int sgn = 1)
{
    const int t = lane & 15, j0 = 8 * (lane >> 4);
    uint4 uh, ul;
    unsigned* ph = (unsigned*)&uh;
    unsigned* pl = (unsigned*)&ul;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const unsigned u0 = live ? wt[e0 + sgn * (j0 + 2 * w - t)] : 0u;
        const unsigned u1 = live ? wt[e0 + sgn * (j0 + 2 * w + 1 - t)] : 0u;
        ph[w] = (u0 & 0xFFFFu) | (u1 << 16);
        pl[w] = (u0 >> 16) | (u1 & 0xFFFF0000u);
    }
    __builtin_memcpy(&h, &uh, 16);
    __builtin_memcpy(&l, &ul, 16);
}

// the packed weight of entry e into the four-entry groups that hold it
// (group i holds entries i .. i + 3)
DEV void mx_wq_put(uint4* wq, int e, unsigned v)
{
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (e - q >= 0) ((unsigned*)&wq[e - q])[q] = v;
}

// mx_tile from four-entry groups: two 16-byte reads per tile instead of
// eight 4-byte reads (entries ascend with the column for sgn = 1, descend
// for sgn = -1)
DEV void mx_tile4(const uint4* wq, int e0, int lane, bool live, bf16x8& h, bf16x8& l, int sgn = 1)
{
    const int t = lane & 15, j0 = 8 * (lane >> 4);
    unsigned u[8];
    if (sgn > 0) {
        const uint4 q0 = wq[e0 + j0 - t], q1 = wq[e0 + j0 - t + 4];
        u[0] = q0.x; u[1] = q0.y; u[2] = q0.z; u[3] = q0.w;
        u[4] = q1.x; u[5] = q1.y; u[6] = q1.z; u[7] = q1.w;
    } else {
        const int e1 = e0 + t - j0;
        const uint4 q0 = wq[e1 - 3], q1 = wq[e1 - 7];
        u[0] = q0.w; u[1] = q0.z; u[2] = q0.y; u[3] = q0.x;
        u[4] = q1.w; u[5] = q1.z; u[6] = q1.y; u[7] = q1.x;
    }
    uint4 uh, ul;
    unsigned* ph = (unsigned*)&uh;
    unsigned* pl = (unsigned*)&ul;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const unsigned u0 = live ? u[2 * w] : 0u, u1 = live ? u[2 * w + 1] : 0u;
        ph[w] = (u0 & 0xFFFFu) | (u1 << 16);
        pl[w] = (u0 >> 16) | (u1 & 0xFFFF0000u);
    }
    __builtin_memcpy(&h, &uh, 16);
    __builtin_memcpy(&l, &ul, 16);
}

// ------------------------------------------------------------------ kernels

struct MxShared {
    MxHead hd[MX_MAXN];          // per mask
    MaskP mp[MX_MAXN];           // per mask: window parameters
    int ints[4 * MX_MAXN];       // support search: bounds, then a precomputed core weight
    uint4 wq[MX_MAXN][MXWT];     // packed per-offset weights (forward or backward tile offsets), in
                                 //   groups of four consecutive entries
    unsigned dt[MX_MAXN][2][MXWT];      // backward: d/da, d/db weights of the same offsets
    int fd[MX_MAXN][NKMAX];      // backward: K-step s has d/da (bit 0) / d/db (bit 1) weights
    float R[MX_MAXN][MXG];       // forward: reference of the terms; backward: Q
    float C[MX_MAXN][MXG];       // backward: constant of the adjoint terms' exponent
    int frag[MXG];               // trajectory handed to the generic executor
    int omin[MX_MAXN][MXG];      // forward: floor(min O), ceil(max O) over the trajectory
    int omax[MX_MAXN][MXG];
    int dstep[MX_MAXN][NDMAX];   // backward: K-step and kind (0: d/da, 1: d/db) of each derivative tile
    int dwhich[MX_MAXN][NDMAX];
    int nd[MX_MAXN];
    int over;                    // backward: more derivative tiles than NDMAX
    float pp[MX_MAXN][2][2][MXG];       // backward: d/da, d/db partials per matrix wave
};

// trajectory b goes to the generic executor (which finds it by its flag);
// its saved traces are not valid
DEV void mx_handoff(const KArgs& ka, const MxArgs& mx, int64_t b)
{
    mx.handed[b] = 1;
    if (ka.saved_flag) ka.saved_flag[b] = 0;
}

// byte offset in a ring row of the 8-position group starting at position p (p % 8 == 0)
DEV int ring_off(int p) { return (p % MXRING) / 8 * 32; }

// byte offset in a ring row of position pr + d, for pr < MXRING and
// 0 <= d < MXRING, both multiples of 8 (a position's two bf16 halves are 4
// bytes, so 8-position groups of 32 bytes put position p at byte 4 p)
DEV int ring_byte(int pr, int d)
{
    const int b = 4 * (pr + d);
    return b >= 4 * MXRING ? b - 4 * MXRING : b;
}

// per-mask constants of the linear predicate and the exponent scale, in
// registers (reading them from the plan inside a loop would put a load and a
// wait in every iteration)
template <int DD>
struct MxMask {
    float sg, beta, sbl;         // sign (-1 for Always), beta, sg beta log2(e)
    float c, w[DD];              // predicate w . x - c
};

template <int DD>
DEV MxMask<DD> mx_mask(const DevPlan* Pk, const float* params, int m)
{
    MxMask<DD> r;
    const Instr& I = Pk->ins[Pk->fused.ins[m]];
    r.sg = (I.flags & F_MIN) ? -1.f : 1.f;
    r.beta = params[I.beta];
    r.sbl = r.sg * r.beta * LOG2E;
    const float* cf = &Pk->coef[Pk->ins[Pk->fused.pred[m]].coef];
    r.c = cf[0];
#pragma unroll
    for (int d = 0; d < DD; ++d) r.w[d] = cf[1 + d];
    return r;
}

template <int DD>
DEV float mx_zx(const MxMask<DD>& M, const float* xv)
{
    float u = -M.c;
#pragma unroll
    for (int d = 0; d < DD; ++d) u = fmaf(M.w[d], xv[d], u);
    return M.sbl * u;
}

// the root: the smooth And/Or over the mask traces (the same formula as the
// fused kernels' fused_root), with its constants in registers
struct MxRoot {
    bool nary;
    float sg, bl, ibl;
};

DEV MxRoot mx_root_consts(const DevPlan& P, const float* params)
{
    MxRoot r;
    r.nary = P.fused.root_nary != 0 || P.fused.n > 1;
    r.sg = P.fused.nary_min ? -1.f : 1.f;
    r.bl = r.nary ? params[P.fused.nary_beta] * LOG2E : 1.f;
    r.ibl = 1.f / r.bl;
    return r;
}

// four consecutive floats at p[i0 ..] (fewer when n_valid < 4), vectorised when aligned
DEV void store4(float* p, int64_t i0, int n_valid, const float* v)
{
    if (n_valid >= 4 && (((uintptr_t)(p + i0)) & 15) == 0) {
        *(float4*)(p + i0) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        for (int r = 0; r < 4 && r < n_valid; ++r) p[i0 + r] = v[r];
    }
}

// a where c, else b, as bit operations on a mask the compiler cannot see
// through (a select of an expensive value may otherwise become a branch
// around its computation)
DEV float mx_sel(bool c, float a, float b)
{
    int m = -(int)c;
    asm volatile("" : "+v"(m));
    return __int_as_float((__float_as_int(a) & m) | (__float_as_int(b) & ~m));
}

// four consecutive outputs at p (n_valid >= 1 of them in the trajectory).
// VEC: T is a multiple of 4 and the rows are 16-byte aligned, so all four
// are valid and one 16-byte store writes them.
template <bool VEC>
DEV void mx_store4(float* p, int n_valid, const float* v)
{
    if (VEC) *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
    else store4(p, 0, n_valid, v);
}

// keep a value in registers across a loop (the compiler may otherwise reload
// loop-invariant tiles from memory inside it, each load followed by a wait)
DEV void mx_pin(bf16x8& v) { asm volatile("" : "+v"(v)); }


// 8 positions j .. j+7 (DD floats each) of row xb, from clamped addresses
// and with no mask: values at positions outside [0, L) are those of a valid
// position, and every user masks them itself (a mask applied here makes the
// compiler wait for the load where the masked value is formed).  VEC: T a
// multiple of 4, 16-byte aligned rows and j a multiple of 4, so that each
// group of 4 positions lies wholly inside or outside [0, L) and is read with
// 16-byte loads from its clamped start.
template <int DD, bool VEC>
DEV void mx_load8(const float* xb, int j, int L, float* v)
{
    if (VEC) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const float4* p = (const float4*)(xb + (int64_t)min(max(j + 4 * g, 0), L - 4) * DD);
#pragma unroll
            for (int d = 0; d < DD; ++d) {
                const float4 u = p[d];
                float* o = v + 4 * g * DD + 4 * d;
                o[0] = u.x;
                o[1] = u.y;
                o[2] = u.z;
                o[3] = u.w;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int jc = min(max(j + q, 0), L - 1);
#pragma unroll
            for (int d = 0; d < DD; ++d) v[q * DD + d] = xb[(int64_t)jc * DD + d];
        }
    }
}

// 4 positions j .. j+3 (j >= 0; a multiple of 4 when VEC), unmasked as mx_load8
template <int DD, bool VEC>
DEV void mx_load4(const float* xb, int j, int L, float* v)
{
    if (VEC) {
        const float4* p = (const float4*)(xb + (int64_t)min(j, L - 4) * DD);
#pragma unroll
        for (int d = 0; d < DD; ++d) {
            const float4 u = p[d];
            v[4 * d] = u.x;
            v[4 * d + 1] = u.y;
            v[4 * d + 2] = u.z;
            v[4 * d + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jc = min(j + r, L - 1);
#pragma unroll
            for (int d = 0; d < DD; ++d) v[r * DD + d] = xb[(int64_t)jc * DD + d];
        }
    }
}

// bytes of LDS of the matrix-core kernels beyond the rings: two buffers
// (alternating rounds) of the matrix waves' results, 8 tiles per mask
constexpr size_t mx_xch_bytes(int n, int D, bool bwd)
{
    return (void)D, (void)bwd, (size_t)2 * n * 8 * 64 * 16;
}

// the root (the smooth And/Or of the mask traces) and log2 of the softmax
// weight of every child, from su_k = sg * trace_k (sg = -1 for a smooth
// And).  With two children the larger weight's term is exactly 1, so the
// sum takes one exponential.
template <int N>
DEV float mx_root_lws(const MxRoot& R, const float* su, float* lw)
{
    static_assert(N == 1 || N == 2, "one or two masks under the root");
    if (N == 1) {
        // (an n-ary root of one child: its weight is 1 and the root is the trace)
        lw[0] = 0.f;
        return R.sg * su[0];
    }
    const float m = fmaxf(su[0], su[N - 1]);
    const float ls = lg2(1.f + ex2(-fabsf(su[0] - su[N - 1]) * R.bl));
#pragma unroll
    for (int k = 0; k < N; ++k) lw[k] = (su[k] - m) * R.bl - ls;
    return R.sg * (m + ls * R.ibl);
}

// Forward: traces of the masks, the root, and for the backward l = log2 p_m
// - lg2(S) per mask and output (saved), plus each trajectory's range of O
// and its reference R.
//
// The work-group's 6N waves take two roles, one round apart.  Matrix waves
// (2 per mask: w < 2N) compute the window sums of round k for their mask:
// four tiles at outputs 128 k + 16 h + 32 j (h = w % 2, j < 4), which read
// the same staged terms at K-steps s - j, so each read of the ring feeds up
// to 12 products; the hi and lo weight tiles stay in registers.  The sums go
// to an LDS buffer (two, alternating by round).  Staging waves (4N, one
// staging unit per thread) turn round k - 1's sums into traces, the root and
// l, store them, and stage block k + 4 of every mask.  With N = 2 each SIMD
// runs one matrix wave and two staging waves, whose transcendental chains
// hide each other's latency.  One barrier per round.
template <int N, int DD, bool VEC>
__global__ void __launch_bounds__(384 * N, 1) stl_mx_fwd(DevPlan plan, Batch bt, KArgs ka, MxArgs mx)
{
    extern __shared__ __align__(16) unsigned char mxs[];
    __shared__ MxShared sh;
    const DevPlan& P = plan;
    // the plan is read from the kernel-argument segment where the mask index
    // is a run-time value (indexing the by-value argument would copy it to
    // private memory)
    const DevPlan* Pk = (const DevPlan*)__builtin_amdgcn_kernarg_segment_ptr();
    const MxRoot RC = mx_root_consts(P, ka.params);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int L = (int)bt.T;
    const int64_t g0 = (int64_t)blockIdx.x * MXG;
    const bool matrix = wv < 2 * N;
    const int vt = tid - 128 * N;                // staging thread index
    // ---- the reference sample (positions i * ceil(L / 32), i < 32, one per
    // staging thread and row it serves) is read first: it needs no mask data
    const int hs = vt >> 5, l32 = lane & 31;
    float xs[2 / N][DD];
    if (!matrix) {
        const int j = min(L - 1, l32 * ((L + 31) / 32));
#pragma unroll
        for (int i = 0; i < 2 / N; ++i) {
            const int64_t b = g0 + hs + 8 * N * i;
#pragma unroll
            for (int d = 0; d < DD; ++d) xs[i][d] = bt.x[((b < bt.B ? b : 0) * L + j) * DD + d];
        }
    }
    // ---- per mask: support, core, tile geometry, and the weights of the
    // forward tiles' offsets kf - 15 .. kf + 32 NKMAX (packed bf16 hi, lo)
    mx_heads<N>(mx, ka.params, L, sh);
    // (for the backward of the same parameters)
    if (blockIdx.x == 0 && tid < N && mx.heads) mx.heads[tid] = sh.hd[tid];
    bool ok = true;
#pragma unroll
    for (int mm = 0; mm < N; ++mm) ok = ok && sh.hd[mm].ok;
    if (!ok) {
        // the masks do not fit the matrix-core path: the generic executor takes every trajectory
        if (tid < MXG && g0 + tid < bt.B) mx_handoff(ka, mx, g0 + tid);
        return;
    }
    // ---- staging units: unit u = (mask u / 256, row (u / 16) % 16, 8-position
    // group u % 16) of a block; position p of mask m holds the term of x at
    // kf_m + p.  Staging thread v owns unit v in every block; the mask is
    // uniform over a wave.
    struct Unit {
        MxMask<DD> M;
        const float* xb;
        unsigned char* row;
        float R;        // the row's reference (set once the references are known)
        int off;        // kf + 8 g: x index of the unit's first position in block 0
        int g8;         // 8 g
        int kf;
        bool act, any;
    };
    auto unit = [&](int u) {
        Unit U;
        const int um = __builtin_amdgcn_readfirstlane(u >> 8), ur = (u >> 4) & 15, ug = u & 15;
        const MxHead& TU = sh.hd[um];
        const int64_t b = g0 + ur;
        U.M = mx_mask<DD>(Pk, ka.params, um);
        U.xb = bt.x + (b < bt.B ? b : 0) * (int64_t)L * DD;
        U.row = mxs + (um * MXG + ur) * MXRS;
        U.R = 0.f;
        U.off = TU.kf + 8 * ug;
        U.g8 = 8 * ug;
        U.kf = TU.kf;
        U.any = TU.any;
        U.act = b < bt.B && TU.any;
        return U;
    };
    auto stage_load = [&](const Unit& U, int blk, float* xv) {
        mx_load8<DD, VEC>(U.xb, MXBLK * blk + U.off, L, xv);
    };
    // block blk of the unit's mask lies wholly inside the trajectory (a
    // uniform condition: no position needs a select; rows past the batch
    // stage terms of a valid row, which only their own unused outputs read)
    auto unit_full = [&](const Unit& U, int blk) { return U.any && MXBLK * blk + U.kf + MXBLK <= L; };
    auto stage_write = [&](auto full, const Unit& U, int blk, const float* xv, bool& frag) {
        constexpr bool FULL = decltype(full)::value;
        const int p0 = MXBLK * blk + U.g8, j0 = MXBLK * blk + U.off;
        float e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float d = mx_zx<DD>(U.M, xv + q * DD) - U.R;
            const float t = ex2(fminf(fmaxf(d, -MX_HALF), MX_HALF));
            if (FULL) {
                frag |= !(fabsf(d) <= MX_HALF);
                e[q] = t;
            } else {
                // (selects, not branches: x reads as 0 outside the trajectory)
                const bool in = U.act && j0 + q < L;
                frag |= in & !(fabsf(d) <= MX_HALF);
                e[q] = mx_sel(in, t, 0.f);
            }
        }
        bf16x8 h, l;
        split8(e, h, l);
        unsigned char* q = U.row + ring_off(p0);
        *(bf16x8*)q = h;
        *(bf16x8*)(q + 16) = l;
    };
    // x of blocks 0 .. 3 is requested as soon as the windows are known
    Unit U = unit(matrix ? 0 : vt);
    float xv[4][8 * DD];
    if (!matrix) {
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) stage_load(U, blk, xv[blk]);
    }
    for (int i = tid; i < N * MXWT; i += blockDim.x) {
        const int mm = i / MXWT, e = i % MXWT;
        mx_wq_put(sh.wq[mm], e, mx_wpack(sh.hd[mm], sh.mp[mm], sh.hd[mm].kf - 15 + e));
    }
    // (ordered before every use by the barrier that follows the references)
    if (tid < MXG) {
        sh.frag[tid] = 0;
#pragma unroll
        for (int mm = 0; mm < N; ++mm) {
            sh.omin[mm][tid] = INT_MAX;
            sh.omax[mm][tid] = INT_MIN;
        }
    }
    float* accb = (float*)(mxs + N * MXG * MXRS);                   // [2][N][2][4][64][4] window sums
    const int nround = (L + MXROUND - 1) / MXROUND;
    // bodies of the loop below (both roles run the same number, one barrier
    // each): round k's sums in body k, its outputs in body k + 1; an even
    // count lets the staging waves unroll by two with no conditional body
    const int nbody = (nround + 2) & ~1;
    __syncthreads();            // heads and per-offset weights known
    if (matrix) {
        // ---------------------------------------------------------- matrix waves
        // (the weight tiles are built while the staging waves compute the
        // references and stage blocks 0 .. 3).  The K-loop is compiled for
        // KS = NKMAX and KS = NKMAX - 1 steps and chosen by the window
        // (uniform): a window of fewer steps skips the last step's products.
        const int m = wv >> 1, hh = wv & 1;
        const int NKm = __builtin_amdgcn_readfirstlane(sh.hd[m].NK);
        auto run = [&](auto ks) {
            constexpr int KS = decltype(ks)::value;
            bf16x8 Wh[KS], Wl[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) mx_tile4(sh.wq[m], 32 * s + 15, lane, s < NKm, Wh[s], Wl[s]);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                mx_pin(Wh[s]);
                mx_pin(Wl[s]);
            }
            __syncthreads();        // references known
            __syncthreads();        // blocks 0 .. 3 staged
            const int bc = lane & 15, rq = lane >> 4;
            const unsigned char* ebase = mxs + (m * MXG + bc) * MXRS;
            for (int k = 0; k < nbody; ++k) {
                if (k < nround) {
                    const int t0 = MXROUND * k + 16 * hh;
                    const int pr = (t0 + 8 * rq) % MXRING;
                    mxf4 acc[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[j] = mxf4{0.f, 0.f, 0.f, 0.f};
                    // each K-step's terms are read one step ahead of their products
                    bf16x8 eh = ld_bf16x8(ebase + ring_byte(pr, 0)), el = ld_bf16x8(ebase + ring_byte(pr, 0) + 16);
#pragma unroll
                    for (int s = 0; s < KS + 3; ++s) {
                        bf16x8 ehn = eh, eln = el;
                        if (s + 1 < KS + 3) {
                            const unsigned char* ep = ebase + ring_byte(pr, 32 * (s + 1));
                            ehn = ld_bf16x8(ep);
                            eln = ld_bf16x8(ep + 16);
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int st = s - j;
                            if (st >= 0 && st < KS) {
                                acc[j] = mfma(Wh[st], eh, acc[j]);
                                acc[j] = mfma(Wh[st], el, acc[j]);
                                acc[j] = mfma(Wl[st], eh, acc[j]);
                            }
                        }
                        eh = ehn;
                        el = eln;
                    }
                    float4* ob = (float4*)accb + ((((k & 1) * N + m) * 2 + hh) * 4) * 64 + lane;
#pragma unroll
                    for (int j = 0; j < 4; ++j) ob[j * 64] = make_float4(acc[j][0], acc[j][1], acc[j][2], acc[j][3]);
                }
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    mx_pin(Wh[s]);
                    mx_pin(Wl[s]);
                }
                __syncthreads();
            }
        };
        if (NKm < NKMAX) run(std::integral_constant<int, NKMAX - 1>{});
        else run(std::integral_constant<int, NKMAX>{});
    } else {
        // ---------------------------------------------------------- staging waves
        const int vw = wv - 2 * N;
        bool sfrag = false;
        // ---- references: midpoint of the exponents over the sample of each
        // trajectory, reduced over each half-wave; the loads of blocks 0 .. 3
        // are in flight meanwhile
        {
#pragma unroll
            for (int i = 0; i < 2 / N; ++i) {
                const int r = hs + 8 * N * i;
                const bool bin = g0 + r < bt.B;
#pragma unroll
                for (int mm = 0; mm < N; ++mm) {
                    const MxMask<DD> M = mx_mask<DD>(Pk, ka.params, mm);
                    const float z = bin ? mx_zx<DD>(M, xs[i]) : -INFINITY;
                    const float zmax = half_max(z), zmin = half_min(bin ? z : INFINITY);
                    if (l32 == 0) sh.R[mm][r] = zmax >= zmin ? floorf(0.5f * (zmax + zmin)) : 0.f;
                }
            }
            __syncthreads();    // references known
            U.R = sh.R[vt >> 8][(vt >> 4) & 15];
#pragma unroll
            for (int blk = 0; blk < 4; ++blk) stage_write(std::false_type{}, U, blk, xv[blk], sfrag);
        }
        const int bc = lane & 15, rq = lane >> 4;
        const int64_t bo = g0 + bc;
        const bool bvalid = bo < bt.B;
        // per mask: sg_root * trace = c2 * lg2(window sum) + c1 where the
        // window is not empty (O = Rb + lg2(window sum)), else spad
        float Rb[N], c1[N], c2[N], spad[N];
        int klo[N];
        bool any[N], allany = true;
        int klomax = 0;
#pragma unroll
        for (int mm = 0; mm < N; ++mm) {
            const MxHead& T = sh.hd[mm];
            const MxMask<DD> M = mx_mask<DD>(Pk, ka.params, mm);
            Rb[mm] = sh.R[mm][bc] + T.lscale;
            c2[mm] = RC.sg * M.sg / (M.beta * LOG2E);
            c1[mm] = c2[mm] * Rb[mm];
            spad[mm] = -RC.sg * M.sg * P.rho_pad;               // empty window
            klo[mm] = T.klo;
            any[mm] = T.any;
            allany = allany && T.any;
            klomax = max(klomax, T.klo);
        }
        // range of lg2(window sum) over the outputs (O is monotone in it)
        float lmin[N], lmax[N];
#pragma unroll
        for (int mm = 0; mm < N; ++mm) {
            lmin[mm] = INFINITY;
            lmax[mm] = -INFINITY;
        }
        float* const root = ka.root;
        float* const saved = ka.saved;
        // outputs of round kr, tile tau: the traces, the root and l.  FULL:
        // every output of the round has a window inside the trajectory for
        // every mask (a uniform condition), so no output needs a select.
        auto outputs = [&](auto full, const int kr, const int tau) {
            constexpr bool FULL = decltype(full)::value;
            const float4* ib = (const float4*)accb + (kr & 1) * N * 8 * 64 + lane;
            const int hh = tau >> 2, j = tau & 3;
            const int t0 = MXROUND * kr + 16 * hh + 32 * j + 4 * rq;
            float su[N][4], la[N][4];
#pragma unroll
            for (int mm = 0; mm < N; ++mm) {
                const float4 a4 = ib[((mm * 2 + hh) * 4 + j) * 64];
                const float a[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const float lo = lg2(a[rr]);
                    const float u = fmaf(lo, c2[mm], c1[mm]);
                    if (FULL) {
                        su[mm][rr] = u;
                        la[mm][rr] = lo;
                        lmin[mm] = fminf(lmin[mm], lo);
                        lmax[mm] = fmaxf(lmax[mm], lo);
                    } else {
                        // (selects, not branches)
                        const bool in = any[mm] && t0 + rr + klo[mm] <= L - 1;
                        su[mm][rr] = mx_sel(in, u, spad[mm]);
                        la[mm][rr] = mx_sel(in, lo, 0.f);
                        lmin[mm] = fminf(lmin[mm], mx_sel(in, lo, INFINITY));
                        lmax[mm] = fmaxf(lmax[mm], mx_sel(in, lo, -INFINITY));
                    }
                }
            }
            const int nv = L - t0;
            if (bvalid && (FULL || nv > 0)) {
                float rt[4], ll[N][4];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    float v[N], lw[N];
#pragma unroll
                    for (int mm = 0; mm < N; ++mm) v[mm] = su[mm][rr];
                    rt[rr] = mx_root_lws<N>(RC, v, lw);
#pragma unroll
                    for (int mm = 0; mm < N; ++mm) ll[mm][rr] = lw[mm] - la[mm][rr];
                }
                if (root) mx_store4<VEC && FULL>(root + bo * (int64_t)L + t0, nv, rt);
                if (saved) {
#pragma unroll
                    for (int mm = 0; mm < N; ++mm)
                        mx_store4<VEC && FULL>(saved + ((int64_t)mm * bt.B + bo) * L + t0, nv, ll[mm]);
                }
            }
        };
        // x of block k + 4 is loaded two rounds before it is staged (memory
        // latency under load exceeds one round); the loop is unrolled by two
        // so that the two prefetch buffers keep static register names
        float xq0[8 * DD], xq1[8 * DD];
        stage_load(U, 4, xq0);
        __syncthreads();        // blocks 0 .. 3 staged
        auto body = [&](const int k, const float* xn, float* xnext) {
            // (unconditional: the addresses are clamped, and a conditional load
            // would be waited for where the branches join)
            stage_load(U, k + 5, xnext);
            if (k >= 1 && k <= nround) {
                // outputs of round k - 1: this wave's tiles tau = vw * 2 / N + i
                const int kr = k - 1;
                const bool full = allany && MXROUND * kr + MXROUND + klomax <= L;
#pragma unroll
                for (int i = 0; i < 2 / N; ++i) {
                    if (full) outputs(std::true_type{}, kr, vw * (2 / N) + i);
                    else outputs(std::false_type{}, kr, vw * (2 / N) + i);
                }
            }
            if (k < nround) {
                if (unit_full(U, k + 4)) stage_write(std::true_type{}, U, k + 4, xn, sfrag);
                else stage_write(std::false_type{}, U, k + 4, xn, sfrag);
            }
            __syncthreads();
        };
        for (int k = 0; k < nbody; k += 2) {
            body(k, xq0, xq1);
            body(k + 1, xq1, xq0);
        }
#pragma unroll
        for (int mm = 0; mm < N; ++mm)
            if (any[mm] && bvalid && lmin[mm] <= lmax[mm]) {
                atomicMin(&sh.omin[mm][bc], (int)floorf(Rb[mm] + lmin[mm]));
                atomicMax(&sh.omax[mm][bc], (int)ceilf(Rb[mm] + lmax[mm]));
            }
        if (sfrag) atomicOr(&sh.frag[(vt >> 4) & 15], 1);
    }
    // ---- exponent ranges of the traces and the references (for the
    // backward), hand-offs
    __syncthreads();
    if (mx.ranges && tid < N * MXG) {
        const int mm = tid / MXG, r = tid % MXG;
        if (g0 + r < bt.B) {
            int* rp = mx.ranges + ((g0 + r) * N + mm) * 3;
            rp[0] = sh.omin[mm][r];
            rp[1] = sh.omax[mm][r];
            rp[2] = (int)sh.R[mm][r];
        }
    }
    // this group's rows: hand-off flag (no other work-group touches them), and
    // for a saving forward the saved traces' flag (2: written by this path,
    // with their exponent ranges)
    if (tid < MXG && g0 + tid < bt.B) {
        if (sh.frag[tid]) {
            mx_handoff(ka, mx, g0 + tid);
        } else {
            mx.handed[g0 + tid] = 0;
            if (ka.saved_flag) ka.saved_flag[g0 + tid] = 2;
        }
    }
}

// Backward, with the forward's two roles: matrix waves (2 per mask) compute
// round k's transposed window sums D_j = sum_t w_{j-t} H_t over four 32-aligned
// output tiles (sharing each ring read) and the band derivative sums, take
// 2^{z_j + Q} at their outputs, add d/da, d/db into their partials and pass
// the d/dx factors to LDS; staging waves add the masks' d/dx of round k - 1,
// store it, and stage block k + 4 of every mask's H.
template <int N, int DD, bool VEC>
__global__ void __launch_bounds__(256 * N, 1) stl_mx_bwd(DevPlan plan, Batch bt, KArgs ka, MxArgs mx)
{
    extern __shared__ __align__(16) unsigned char mxs[];
    __shared__ MxShared sh;
    const DevPlan& P = plan;
    const DevPlan* Pk = (const DevPlan*)__builtin_amdgcn_kernarg_segment_ptr();
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int L = (int)bt.T;
    const int64_t g0 = (int64_t)blockIdx.x * MXG;
    // this group's hand-off flags (no other work-group touches them) are
    // cleared by the thread that then decides the row's hand-off (stores are
    // left to the end: a wait for a load would also wait for them)
    auto finish_row = [&](int r, bool hand) {
        if (g0 + r >= bt.B) return;
        mx.handed[g0 + r] = 0;
        if (hand) mx_handoff(ka, mx, g0 + r);
    };
    // ---- per mask: support, core, tile geometry; the weights of the
    // backward tiles' offsets kb - 32 NKMAX - 31 .. kb + 15 and their d/da,
    // d/db (bands only: the core contributes nothing to d/da, d/db to fp32
    // rounding)
    // (the forward's heads: the same parameters give the same values)
    if (mx.heads) {
        if (tid < N) {
            sh.hd[tid] = mx.heads[tid];
            sh.mp[tid] = mx_mask_params(mx, ka.params, tid);
        }
        __syncthreads();
    } else {
        mx_heads<N>(mx, ka.params, L, sh);
    }
    bool ok = true;
#pragma unroll
    for (int mm = 0; mm < N; ++mm) ok = ok && sh.hd[mm].ok;
    if (!ok) {
        if (tid < MXG) finish_row(tid, true);
        return;
    }
    // G and l of blocks 0 .. 3 are requested as soon as the windows are
    // known (rows of trajectories handed off are read too: their terms are
    // masked where they are staged)
    float gv0[4][8], lv0[4][8];
    {
        const int um = tid >> 8, ur = (tid >> 4) & 15, ug = tid & 15;
        const int64_t b = g0 + ur < bt.B ? g0 + ur : 0;
        const float* Gp = ka.G + b * (int64_t)L;
        const float* lp = ka.saved_in + ((int64_t)um * bt.B + b) * L;
        const int t0u = 8 * ug - sh.hd[um].kb;
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            mx_load8<1, VEC>(Gp, MXBLK * blk + t0u, L, gv0[blk]);
            mx_load8<1, VEC>(lp, MXBLK * blk + t0u, L, lv0[blk]);
        }
    }
    if (tid == 0) sh.over = 0;
    if (tid < MXG) sh.frag[tid] = 0;
    if (tid < N * NKMAX) sh.fd[tid / NKMAX][tid % NKMAX] = 0;
    __syncthreads();
    for (int i = tid; i < N * MXWT; i += blockDim.x) {
        const int mm = i / MXWT, e = i % MXWT;
        const MxHead& h = sh.hd[mm];
        const MaskP mp = sh.mp[mm];
        const int k = h.kb - 32 * (NKMAX - 1) - 31 + e;
        mx_wq_put(sh.wq[mm], e, mx_wpack(h, mp, k));
        float da = 0.f, db = 0.f;
        if (k >= h.klo && k <= h.khi && !(k >= h.clo && k <= h.chi)) mask_wk(mp, k, &da, &db);
        unsigned hi, lo;
        split2((double)da, hi, lo);
        sh.dt[mm][0][e] = hi | (lo << 16);
        split2((double)db, hi, lo);
        sh.dt[mm][1][e] = hi | (lo << 16);
        // K-step s reads entries 32 (NKMAX - 1 - s) .. + 46: it has d/da
        // (d/db) weights where one of them does
        const int nz = (da != 0.f ? 1 : 0) | (db != 0.f ? 2 : 0);
        if (nz) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int st = NKMAX - 1 - e / 32 + q;     // the steps whose entries include e
                if (st >= 0 && st < NKMAX && e - 32 * (NKMAX - 1 - st) <= 46) atomicOr(&sh.fd[mm][st], nz);
            }
        }
    }
    __syncthreads();
    // ---- per mask: the list of derivative tiles (K-step, kind) in order of
    // (kind, s): the d/da tiles first; lane (m, kind, s) of the first wave
    // finds its place by a count of the set flags before it
    if (tid < 64) {
        const int mm = tid / (2 * NKMAX), w = (tid / NKMAX) & 1, s = tid % NKMAX;
        const bool f = mm < N && s < min(sh.hd[mm < N ? mm : 0].NK, NKMAX) && ((sh.fd[mm < N ? mm : 0][s] >> w) & 1);
        const unsigned long long bal = __ballot(f);
        const unsigned long long below = bal & ((1ull << tid) - 1ull) & ~((1ull << (mm * 2 * NKMAX)) - 1ull);
        const int idx = __popcll(below);
        if (f && idx < NDMAX) {
            sh.dstep[mm][idx] = s;
            sh.dwhich[mm][idx] = w;
        }
        if (mm < N && s == 0 && w == 0) {
            const unsigned long long mine = (bal >> (mm * 2 * NKMAX)) & ((1ull << (2 * NKMAX)) - 1ull);
            const int total = __popcll(mine);
            sh.nd[mm] = min(total, NDMAX);
            if (total > NDMAX) sh.over = 1;
        }
    }
    // ---- per trajectory: saved data valid; the reference Q (from the
    // forward's range of O) and the constant C = -(R + lscale) - Q of the
    // adjoint terms' exponent l + C
    if (tid < N * MXG) {
        const int mm = tid / MXG, r = tid % MXG;
        const int64_t b = g0 + r;
        float Q = 0.f, C = 0.f;
        if (b < bt.B) {
            bool frag = ka.saved_flag[b] != 2;
            if (!frag) {
                const int* rp = mx.ranges + (b * N + mm) * 3;
                const int lo = rp[0], hi = rp[1];
                if (lo <= hi) {
                    if ((float)hi - (float)lo > 2.f * MX_HALF) frag = true;
                    else Q = -floorf(0.5f * ((float)lo + (float)hi));
                }
                C = ((float)(-rp[2]) - Q) - sh.hd[mm].lscale;
            }
            if (frag) atomicOr(&sh.frag[r], 1);
        }
        sh.R[mm][r] = Q;
        sh.C[mm][r] = C;
    }
    __syncthreads();
    const bool over = sh.over != 0;
    // ---- staging units (as in the forward): unit u = (mask u / 256, row
    // (u / 16) % 16, 8-position group u % 16).  Position p of mask m is time
    // t = p - kb_m; H_m(t) = G(t) 2^{l_m(t) + C} (0 outside the trajectory and
    // where the window of t is empty)
    struct Unit {
        const float* G;
        const float* l;
        unsigned char* row;
        float C;
        int t0;         // time of the unit's first position in block 0
        int g8;
        int klo;
        bool act;
    };
    auto unit = [&](int u) {
        Unit U;
        const int um = u >> 8, ur = (u >> 4) & 15, ug = u & 15;
        const MxHead& TU = sh.hd[um];
        const int64_t b = g0 + ur;
        const bool row = b < bt.B && !sh.frag[ur] && !over;
        U.G = ka.G + (row ? b : 0) * (int64_t)L;
        U.l = ka.saved_in + ((int64_t)um * bt.B + (row ? b : 0)) * L;
        U.row = mxs + (um * MXG + ur) * MXRS;
        U.C = sh.C[um][ur];
        U.t0 = 8 * ug - TU.kb;
        U.g8 = 8 * ug;
        U.klo = TU.klo;
        U.act = row && TU.any;
        return U;
    };
    auto stage_load = [&](const Unit& U, int blk, float* gv, float* lv) {
        mx_load8<1, VEC>(U.G, MXBLK * blk + U.t0, L, gv);
        mx_load8<1, VEC>(U.l, MXBLK * blk + U.t0, L, lv);
    };
    auto stage_write = [&](const Unit& U, int blk, const float* gv, const float* lv) {
        const int t0 = MXBLK * blk + U.t0;
        float h[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int t = t0 + q;
            // l + C <= -O - Q lies within [-MX_HALF, MX_HALF] (the forward's range check)
            const float hv = gv[q] * ex2(fminf(fmaxf(lv[q] + U.C, -2.f * MX_HALF), 2.f * MX_HALF));
            h[q] = mx_sel(U.act && t >= 0 && t + U.klo <= L - 1, hv, 0.f);
        }
        bf16x8 hh, hl;
        split8(h, hh, hl);
        unsigned char* q = U.row + ring_off(MXBLK * blk + U.g8);
        *(bf16x8*)q = hh;
        *(bf16x8*)(q + 16) = hl;
    };
    {
        const Unit U = unit(tid);
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) stage_write(U, blk, gv0[blk], lv0[blk]);
    }
    // derivative tiles of every mask in LDS ([n][NDMAX][hi, lo][lane], zero
    // tiles in unused slots)
    float* gbuf = (float*)(mxs + N * MXG * MXRS);       // [2][N][2][4][64][4] d/dx factors
    uint4* dlds = (uint4*)(mxs + N * MXG * MXRS + mx_xch_bytes(N, DD, true));
    for (int e = tid; e < N * NDMAX * 64; e += blockDim.x) {
        const int mm = e / (NDMAX * 64), d = (e / 64) % NDMAX, l = e & 63;
        bf16x8 th, tl;
        const bool use = d < sh.nd[mm];
        const int st = use ? sh.dstep[mm][d] : 0;
        mx_tile(sh.dt[mm][use ? sh.dwhich[mm][d] : 0], 32 * (NKMAX - 1 - st) + 31, l, use, th, tl, -1);
        __builtin_memcpy(&dlds[(mm * NDMAX + d) * 128 + l], &th, 16);
        __builtin_memcpy(&dlds[(mm * NDMAX + d) * 128 + 64 + l], &tl, 16);
    }
    const int nround = (L + MXROUND - 1) / MXROUND;
    const int nbody = (nround + 2) & ~1;        // as in the forward: even, both roles alike
    const bool matrix = wv < 2 * N;
    const int bc = lane & 15, rq = lane >> 4;
    const int64_t bo = g0 + bc;
    const bool bvalid = bo < bt.B && !sh.frag[bc] && !over;
    __syncthreads();
    if (matrix) {
        // ---------------------------------------------------------- matrix waves
        const int m = wv >> 1, hh = wv & 1;
        const MxMask<DD> M = mx_mask<DD>(Pk, ka.params, m);
        const bool any = sh.hd[m].any;
        const int NKm = __builtin_amdgcn_readfirstlane(sh.hd[m].NK);
        const int nd = sh.nd[m];
        int dst[NDMAX];
        bool isb[NDMAX];
#pragma unroll
        for (int d = 0; d < NDMAX; ++d) {
            const bool use = d < nd;
            dst[d] = use ? sh.dstep[m][d] : 0;
            isb[d] = use && sh.dwhich[m][d] != 0;
        }
        const uint4* dl_m = dlds + m * NDMAX * 128 + lane;
        const float* xo = bt.x + (bo < bt.B ? bo : 0) * (int64_t)L * DD;
        const unsigned char* hbase = mxs + (m * MXG + bc) * MXRS;
        const float Qb = sh.R[m][bc];
        float pam = 0.f, pbm = 0.f;
        // The K-loop is compiled for KS = NKMAX and KS = NKMAX - 1 steps and
        // chosen by the window (uniform), as in the forward.
        auto run = [&](auto ks) {
        constexpr int KS = decltype(ks)::value;
        bf16x8 Wh[KS], Wl[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
            mx_tile4(sh.wq[m], 32 * (NKMAX - 1 - s) + 31, lane, s < NKm, Wh[s], Wl[s], -1);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            mx_pin(Wh[s]);
            mx_pin(Wl[s]);
        }
        // x at this lane's outputs of the four tiles, loaded one round ahead
        // (unconditionally: the addresses are clamped)
        float xv[4][4 * DD];
#pragma unroll
        for (int j = 0; j < 4; ++j) mx_load4<DD, VEC>(xo, 16 * hh + 32 * j + 4 * rq, L, xv[j]);
        for (int k = 0; k < nbody; ++k) {
            if (k < nround) {
                const int t0 = MXROUND * k + 16 * hh;
                // 2^{z_j + Q} = f 2^n at this lane's outputs (the products below are
                // moderate even where the factors are not); f = 0 where j is not an
                // output.  (Independent of the products: computed while they run.)
                float fj[4][4];
                int nj[4][4];
                auto factor = [&](int j, int rr) {
                    const int t = t0 + 32 * j + 4 * rq + rr;
                    const float e = mx_zx<DD>(M, xv[j] + rr * DD) + Qb;
                    const float fl = floorf(e);
                    fj[j][rr] = mx_sel(any && bvalid && t < L, ex2(e - fl), 0.f);
                    nj[j][rr] = (int)fminf(fmaxf(fl, -300.f), 300.f);
                };
                const int pr = (t0 + 8 * rq) % MXRING;
                mxf4 acc[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j] = mxf4{0.f, 0.f, 0.f, 0.f};
                bf16x8 eh = ld_bf16x8(hbase + ring_byte(pr, 0)), el = ld_bf16x8(hbase + ring_byte(pr, 0) + 16);
#pragma unroll
                for (int s = 0; s < KS + 3; ++s) {
                    bf16x8 ehn = eh, eln = el;
                    if (s + 1 < KS + 3) {
                        const unsigned char* ep = hbase + ring_byte(pr, 32 * (s + 1));
                        ehn = ld_bf16x8(ep);
                        eln = ld_bf16x8(ep + 16);
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int st = s - j;
                        if (st >= 0 && st < KS) {
                            acc[j] = mfma(Wh[st], eh, acc[j]);
                            acc[j] = mfma(Wh[st], el, acc[j]);
                            acc[j] = mfma(Wl[st], eh, acc[j]);
                        }
                    }
                    eh = ehn;
                    el = eln;
                    // (one factor per step, among the products: the scheduler
                    // keeps each step's instructions together; the last step
                    // also takes those of the steps a shorter loop lacks)
                    if (s < 15) factor(s >> 2, s & 3);
                    if (s == KS + 2)
#pragma unroll
                        for (int q = KS + 3; q < 15; ++q) factor(q >> 2, q & 3);
                    __builtin_amdgcn_sched_barrier(0);
                }
                factor(3, 3);
#pragma unroll
                for (int j = 0; j < 4; ++j) mx_load4<DD, VEC>(xo, t0 + MXROUND + 32 * j + 4 * rq, L, xv[j]);
                // d/dx factors (times w of the predicate, by the staging waves)
                float4* ob = (float4*)gbuf + ((((k & 1) * N + m) * 2 + hh) * 4) * 64 + lane;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float g[4];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) g[rr] = ldexpf(acc[j][rr] * fj[j][rr], nj[j][rr]);
                    ob[j * 64] = make_float4(g[0], g[1], g[2], g[3]);
                }
                // derivative sums: product (d, j) of tile d and the terms of
                // K-step dst[d] + j goes into accumulator j.  The weighted sum
                // over this lane's outputs is linear, so each kind's products
                // are summed on the matrix cores and weighted once: the tiles
                // are listed d/da first (na of them), and the d/da sums are
                // taken where the d/db tiles begin.  Terms are read one product
                // ahead.
                int na = 0;
#pragma unroll
                for (int d = 0; d < NDMAX; ++d) na += (d < nd && !isb[d]) ? 1 : 0;
                na = __builtin_amdgcn_readfirstlane(na);
                auto wsum = [&](const mxf4* a) {
                    float r = 0.f;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int q = 0; q < 4; ++q) r += ldexpf(a[j][q] * fj[j][q], nj[j][q]);
                    return r;
                };
                mxf4 ad[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) ad[j] = mxf4{0.f, 0.f, 0.f, 0.f};
                bf16x8 dh = ld_bf16x8(hbase + ring_byte(pr, 32 * dst[0])),
                       dl = ld_bf16x8(hbase + ring_byte(pr, 32 * dst[0]) + 16);
                bf16x8 Dh, Dl;
#pragma unroll
                for (int i = 0; i < NDMAX * 4; ++i) {
                    const int d = i >> 2, j = i & 3;
                    if (j == 0) {
                        Dh = ld_bf16x8(dl_m + d * 128);
                        Dl = ld_bf16x8(dl_m + d * 128 + 64);
                        if (d > 0 && d == na) {
                            // (uniform) the d/da tiles are done
                            pam += wsum(ad);
#pragma unroll
                            for (int j2 = 0; j2 < 4; ++j2) ad[j2] = mxf4{0.f, 0.f, 0.f, 0.f};
                        }
                    }
                    bf16x8 dhn = dh, dln = dl;
                    if (i + 1 < NDMAX * 4) {
                        const unsigned char* ep = hbase + ring_byte(pr, 32 * (dst[(i + 1) >> 2] + ((i + 1) & 3)));
                        dhn = ld_bf16x8(ep);
                        dln = ld_bf16x8(ep + 16);
                    }
                    ad[j] = mfma(Dh, dh, ad[j]);
                    ad[j] = mfma(Dh, dl, ad[j]);
                    ad[j] = mfma(Dl, dh, ad[j]);
                    dh = dhn;
                    dl = dln;
                }
                // (the last kind's sums: d/db, or d/da when every listed tile is one)
                const float last = wsum(ad);
                pam += na >= nd ? last : 0.f;
                pbm += na >= nd ? 0.f : last;
            }
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                mx_pin(Wh[s]);
                mx_pin(Wl[s]);
            }
            __syncthreads();
        }
        };
        if (NKm < NKMAX) run(std::integral_constant<int, NKMAX - 1>{});
        else run(std::integral_constant<int, NKMAX>{});
        // ---- d/da, d/db partials: lanes of one trajectory (l, l + 16, l + 32,
        // l + 48), then the mask's two matrix waves in order
        pam *= M.sg / M.beta;
        pbm *= M.sg / M.beta;
        pam += __shfl_xor(pam, 16);
        pbm += __shfl_xor(pbm, 16);
        pam += __shfl_xor(pam, 32);
        pbm += __shfl_xor(pbm, 32);
        if (lane < MXG) {
            sh.pp[m][0][hh][lane] = pam;
            sh.pp[m][1][hh][lane] = pbm;
        }
    } else {
        // ---------------------------------------------------------- staging waves
        const int vw = wv - 2 * N, vt = tid - 128 * N;
        float wd[N][DD];
#pragma unroll
        for (int mm = 0; mm < N; ++mm) {
            const MxMask<DD> M = mx_mask<DD>(Pk, ka.params, mm);
#pragma unroll
            for (int d = 0; d < DD; ++d) wd[mm][d] = M.w[d];
        }
        float* const dx = ka.dx;
        const Unit U0 = unit(vt), U1 = unit(vt + 128 * N);
        // G and l of block k + 4 are loaded two rounds before they are staged
        float gq0[2][8], lq0[2][8], gq1[2][8], lq1[2][8];
        stage_load(U0, 4, gq0[0], lq0[0]);
        stage_load(U1, 4, gq0[1], lq0[1]);
        auto body = [&](const int k, float (*gn)[8], float (*ln)[8], float (*gx)[8], float (*lx)[8]) {
            stage_load(U0, k + 5, gx[0], lx[0]);
            stage_load(U1, k + 5, gx[1], lx[1]);
            if (k >= 1 && k <= nround) {
                // d/dx of round k - 1: this wave's tiles tau = vw * 4 / N + i
                const int kr = k - 1;
                const float4* ib = (const float4*)gbuf + (kr & 1) * N * 8 * 64 + lane;
#pragma unroll
                for (int i = 0; i < 4 / N; ++i) {
                    const int tau = vw * (4 / N) + i, hh = tau >> 2, j = tau & 3;
                    const int j0 = MXROUND * kr + 16 * hh + 32 * j + 4 * rq;
                    float g[4 * DD];
#pragma unroll
                    for (int q = 0; q < 4 * DD; ++q) g[q] = 0.f;
#pragma unroll
                    for (int mm = 0; mm < N; ++mm) {
                        const float4 a4 = ib[((mm * 2 + hh) * 4 + j) * 64];
                        const float a[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                            for (int d = 0; d < DD; ++d) g[rr * DD + d] = fmaf(wd[mm][d], a[rr], g[rr * DD + d]);
                    }
                    const int nv = min(4, L - j0);
                    if (bvalid && nv > 0) {
                        float* dp = dx + (bo * (int64_t)L + j0) * DD;
                        if (VEC || (nv == 4 && (((uintptr_t)dp) & 15) == 0)) {
#pragma unroll
                            for (int q = 0; q < DD; ++q)
                                *(float4*)(dp + 4 * q) = make_float4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
                        } else {
                            for (int q = 0; q < nv * DD; ++q) dp[q] = g[q];
                        }
                    }
                }
            }
            if (k < nround) {
                stage_write(U0, k + 4, gn[0], ln[0]);
                stage_write(U1, k + 4, gn[1], ln[1]);
            }
            __syncthreads();
        };
        for (int k = 0; k < nbody; k += 2) {
            body(k, gq0, lq0, gq1, lq1);
            body(k + 1, gq1, lq1, gq0, lq0);
        }
    }
    __syncthreads();
    if (tid < 2 * N * MXG) {
        const int mm = tid / (2 * MXG), ab = (tid / MXG) & 1, r = tid % MXG;
        const int64_t bq = g0 + r;
        if (bq < bt.B && !sh.frag[r] && !over) {
            const float s = sh.pp[mm][ab][0][r] + sh.pp[mm][ab][1][r];
            const int slot = Pk->ins[Pk->fused.ins[mm]].mslot;
            if (slot >= 0) mx.part[(bq * P.n_masks + slot) * 2 + ab] = s;
        }
    }
    if (tid < MXG) finish_row(tid, sh.frag[tid] || over);
}

}  // namespace stlmi
