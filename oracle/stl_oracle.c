/*
 * FP64 reference for STL robustness traces and their gradients.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Every operator is evaluated straight from its definition, one output at a
 * time, with plain loops over the window (O(L*|window|)) and, for Until, a
 * loop over the inner index with the running minimum (O(L*b)).  Paper
 * references (arXiv 2501.04194):
 *   - quantitative semantics (robustness)       : Sec. III-B, eq. (quantitative)
 *   - derived operators Or / Eventually / Always: Sec. III-B, after eq. (grammar)
 *   - logsumexp smooth max / min                : Sec. III-C
 *   - robustness trace                          : Sec. III-D, Definition 1
 *   - Eventually / Always by masked window max  : Sec. IV-B, Steps 1-3, Example 1
 *   - Until as max_i min(min_{k<=i} phi, psi_i)  : Sec. IV-C, Steps 1-3
 *   - LSE associativity (flat == nested)        : Sec. IV-D
 *   - smooth time-interval mask                 : Sec. VI, eq. (smooth mask)
 *
 * Readings of the paper used here (each one is listed in the design notes):
 *   - a trace has L samples, indices 0..L-1; intervals [a,b] are inclusive
 *     timestep offsets; b < 0 encodes an unbounded interval (to the end).
 *   - pad policy NEUTRAL (default): window positions past L-1 are dropped; an
 *     empty window gives -rho_pad for max-type and +rho_pad for min-type
 *     operators.  LAST: positions past the end read u[L-1] (each counts once
 *     in a smooth sum).  CONST: they read pad_value.  Unbounded windows and
 *     Until always clip (NEUTRAL).  On a window with a bounded smooth mask,
 *     LAST / CONST give every offset k of the mask support with t+k past
 *     the end one pad copy of weight w_k (the support ends where w_k drops
 *     to zero, which it does past b for eps > 0).
 *   - a smooth mask on Until weights the outer index i (the psi index, the
 *     one the interval [a,b] constrains); the running smooth min of phi over
 *     [0,i] is not weighted.  The hard variant keeps {i : w_i > 0}.
 *   - smooth operators use beta (= 1/temperature) inside the exponent:
 *     smax(V) = (1/beta) log sum exp(beta v), smin(V) = -smax(-V).
 *     smooth = 2 selects the softmax-weighted form of Sec. III-C instead,
 *     smax(V) = sum v exp(beta v) / sum exp(beta v) (the printed denominator
 *     index is read as running over all of V), smin(V) = -smax(-V); on And/Or
 *     and on unmasked Eventually/Always windows.
 *   - the smooth mask weight enters the logsumexp as a multiplicative weight:
 *     out_t = (1/beta) log sum_{k>=0, t+k<L} w_k exp(beta u_{t+k}),
 *     w_k = max(sig(c(k-a)) - sig(c(k-b)) - eps, 0), a and b in timesteps.
 *     The hard variant takes the max over {k : w_k > 0}.
 *   - Until is inclusive: phi must also hold at the psi index.
 *   - hard tie-break: the lowest time index wins; for n-ary and/or the lowest
 *     child wins; in Until's min(min phi, psi) the phi side wins ties.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { O_TRUE = 0, O_LINEAR = 1, O_NORM = 2, O_NOT = 3, O_AND = 4, O_OR = 5,
       O_EV = 6, O_ALW = 7, O_UNTIL = 8 };
enum { P_NEUTRAL = 0, P_LAST = 1, P_CONST = 2 };

#define OMAXCH 16
#define OMAXD 16

typedef struct {
    int op;
    int nch;
    int ch[OMAXCH];      /* child node indices; always smaller than this node's */
    int smooth;
    double beta;
    int a, b;            /* b < 0 : unbounded */
    int masked;          /* smooth sigmoid time mask instead of [a,b] */
    double ma, mb, mc, meps;
    int mb_inf;
    int pad;
    double pad_value;
    int D;
    double w[OMAXD];     /* linear: w.x - c */
    double c;
    int m;               /* norm: sign*(||A x - p|| - r), A is m x D */
    double A[4 * OMAXD];
    double p[4];
    double r;
    double sign;
} onode;

/* ---------------------------------------------------------------- helpers */

static double sigm(double z)
{
    if (z >= 0) return 1.0 / (1.0 + exp(-z));
    double e = exp(z);
    return e / (1.0 + e);
}

/* Smooth mask weight of Sec. VI for offset k (timesteps):
 * sig(x) - sig(y) - eps with x = c(k-a), y = c(k-b).  The difference is
 * evaluated through the identity sig(x) - sig(y) = sig(x) sig(-y) (1 - e^{y-x})
 * (put the two fractions over one denominator), which has no cancellation:
 * where both sigmoids round to 1 the literal difference is 0 in fp64 while
 * the weight is e^{-y}-small but positive, and with eps = 0 such weights can
 * still carry a large exponential term. */
static double mask_weight(const onode *nd, int k)
{
    double x = nd->mc * ((double)k - nd->ma);
    double d;
    if (nd->mb_inf) {
        d = sigm(x);
    } else {
        double y = nd->mc * ((double)k - nd->mb);
        d = sigm(x) * sigm(-y) * -expm1(y - x);
    }
    double w = d - nd->meps;
    return w > 0 ? w : 0.0;
}

/* d w_k / d a = -c sig'(x) and d w_k / d b = c sig'(y), sig' = sig(.) sig(-.)
 * (no 1 - sig cancellation), zero where the max(.,0) clamp is active. */
static void mask_weight_grad(const onode *nd, int k, double *dwa, double *dwb)
{
    double w = mask_weight(nd, k);
    if (w <= 0) { *dwa = 0; *dwb = 0; return; }
    double x = nd->mc * ((double)k - nd->ma);
    *dwa = -nd->mc * sigm(x) * sigm(-x);
    if (nd->mb_inf) { *dwb = 0; return; }
    double y = nd->mc * ((double)k - nd->mb);
    *dwb = nd->mc * sigm(y) * sigm(-y);
}

/* Orientation: +1 for max-type operators (or, eventually), -1 for min-type.
 * A min-type operator is evaluated as the max-type one on sign-flipped values
 * (Sec. III-B derives Always and And from Eventually and Or by negation). */
static double orient(int op)
{
    return (op == O_AND || op == O_ALW) ? -1.0 : 1.0;
}

/* One window element: value (already oriented), weight, gradient target. */
typedef struct { double v, w; int src, off; } welem;   /* off: mask offset k */

/* Collect the window of a temporal node at time t (oriented values). */
static int gather_window(const onode *nd, const double *u, int L, int t, double sg,
                         const double *wtab, welem *out)
{
    int n = 0;
    if (nd->masked) {
        for (int k = 0; t + k < L; ++k) {
            double w = wtab[k];
            if (w > 0) { out[n].v = sg * u[t + k]; out[n].w = w; out[n].src = t + k; out[n].off = k; ++n; }
        }
        if (nd->pad != P_NEUTRAL && !nd->mb_inf) {
            /* offsets past the signal end: one pad copy per support offset */
            for (int k = L - t; ; ++k) {
                double w = mask_weight(nd, k);
                if (w > 0) {
                    out[n].v = sg * (nd->pad == P_LAST ? u[L - 1] : nd->pad_value);
                    out[n].w = w;
                    out[n].src = nd->pad == P_LAST ? L - 1 : -1;
                    out[n].off = k;
                    ++n;
                } else if ((double)k > nd->mb) {
                    break;
                }
            }
        }
        return n;
    }
    int ihi = nd->b < 0 ? (L - 1 - t) : nd->b;
    for (int i = nd->a; i <= ihi; ++i) {
        int j = t + i;
        if (j <= L - 1) { out[n].v = sg * u[j]; out[n].w = 1; out[n].src = j; out[n].off = i; ++n; }
        else if (nd->b >= 0 && nd->pad == P_LAST) {
            out[n].v = sg * u[L - 1]; out[n].w = 1; out[n].src = L - 1; out[n].off = i; ++n;
        } else if (nd->b >= 0 && nd->pad == P_CONST) {
            out[n].v = sg * nd->pad_value; out[n].w = 1; out[n].src = -1; out[n].off = i; ++n;
        }
    }
    return n;
}

/* hard max: strict '>' keeps the first (lowest-index) maximiser */
static int hard_argmax(const welem *e, int n)
{
    int best = 0;
    for (int i = 1; i < n; ++i)
        if (e[i].v > e[best].v) best = i;
    return best;
}

/* weighted logsumexp (1/beta) log sum w exp(beta v), max-shifted */
static double wlse(const welem *e, int n, double beta)
{
    double m = e[0].v;
    for (int i = 1; i < n; ++i) if (e[i].v > m) m = e[i].v;
    double s = 0;
    for (int i = 0; i < n; ++i) s += e[i].w * exp(beta * (e[i].v - m));
    return m + log(s) / beta;
}

/* softmax-weighted mean sum w v exp(beta v) / sum w exp(beta v), max-shifted */
static double wsoft(const welem *e, int n, double beta)
{
    double m = e[0].v;
    for (int i = 1; i < n; ++i) if (e[i].v > m) m = e[i].v;
    double s0 = 0, s1 = 0;
    for (int i = 0; i < n; ++i) {
        double q = e[i].w * exp(beta * (e[i].v - m));
        s0 += q;
        s1 += q * e[i].v;
    }
    return s1 / s0;
}

/* d wsoft / d v_k = p_k (1 + beta (v_k - r)), p_k = w_k exp(beta v_k) / sum */
static void wsoft_grad(const welem *e, int n, double beta, double r, double *d)
{
    double m = e[0].v;
    for (int i = 1; i < n; ++i) if (e[i].v > m) m = e[i].v;
    double s0 = 0;
    for (int i = 0; i < n; ++i) s0 += e[i].w * exp(beta * (e[i].v - m));
    for (int i = 0; i < n; ++i) d[i] = e[i].w * exp(beta * (e[i].v - m)) / s0 * (1.0 + beta * (e[i].v - r));
}

/* ------------------------------------------------------------- forward */

static void fwd_node(const onode *nodes, int idx, const double *x, int L, int D,
                     double rho_max, double rho_pad, double *tr, welem *buf, double *wtab,
                     double *tmpR)
{
    const onode *nd = &nodes[idx];
    double *out = tr + (size_t)idx * L;
    switch (nd->op) {
    case O_TRUE:
        for (int t = 0; t < L; ++t) out[t] = rho_max;
        break;
    case O_LINEAR:
        for (int t = 0; t < L; ++t) {
            double s = 0;
            for (int d = 0; d < D; ++d) s += nd->w[d] * x[(size_t)t * D + d];
            out[t] = s - nd->c;
        }
        break;
    case O_NORM:
        for (int t = 0; t < L; ++t) {
            double q = 0;
            for (int i = 0; i < nd->m; ++i) {
                double z = -nd->p[i];
                for (int d = 0; d < D; ++d) z += nd->A[i * D + d] * x[(size_t)t * D + d];
                q += z * z;
            }
            out[t] = nd->sign * (sqrt(q) - nd->r);
        }
        break;
    case O_NOT: {
        const double *u = tr + (size_t)nd->ch[0] * L;
        for (int t = 0; t < L; ++t) out[t] = -u[t];
        break;
    }
    case O_AND:
    case O_OR: {
        double sg = orient(nd->op);
        for (int t = 0; t < L; ++t) {
            for (int k = 0; k < nd->nch; ++k) {
                buf[k].v = sg * tr[(size_t)nd->ch[k] * L + t]; buf[k].w = 1; buf[k].src = k;
            }
            double r = nd->smooth == 2 ? wsoft(buf, nd->nch, nd->beta)
                       : nd->smooth ? wlse(buf, nd->nch, nd->beta) : buf[hard_argmax(buf, nd->nch)].v;
            out[t] = sg * r;
        }
        break;
    }
    case O_EV:
    case O_ALW: {
        double sg = orient(nd->op);
        const double *u = tr + (size_t)nd->ch[0] * L;
        if (nd->masked) for (int k = 0; k < L; ++k) wtab[k] = mask_weight(nd, k);
        for (int t = 0; t < L; ++t) {
            int n = gather_window(nd, u, L, t, sg, wtab, buf);
            double r;
            if (n == 0) r = -rho_pad;
            else if (nd->smooth == 2) r = wsoft(buf, n, nd->beta);
            else if (nd->smooth) r = wlse(buf, n, nd->beta);
            else r = buf[hard_argmax(buf, n)].v;
            out[t] = sg * r;
        }
        break;
    }
    case O_UNTIL: {
        const double *phi = tr + (size_t)nd->ch[0] * L;
        const double *psi = tr + (size_t)nd->ch[1] * L;
        double beta = nd->beta;
        if (nd->masked) for (int k = 0; k < L; ++k) wtab[k] = mask_weight(nd, k);
        for (int t = 0; t < L; ++t) {
            /* a masked Until walks every i to the end and keeps those with w_i > 0 */
            int imax = (nd->b < 0 || nd->masked) ? L - 1 - t : (nd->b < L - 1 - t ? nd->b : L - 1 - t);
            if (!nd->masked && nd->a > imax) { out[t] = -rho_pad; continue; }
            if (!nd->smooth) {
                double R = 0, best = 0;
                int have = 0;
                for (int i = 0; i <= imax; ++i) {
                    double f = phi[t + i];
                    if (i == 0 || f < R) R = f;              /* running min over k in [0,i] */
                    if (nd->masked ? wtab[i] > 0 : i >= nd->a) {
                        double v = (R <= psi[t + i]) ? R : psi[t + i];  /* min(R, psi) */
                        if (!have || v > best) { best = v; have = 1; }
                    }
                }
                out[t] = have ? best : -rho_pad;
            } else {
                /* R_i = smin(phi_t..phi_{t+i}) via a max-shifted running sum of
                 * exp(-beta phi); v_i = smin(R_i, psi_{t+i}); out = smax_i v_i. */
                double mneg = 0, s = 0;
                int nv = 0;
                for (int i = 0; i <= imax; ++i) {
                    double q = -phi[t + i];
                    if (i == 0) { mneg = q; s = 1; }
                    else if (q > mneg) { s = s * exp(beta * (mneg - q)) + 1; mneg = q; }
                    else s += exp(beta * (q - mneg));
                    double R = -(mneg + log(s) / beta);
                    tmpR[i] = R;
                    if (nd->masked ? wtab[i] > 0 : i >= nd->a) {
                        double p = psi[t + i];
                        /* smin of the pair (R, psi) */
                        double lo = R < p ? R : p;
                        double v = lo - log(exp(-beta * (R - lo)) + exp(-beta * (p - lo))) / beta;
                        buf[nv].v = v; buf[nv].w = nd->masked ? wtab[i] : 1; buf[nv].src = i; buf[nv].off = i;
                        ++nv;
                    }
                }
                out[t] = nv ? wlse(buf, nv, beta) : -rho_pad;
            }
        }
        break;
    }
    }
}

/* Forward for one trajectory: traces tr[n][L]; leaf rows flagged in
 * `override_mask` are taken from `override_tr` instead of being computed. */
static void fwd_traj(const onode *nodes, int n, const double *x, int L, int D,
                     double rho_max, double rho_pad, const int *override_mask,
                     const double *override_tr, double *tr, welem *buf, double *wtab, double *tmpR)
{
    for (int i = 0; i < n; ++i) {
        if (override_mask && override_mask[i]) {
            memcpy(tr + (size_t)i * L, override_tr + (size_t)i * L, sizeof(double) * L);
            continue;
        }
        fwd_node(nodes, i, x, L, D, rho_max, rho_pad, tr, buf, wtab, tmpR);
    }
}

/* ------------------------------------------------------------- backward */

static void bwd_node(const onode *nodes, int idx, const double *x, int L, int D,
                     double rho_pad, const double *tr, double *gb, double *dx, double *dpar,
                     welem *buf, double *wtab, double *dwa, double *dwb, double *tmpR,
                     double *tmpV, double *tmpRb)
{
    const onode *nd = &nodes[idx];
    const double *g = gb + (size_t)idx * L;
    const double *out = tr + (size_t)idx * L;
    switch (nd->op) {
    case O_TRUE:
        break;
    case O_LINEAR:
        for (int t = 0; t < L; ++t)
            for (int d = 0; d < D; ++d) dx[(size_t)t * D + d] += nd->w[d] * g[t];
        break;
    case O_NORM:
        for (int t = 0; t < L; ++t) {
            double z[4], q = 0;
            for (int i = 0; i < nd->m; ++i) {
                z[i] = -nd->p[i];
                for (int d = 0; d < D; ++d) z[i] += nd->A[i * D + d] * x[(size_t)t * D + d];
                q += z[i] * z[i];
            }
            double nz = sqrt(q);
            if (nz <= 0) continue;                   /* subgradient 0 at A x = p */
            for (int d = 0; d < D; ++d) {
                double s = 0;
                for (int i = 0; i < nd->m; ++i) s += nd->A[i * D + d] * z[i];
                dx[(size_t)t * D + d] += nd->sign * g[t] * s / nz;
            }
        }
        break;
    case O_NOT: {
        double *gc = gb + (size_t)nd->ch[0] * L;
        for (int t = 0; t < L; ++t) gc[t] -= g[t];
        break;
    }
    case O_AND:
    case O_OR: {
        double sg = orient(nd->op);
        for (int t = 0; t < L; ++t) {
            for (int k = 0; k < nd->nch; ++k) {
                buf[k].v = sg * tr[(size_t)nd->ch[k] * L + t]; buf[k].w = 1; buf[k].src = k;
            }
            if (nd->smooth == 2) {
                double d[OMAXCH];
                wsoft_grad(buf, nd->nch, nd->beta, sg * out[t], d);
                for (int k = 0; k < nd->nch; ++k) gb[(size_t)nd->ch[k] * L + t] += g[t] * d[k];
            } else if (nd->smooth) {
                double o = sg * out[t];
                for (int k = 0; k < nd->nch; ++k)
                    gb[(size_t)nd->ch[k] * L + t] += g[t] * exp(nd->beta * (buf[k].v - o));
            } else {
                int k = hard_argmax(buf, nd->nch);
                gb[(size_t)nd->ch[k] * L + t] += g[t];
            }
        }
        break;
    }
    case O_EV:
    case O_ALW: {
        double sg = orient(nd->op);
        const double *u = tr + (size_t)nd->ch[0] * L;
        double *gu = gb + (size_t)nd->ch[0] * L;
        if (nd->masked)
            for (int k = 0; k < L; ++k) { wtab[k] = mask_weight(nd, k); mask_weight_grad(nd, k, &dwa[k], &dwb[k]); }
        for (int t = 0; t < L; ++t) {
            int n = gather_window(nd, u, L, t, sg, wtab, buf);
            if (n == 0 || g[t] == 0) continue;
            if (!nd->smooth) {
                int k = hard_argmax(buf, n);
                if (buf[k].src >= 0) gu[buf[k].src] += g[t];
                continue;
            }
            if (nd->smooth == 2) {
                wsoft_grad(buf, n, nd->beta, sg * out[t], tmpV);
                for (int k = 0; k < n; ++k)
                    if (buf[k].src >= 0) gu[buf[k].src] += g[t] * tmpV[k];
                continue;
            }
            double o = sg * out[t];
            double ga = 0, gbb = 0;
            for (int k = 0; k < n; ++k) {
                double e = exp(nd->beta * (buf[k].v - o));        /* d out / d (w_k e^{beta v}) * ... */
                if (buf[k].src >= 0) gu[buf[k].src] += g[t] * buf[k].w * e;
                if (nd->masked) {
                    int off = buf[k].off;
                    double da, db;
                    if (off < L) { da = dwa[off]; db = dwb[off]; }
                    else mask_weight_grad(nd, off, &da, &db);   /* a pad copy past the end */
                    ga += da * e;
                    gbb += db * e;
                }
            }
            if (nd->masked) {
                dpar[2 * idx + 0] += g[t] * sg * ga / nd->beta;
                dpar[2 * idx + 1] += g[t] * sg * gbb / nd->beta;
            }
        }
        break;
    }
    case O_UNTIL: {
        const double *phi = tr + (size_t)nd->ch[0] * L;
        const double *psi = tr + (size_t)nd->ch[1] * L;
        double *gphi = gb + (size_t)nd->ch[0] * L;
        double *gpsi = gb + (size_t)nd->ch[1] * L;
        double beta = nd->beta;
        if (nd->masked)
            for (int k = 0; k < L; ++k) { wtab[k] = mask_weight(nd, k); mask_weight_grad(nd, k, &dwa[k], &dwb[k]); }
        for (int t = 0; t < L; ++t) {
            int imax = (nd->b < 0 || nd->masked) ? L - 1 - t : (nd->b < L - 1 - t ? nd->b : L - 1 - t);
            if ((!nd->masked && nd->a > imax) || g[t] == 0) continue;
            if (!nd->smooth) {
                double R = 0, best = 0;
                int kR = 0, have = 0, tgt_phi = 0, tgt = 0;
                for (int i = 0; i <= imax; ++i) {
                    double f = phi[t + i];
                    if (i == 0 || f < R) { R = f; kR = i; }
                    if (nd->masked ? wtab[i] > 0 : i >= nd->a) {
                        int phiwin = R <= psi[t + i];
                        double v = phiwin ? R : psi[t + i];
                        if (!have || v > best) { best = v; have = 1; tgt_phi = phiwin; tgt = phiwin ? kR : i; }
                    }
                }
                if (!have) continue;                         /* empty window: constant output */
                if (tgt_phi) gphi[t + tgt] += g[t]; else gpsi[t + tgt] += g[t];
                continue;
            }
            /* forward recompute: R_i (running smin of phi) and v_i = smin(R_i, psi_{t+i}) */
            double mneg = 0, s = 0;
            int nv = 0;
            for (int i = 0; i <= imax; ++i) {
                double q = -phi[t + i];
                if (i == 0) { mneg = q; s = 1; }
                else if (q > mneg) { s = s * exp(beta * (mneg - q)) + 1; mneg = q; }
                else s += exp(beta * (q - mneg));
                tmpR[i] = -(mneg + log(s) / beta);
                if (nd->masked ? wtab[i] > 0 : i >= nd->a) {
                    ++nv;
                    double R = tmpR[i], p = psi[t + i];
                    double lo = R < p ? R : p;
                    tmpV[i] = lo - log(exp(-beta * (R - lo)) + exp(-beta * (p - lo))) / beta;
                }
            }
            if (nv == 0) continue;                           /* empty window: constant output */
            double o = out[t];
            double ga = 0, gbb = 0;
            /* reverse sweep: R_i = smin2(R_{i-1}, phi_{t+i}) (Sec. IV-D: the
             * running smooth min equals the flat one) */
            for (int i = 0; i <= imax; ++i) tmpRb[i] = 0;
            for (int i = imax; i >= 0; --i) {
                if (nd->masked ? wtab[i] > 0 : i >= nd->a) {
                    double e = exp(beta * (tmpV[i] - o));
                    double gv = g[t] * (nd->masked ? wtab[i] : 1.0) * e;    /* d out / d v_i */
                    if (nd->masked) { ga += dwa[i] * e; gbb += dwb[i] * e; }
                    tmpRb[i] += gv * exp(-beta * (tmpR[i] - tmpV[i]));       /* d v_i / d R_i */
                    gpsi[t + i] += gv * exp(-beta * (psi[t + i] - tmpV[i])); /* d v_i / d psi */
                }
                if (i == 0) { gphi[t] += tmpRb[0]; break; }
                gphi[t + i] += tmpRb[i] * exp(-beta * (phi[t + i] - tmpR[i]));
                tmpRb[i - 1] += tmpRb[i] * exp(-beta * (tmpR[i - 1] - tmpR[i]));
            }
            if (nd->masked) {
                /* d out / d w_i = exp(beta (v_i - out)) / beta */
                dpar[2 * idx + 0] += g[t] * ga / beta;
                dpar[2 * idx + 1] += g[t] * gbb / beta;
            }
        }
        break;
    }
    }
    (void)rho_pad;
}

/* ------------------------------------------------------------- batch API */

typedef struct {
    welem *buf;
    double *wtab, *dwa, *dwb, *tmpR, *tmpV, *tmpRb, *tr, *gb;
} scratch_t;

/* largest window any node can gather for trajectories of length <= L */
static size_t window_cap(const onode *nodes, int n, int L)
{
    size_t cap = (size_t)L + OMAXCH + 16;
    for (int i = 0; i < n; ++i) {
        const onode *nd = &nodes[i];
        if ((nd->op == O_EV || nd->op == O_ALW) && !nd->masked && nd->b >= 0) {
            size_t k = (size_t)(nd->b - nd->a + 1) + 16;
            if (k > cap) cap = k;
        }
        if ((nd->op == O_EV || nd->op == O_ALW) && nd->masked && nd->pad != P_NEUTRAL && !nd->mb_inf) {
            /* pad copies: at most one per offset up to the end of the mask support */
            int kend = 0;
            for (int k = 0; ; ++k) {
                if (mask_weight(nd, k) > 0) kend = k;
                else if ((double)k > nd->mb) break;
            }
            size_t k = (size_t)L + (size_t)kend + 1 + 16;
            if (k > cap) cap = k;
        }
    }
    return cap;
}

static int scratch_alloc(scratch_t *s, const onode *nodes, int n, int L)
{
    size_t Lz = (size_t)(L + OMAXCH + 1);
    s->buf = (welem *)malloc(sizeof(welem) * window_cap(nodes, n, L));
    s->wtab = (double *)malloc(sizeof(double) * Lz);
    s->dwa = (double *)malloc(sizeof(double) * Lz);
    s->dwb = (double *)malloc(sizeof(double) * Lz);
    s->tmpR = (double *)malloc(sizeof(double) * Lz);
    {   /* also the per-element softmax gradients of the widest window */
        size_t wc = window_cap(nodes, n, L);
        s->tmpV = (double *)malloc(sizeof(double) * (wc > Lz ? wc : Lz));
    }
    s->tmpRb = (double *)malloc(sizeof(double) * Lz);
    s->tr = (double *)malloc(sizeof(double) * (size_t)n * Lz);
    s->gb = (double *)malloc(sizeof(double) * (size_t)n * Lz);
    return s->buf && s->wtab && s->dwa && s->dwb && s->tmpR && s->tmpV && s->tmpRb && s->tr && s->gb;
}

static void scratch_free(scratch_t *s)
{
    free(s->buf); free(s->wtab); free(s->dwa); free(s->dwb); free(s->tmpR);
    free(s->tmpV); free(s->tmpRb); free(s->tr); free(s->gb);
}

/*
 * Forward over a batch.  x is [N_total, D] (trajectory b occupies rows
 * offsets[b]..offsets[b+1]-1).  traces receives all node traces as
 * [n][N_total].  override_mask[n] / override_tr[n][N_total] optionally replace
 * node traces (used to feed identical float32 leaf traces to both sides).
 * Returns 0 on success.
 */
int orc_forward(const onode *nodes, int n, const double *x, const long long *offsets, long long B,
                int D, double rho_max, double rho_pad, const int *override_mask,
                const double *override_tr, double *traces)
{
    long long Ntot = offsets[B];
    int Lmax = 1;
    for (long long b = 0; b < B; ++b) {
        long long l = offsets[b + 1] - offsets[b];
        if (l > Lmax) Lmax = (int)l;
    }
    int err = 0;
#pragma omp parallel
    {
        scratch_t s;
        double *ov = NULL;
        int ok = scratch_alloc(&s, nodes, n, Lmax);
        if (override_mask) ov = (double *)malloc(sizeof(double) * (size_t)n * Lmax);
        if (!ok || (override_mask && !ov)) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (long long b = 0; b < B; ++b) {
                long long o0 = offsets[b];
                int L = (int)(offsets[b + 1] - o0);
                if (L <= 0) continue;
                if (override_mask)
                    for (int i = 0; i < n; ++i)
                        if (override_mask[i])
                            memcpy(ov + (size_t)i * L, override_tr + (size_t)i * Ntot + o0, sizeof(double) * L);
                fwd_traj(nodes, n, x + (size_t)o0 * D, L, D, rho_max, rho_pad, override_mask, ov,
                         s.tr, s.buf, s.wtab, s.tmpR);
                for (int i = 0; i < n; ++i)
                    memcpy(traces + (size_t)i * Ntot + o0, s.tr + (size_t)i * L, sizeof(double) * L);
            }
        }
        scratch_free(&s);
        free(ov);
    }
    return err;
}

/*
 * Backward over a batch: G is the upstream gradient of the root trace
 * (node n-1), [N_total].  dx [N_total, D] is overwritten; dparam_traj
 * [B][n][2] receives per-trajectory d/da and d/db of every masked node
 * (summed in trajectory order by the caller for a deterministic total).
 */
int orc_backward(const onode *nodes, int n, const double *x, const long long *offsets, long long B,
                 int D, double rho_max, double rho_pad, const int *override_mask,
                 const double *override_tr, const double *G, double *dx, double *dparam_traj)
{
    long long Ntot = offsets[B];
    int Lmax = 1;
    for (long long b = 0; b < B; ++b) {
        long long l = offsets[b + 1] - offsets[b];
        if (l > Lmax) Lmax = (int)l;
    }
    memset(dx, 0, sizeof(double) * (size_t)Ntot * D);
    memset(dparam_traj, 0, sizeof(double) * (size_t)B * n * 2);
    int err = 0;
#pragma omp parallel
    {
        scratch_t s;
        double *ov = NULL;
        int ok = scratch_alloc(&s, nodes, n, Lmax);
        if (override_mask) ov = (double *)malloc(sizeof(double) * (size_t)n * Lmax);
        if (!ok || (override_mask && !ov)) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (long long b = 0; b < B; ++b) {
                long long o0 = offsets[b];
                int L = (int)(offsets[b + 1] - o0);
                if (L <= 0) continue;
                if (override_mask)
                    for (int i = 0; i < n; ++i)
                        if (override_mask[i])
                            memcpy(ov + (size_t)i * L, override_tr + (size_t)i * Ntot + o0, sizeof(double) * L);
                const double *xb = x + (size_t)o0 * D;
                fwd_traj(nodes, n, xb, L, D, rho_max, rho_pad, override_mask, ov, s.tr, s.buf, s.wtab, s.tmpR);
                memset(s.gb, 0, sizeof(double) * (size_t)n * L);
                memcpy(s.gb + (size_t)(n - 1) * L, G + o0, sizeof(double) * L);
                double *dxb = dx + (size_t)o0 * D;
                double *dp = dparam_traj + (size_t)b * n * 2;
                for (int i = n - 1; i >= 0; --i) {
                    if (override_mask && override_mask[i]) continue;   /* leaf fed from outside */
                    bwd_node(nodes, i, xb, L, D, rho_pad, s.tr, s.gb, dxb, dp, s.buf, s.wtab,
                             s.dwa, s.dwb, s.tmpR, s.tmpV, s.tmpRb);
                }
            }
        }
        scratch_free(&s);
        free(ov);
    }
    (void)rho_max;
    return err;
}

/*
 * Backward that also returns the adjoint of every node trace
 * ([n][N_total]); used by tests that compare per-node gradients.
 */
int orc_backward_nodes(const onode *nodes, int n, const double *x, const long long *offsets,
                       long long B, int D, double rho_max, double rho_pad, const double *G,
                       double *dx, double *dparam_traj, double *node_adj)
{
    long long Ntot = offsets[B];
    int Lmax = 1;
    for (long long b = 0; b < B; ++b) {
        long long l = offsets[b + 1] - offsets[b];
        if (l > Lmax) Lmax = (int)l;
    }
    memset(dx, 0, sizeof(double) * (size_t)Ntot * D);
    memset(dparam_traj, 0, sizeof(double) * (size_t)B * n * 2);
    scratch_t s;
    if (!scratch_alloc(&s, nodes, n, Lmax)) { scratch_free(&s); return 1; }
    for (long long b = 0; b < B; ++b) {
        long long o0 = offsets[b];
        int L = (int)(offsets[b + 1] - o0);
        if (L <= 0) continue;
        const double *xb = x + (size_t)o0 * D;
        fwd_traj(nodes, n, xb, L, D, rho_max, rho_pad, NULL, NULL, s.tr, s.buf, s.wtab, s.tmpR);
        memset(s.gb, 0, sizeof(double) * (size_t)n * L);
        memcpy(s.gb + (size_t)(n - 1) * L, G + o0, sizeof(double) * L);
        for (int i = n - 1; i >= 0; --i)
            bwd_node(nodes, i, xb, L, D, rho_pad, s.tr, s.gb, dx + (size_t)o0 * D,
                     dparam_traj + (size_t)b * n * 2, s.buf, s.wtab, s.dwa, s.dwb, s.tmpR,
                     s.tmpV, s.tmpRb);
        for (int i = 0; i < n; ++i)
            memcpy(node_adj + (size_t)i * Ntot + o0, s.gb + (size_t)i * L, sizeof(double) * L);
    }
    scratch_free(&s);
    return 0;
}

/* Mask weights w_k, k = 0..L-1, for one masked node (used by pins). */
void orc_mask_weights(const onode *nd, int L, double *w, double *dwa, double *dwb)
{
    for (int k = 0; k < L; ++k) {
        w[k] = mask_weight(nd, k);
        mask_weight_grad(nd, k, &dwa[k], &dwb[k]);
    }
}

int orc_sizeof_node(void) { return (int)sizeof(onode); }
