// Plan compiler of the STL robustness library (host only, no HIP): checks
// the caller's node array (Fig. 2: a formula as a graph of operators),
// orders it, lowers each node to the executor's instructions (Sec. III-B/C,
// IV-B/C, VI) and allocates their trace slots by liveness; the longest-first
// processing order of ragged batches; the error channel.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "stl_host.h"

using namespace stlmi;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

stl_status stlmi::fail(stl_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

extern "C" const char* stl_last_error(void) { return g_err.c_str(); }

void stlmi_set_error(const char* msg) { g_err = msg; }

// ------------------------------------------------------------------ plan compiler



namespace {

struct Builder {
    const stl_node* nodes;
    int n_nodes;
    const int32_t* child_idx;
    int n_child_idx;
    const stl_pred* preds;
    int n_preds;
    int D;
    int n_params;
    std::vector<Instr> ins;
    std::vector<std::vector<int>> kids;   // instruction children (instruction indices)
    std::vector<float> coef;
    std::vector<int> pred_ins;
    std::vector<int> mask_params;
    int max_until_b = 0;
    bool has_until = false;

    int new_instr(Instr I, std::vector<int> ch)
    {
        ins.push_back(I);
        kids.push_back(std::move(ch));
        return (int)ins.size() - 1;
    }
};

Instr blank()
{
    Instr I;
    std::memset(&I, 0, sizeof I);
    I.f_out = I.f_in0 = I.f_in1 = -1;
    I.b_out = I.b_in0 = I.b_in1 = -1;
    I.g_out = I.g_in0 = I.g_in1 = -1;
    I.beta = I.mask = I.mslot = -1;
    for (int k = 0; k < MAX_NCH; ++k) I.f_ch[k] = I.b_ch[k] = I.g_ch[k] = -1;
    I.node = -1;
    I.coef = 0;
    I.b = -1;
    return I;
}

// emit the instruction(s) of caller node `id` (post-order); returns instruction index
stl_status emit(Builder& B, int id, int depth, int* out)
{
    if (depth > 256) return fail(STL_E_FORMULA, "formula too deep (cycle?) at node %d", id);
    const stl_node& n = B.nodes[id];
    Instr I = blank();
    I.node = (int16_t)id;
    std::vector<int> ch;
    auto child = [&](int k) { return B.child_idx[n.child_off + k]; };
    // children first
    std::vector<int> kid_ins;
    for (int k = 0; k < n.n_child; ++k) {
        int ci;
        stl_status s = emit(B, child(k), depth + 1, &ci);
        if (s != STL_OK) return s;
        kid_ins.push_back(ci);
    }
    const bool smooth = n.smooth != 0;
    if (n.smooth < 0 || n.smooth > 2) return fail(STL_E_ARG, "node %d: smooth must be 0, 1 or 2", id);
    if (smooth) {
        if (n.beta_param < 0 || n.beta_param >= B.n_params)
            return fail(STL_E_ARG, "node %d: smooth node needs beta_param in [0, n_params)", id);
        I.beta = (int8_t)n.beta_param;
        I.flags |= F_SMOOTH;
    }
    if (n.smooth == 2) {
        // softmax-weighted form: And/Or with at most MAX_NCH children (it is not
        // associative, so no regrouping) and unmasked windows
        const bool win = (n.op == STL_EVENTUALLY || n.op == STL_ALWAYS) && n.mask_param < 0;
        const bool nary = (n.op == STL_AND || n.op == STL_OR) && n.n_child <= MAX_NCH;
        if (!win && !nary)
            return fail(STL_E_UNSUPPORTED,
                        "node %d: the softmax-weighted form applies to And/Or with up to %d children and to "
                        "unmasked Eventually/Always",
                        id, MAX_NCH);
        I.flags |= F_SOFT;
    }
    switch (n.op) {
    case STL_TRUE:
        I.kind = K_TRUE;
        break;
    case STL_PRED_LINEAR:
    case STL_PRED_NORM: {
        if (n.pred < 0 || n.pred >= B.n_preds) return fail(STL_E_ARG, "node %d: pred index out of range", id);
        const stl_pred& p = B.preds[n.pred];
        if (p.kind != n.op) return fail(STL_E_FORMULA, "node %d: predicate kind does not match the node op", id);
        I.kind = n.op == STL_PRED_LINEAR ? K_LIN : K_NORM;
        I.coef = (int16_t)B.coef.size();
        if (n.op == STL_PRED_LINEAR) {
            B.coef.push_back(p.c);
            for (int d = 0; d < B.D; ++d) B.coef.push_back(p.w[d]);
        } else {
            if (p.m < 1 || p.m > 4) return fail(STL_E_UNSUPPORTED, "node %d: norm predicate needs 1..4 rows", id);
            B.coef.push_back((float)p.m);
            B.coef.push_back(p.r);
            B.coef.push_back(p.sign);
            for (int i = 0; i < 4; ++i) B.coef.push_back(p.p[i]);
            for (int i = 0; i < p.m * B.D; ++i) B.coef.push_back(p.A[i]);
        }
        if ((int)B.coef.size() > MAX_COEF) return fail(STL_E_UNSUPPORTED, "too many predicate coefficients");
        if ((int)B.pred_ins.size() >= MAX_PRED) return fail(STL_E_UNSUPPORTED, "more than %d predicates", MAX_PRED);
        break;
    }
    case STL_NOT:
        I.kind = K_NOT;
        break;
    case STL_AND:
    case STL_OR: {
        I.kind = K_NARY;
        if (n.op == STL_AND) I.flags |= F_MIN;
        // more than MAX_NCH children: nest groups left to right (min/max and
        // logsumexp are associative; left nesting keeps the lowest-child tie rule)
        while ((int)kid_ins.size() > MAX_NCH) {
            Instr J = I;
            J.node = -1;
            std::vector<int> grp(kid_ins.begin(), kid_ins.begin() + MAX_NCH);
            J.nch = MAX_NCH;
            int j = B.new_instr(J, grp);
            kid_ins.erase(kid_ins.begin(), kid_ins.begin() + MAX_NCH);
            kid_ins.insert(kid_ins.begin(), j);
        }
        I.nch = (int8_t)kid_ins.size();
        break;
    }
    case STL_EVENTUALLY:
    case STL_ALWAYS:
        if (n.op == STL_ALWAYS) I.flags |= F_MIN;
        if (n.mask_param >= 0) {
            if (n.mask_param + 3 >= B.n_params) return fail(STL_E_ARG, "node %d: mask_param + 3 >= n_params", id);
            if ((int)B.mask_params.size() >= MAX_MASKS) return fail(STL_E_UNSUPPORTED, "too many smooth masks");
            I.kind = K_MASK;
            I.mask = (int8_t)n.mask_param;
            I.mslot = (int8_t)B.mask_params.size();
            B.mask_params.push_back(n.mask_param);
            if (n.mask_unbounded) I.flags |= F_MASK_UNB;
            // pads apply to bounded masks (an unbounded one reaches the end)
            if (n.pad < 0 || n.pad > 2) return fail(STL_E_ARG, "node %d: bad pad policy", id);
            I.pad = (int8_t)(n.mask_unbounded ? STL_PAD_NEUTRAL : n.pad);
            std::memcpy(&I.a, &n.pad_value, sizeof(float));
        } else {
            I.kind = K_WIN;
            if (n.a < 0 || (n.b >= 0 && n.b < n.a) || n.b < -1)
                return fail(STL_E_FORMULA, "node %d: bad interval [%d, %d]", id, n.a, n.b);
            I.a = n.a;
            I.b = n.b;
            if (n.b < 0) I.flags |= F_UNB;
            if (n.pad < 0 || n.pad > 2) return fail(STL_E_ARG, "node %d: bad pad policy", id);
            I.pad = (int8_t)n.pad;
            I.coef = (int16_t)B.coef.size();
            B.coef.push_back(n.pad_value);
        }
        break;
    case STL_UNTIL:
        I.kind = K_UNTIL;
        B.has_until = true;
        if (n.mask_param >= 0) {
            // smooth mask on the Until index: the kernels walk its support,
            // which can reach the end of the trajectory
            if (n.mask_param + 3 >= B.n_params) return fail(STL_E_ARG, "node %d: mask_param + 3 >= n_params", id);
            if ((int)B.mask_params.size() >= MAX_MASKS) return fail(STL_E_UNSUPPORTED, "too many smooth masks");
            I.mask = (int8_t)n.mask_param;
            I.mslot = (int8_t)B.mask_params.size();
            B.mask_params.push_back(n.mask_param);
            if (n.mask_unbounded) I.flags |= F_MASK_UNB;
            I.a = 0;
            I.b = -1;
            I.flags |= F_UNB;
            B.max_until_b = 1 << 30;
            break;
        }
        if (n.a < 0 || (n.b >= 0 && n.b < n.a) || n.b < -1)
            return fail(STL_E_FORMULA, "node %d: bad interval [%d, %d]", id, n.a, n.b);
        I.a = n.a;
        I.b = n.b;
        if (n.b < 0) I.flags |= F_UNB;
        B.max_until_b = std::max(B.max_until_b, n.b < 0 ? (1 << 30) : n.b);
        break;
    default:
        return fail(STL_E_FORMULA, "node %d: unknown op %d", id, n.op);
    }
    int k = B.new_instr(I, kid_ins);
    if (n.op == STL_PRED_LINEAR || n.op == STL_PRED_NORM) B.pred_ins.push_back(k);
    *out = k;
    return STL_OK;
}

int expected_children(int op, int* lo, int* hi)
{
    switch (op) {
    case STL_TRUE: case STL_PRED_LINEAR: case STL_PRED_NORM: *lo = *hi = 0; return 1;
    case STL_NOT: case STL_EVENTUALLY: case STL_ALWAYS: *lo = *hi = 1; return 1;
    case STL_UNTIL: *lo = *hi = 2; return 1;
    case STL_AND: case STL_OR: *lo = 1; *hi = STL_MAX_CHILDREN; return 1;
    default: return 0;
    }
}

// greedy slot allocation over [def, last] intervals
struct SlotAlloc {
    std::vector<int> free_at;   // per slot: first step at which it is free again
    int get(int def_step, int last_step)
    {
        for (size_t s = 0; s < free_at.size(); ++s)
            if (free_at[s] <= def_step) { free_at[s] = last_step + 1; return (int)s; }
        free_at.push_back(last_step + 1);
        return (int)free_at.size() - 1;
    }
};

}  // namespace

extern "C" stl_status stl_compile(const stl_node* nodes, int32_t n_nodes, const int32_t* child_idx,
                                  int32_t n_child_idx, int32_t root, const stl_pred* preds, int32_t n_preds,
                                  int32_t D, int32_t n_params, float rho_max, float rho_pad, stl_plan** out)
{
    if (!out) return fail(STL_E_ARG, "out is NULL");
    *out = nullptr;
    if (!nodes || n_nodes <= 0) return fail(STL_E_ARG, "empty node array");
    if (n_nodes > STL_MAX_NODES) return fail(STL_E_UNSUPPORTED, "more than %d nodes", STL_MAX_NODES);
    if (root < 0 || root >= n_nodes) return fail(STL_E_ARG, "root %d out of range", root);
    if (D < 1 || D > STL_MAX_D) return fail(STL_E_UNSUPPORTED, "D must be in [1, %d]", STL_MAX_D);
    if (n_params < 0 || n_params > 127) return fail(STL_E_UNSUPPORTED, "n_params must be in [0, 127]");
    if (n_child_idx < 0 || (n_child_idx > 0 && !child_idx)) return fail(STL_E_ARG, "bad child index array");
    if (n_preds < 0 || (n_preds > 0 && !preds)) return fail(STL_E_ARG, "bad predicate array");
    if (!(rho_max > 0) || !(rho_pad > 0)) return fail(STL_E_ARG, "rho_max and rho_pad must be > 0");
    // structure: child counts and indices, every node reachable from the root at most once
    std::vector<int> parents(n_nodes, 0);
    for (int i = 0; i < n_nodes; ++i) {
        int lo, hi;
        if (!expected_children(nodes[i].op, &lo, &hi)) return fail(STL_E_FORMULA, "node %d: unknown op %d", i, nodes[i].op);
        if (nodes[i].n_child < lo || nodes[i].n_child > hi)
            return fail(STL_E_FORMULA, "node %d: op %d takes %d..%d children, got %d", i, nodes[i].op, lo, hi,
                        nodes[i].n_child);
        if (nodes[i].n_child > 0 &&
            (nodes[i].child_off < 0 || nodes[i].child_off + nodes[i].n_child > n_child_idx))
            return fail(STL_E_FORMULA, "node %d: children outside child_idx", i);
    }
    // reachability walk (iterative) with cycle / sharing detection
    std::vector<int> stack{root};
    std::vector<int> seen(n_nodes, 0);
    seen[root] = 1;
    while (!stack.empty()) {
        int i = stack.back();
        stack.pop_back();
        for (int k = 0; k < nodes[i].n_child; ++k) {
            int c = child_idx[nodes[i].child_off + k];
            if (c < 0 || c >= n_nodes) return fail(STL_E_FORMULA, "node %d: dangling child %d", i, c);
            if (c == root || seen[c]) return fail(STL_E_FORMULA, "node %d is shared or part of a cycle (formulas are trees)", c);
            seen[c] = 1;
            stack.push_back(c);
        }
    }
    Builder B;
    B.nodes = nodes;
    B.n_nodes = n_nodes;
    B.child_idx = child_idx;
    B.n_child_idx = n_child_idx;
    B.preds = preds;
    B.n_preds = n_preds;
    B.D = D;
    B.n_params = n_params;
    int rootk;
    stl_status s = emit(B, root, 0, &rootk);
    if (s != STL_OK) return s;
    const int n = (int)B.ins.size();
    if (n > MAX_INSTR) return fail(STL_E_UNSUPPORTED, "plan has %d instructions (max %d)", n, MAX_INSTR);
    if ((int)B.coef.size() > MAX_COEF)
        return fail(STL_E_UNSUPPORTED, "predicate and pad coefficients need %d floats (max %d)", (int)B.coef.size(),
                    MAX_COEF);

    // consumers
    std::vector<int> parent(n, -1);
    for (int k = 0; k < n; ++k)
        for (int c : B.kids[k]) parent[c] = k;

    // forward slot map: value of k lives from k to its parent's step
    SlotAlloc fa;
    std::vector<int> fslot(n);
    {
        // intervals: def = k, last = parent step (root: n)
        for (int k = 0; k < n; ++k) {
            int last = parent[k] < 0 ? n : parent[k];
            fslot[k] = fa.get(k, last);
        }
    }
    // backward map: values get their own slots (kept through the adjoint sweep);
    // adjoints are allocated over the reverse sweep.  Step numbering for the
    // sweep: step of adjoint(k) = n - 1 - k; predicates' adjoints live to the
    // final d/dx stage (step n).
    SlotAlloc ga;
    std::vector<int> gslot(n, -1);
    for (int k = n - 1; k >= 0; --k) {
        int def = parent[k] < 0 ? -1 : (n - 1 - parent[k]);
        const bool pred = B.ins[k].kind == K_LIN || B.ins[k].kind == K_NORM;
        int last = pred ? n : (n - 1 - k);
        gslot[k] = ga.get(def, last);   // the parent's own slot stays busy through its step
    }
    // adjoints written by a parent must not share a slot with the parent's own
    // adjoint: the allocation above already keeps the parent's slot busy
    // through its own step (n-1-parent), and children are defined at def+1.
    const int nval = n;
    const int nadj = (int)ga.free_at.size();
    for (int k = 0; k < n; ++k) {
        Instr& I = B.ins[k];
        const auto& ch = B.kids[k];
        I.f_out = (int8_t)fslot[k];
        I.b_out = (int8_t)k;
        I.g_out = (int8_t)(nval + gslot[k]);
        if (I.kind == K_NARY) {
            for (int j = 0; j < (int)ch.size(); ++j) {
                I.f_ch[j] = (int8_t)fslot[ch[j]];
                I.b_ch[j] = (int8_t)ch[j];
                I.g_ch[j] = (int8_t)(nval + gslot[ch[j]]);
            }
        } else {
            if (ch.size() > 0) { I.f_in0 = (int8_t)fslot[ch[0]]; I.b_in0 = (int8_t)ch[0]; I.g_in0 = (int8_t)(nval + gslot[ch[0]]); }
            if (ch.size() > 1) { I.f_in1 = (int8_t)fslot[ch[1]]; I.b_in1 = (int8_t)ch[1]; I.g_in1 = (int8_t)(nval + gslot[ch[1]]); }
        }
    }
    // each smooth Until gets a slot pair in the backward map where the
    // recompute keeps its fp64 outer sums Z_t for the adjoint (index in I.coef)
    int nbwd = nval + nadj;
    for (int k = 0; k < n; ++k) {
        Instr& I = B.ins[k];
        if (I.kind != K_UNTIL) continue;
        I.coef = -1;
        if (I.flags & F_SMOOTH) {
            I.coef = (int16_t)nbwd;
            nbwd += 2;
        }
    }
    stl_plan* p = new (std::nothrow) stl_plan();
    if (!p) return fail(STL_E_ARG, "out of host memory");
    DevPlan& dp = p->dev;
    std::memset(&dp, 0, sizeof dp);
    dp.n_ins = n;
    dp.n_slots_fwd = (int)fa.free_at.size();
    dp.n_slots_bwd = nbwd;
    dp.D = D;
    dp.n_masks = (int)B.mask_params.size();
    dp.n_params = n_params;
    dp.n_pred = (int)B.pred_ins.size();
    dp.root = rootk;
    dp.rho_max = rho_max;
    dp.rho_pad = rho_pad;
    for (int i = 0; i < dp.n_pred; ++i) dp.pred_ins[i] = (int16_t)B.pred_ins[i];
    for (int i = 0; i < dp.n_masks; ++i) dp.mask_param[i] = (int8_t)B.mask_params[i];
    for (int k = 0; k < n; ++k) dp.ins[k] = B.ins[k];
    for (size_t i = 0; i < B.coef.size(); ++i) dp.coef[i] = B.coef[i];
    // fused fast path: root = smooth n-ary over <= 4 smooth-mask nodes on linear
    // predicates, or a single such mask node
    {
        auto is_fmask = [&](int k) {
            const Instr& I = B.ins[k];
            return I.kind == K_MASK && (I.flags & F_SMOOTH) && I.pad == STL_PAD_NEUTRAL && B.kids[k].size() == 1 &&
                   B.ins[B.kids[k][0]].kind == K_LIN;
        };
        FusedDesc& F = dp.fused;
        std::memset(&F, 0, sizeof F);
        const Instr& R = B.ins[rootk];
        if (is_fmask(rootk)) {
            F.n = 1;
            F.root_nary = 0;
            F.ins[0] = (int8_t)rootk;
            F.pred[0] = (int8_t)B.kids[rootk][0];
        } else if (R.kind == K_NARY && (R.flags & F_SMOOTH) && !(R.flags & F_SOFT) && B.kids[rootk].size() <= 4) {
            bool ok = true;
            for (int c : B.kids[rootk]) ok = ok && is_fmask(c);
            if (ok) {
                F.n = (int8_t)B.kids[rootk].size();
                F.root_nary = 1;
                F.nary_min = (R.flags & F_MIN) ? 1 : 0;
                F.nary_beta = R.beta;
                for (int j = 0; j < F.n; ++j) {
                    F.ins[j] = (int8_t)B.kids[rootk][j];
                    F.pred[j] = (int8_t)B.kids[B.kids[rootk][j]][0];
                }
            }
        }
    }
    // trace-output variant: slot k for instruction k (never fused)
    p->dev_trace = dp;
    std::memset(&p->dev_trace.fused, 0, sizeof(FusedDesc));
    DevPlan& tp = p->dev_trace;
    tp.n_slots_fwd = n;
    for (int k = 0; k < n; ++k) {
        Instr& I = tp.ins[k];
        I.f_out = I.b_out;
        I.f_in0 = I.b_in0;
        I.f_in1 = I.b_in1;
        for (int j = 0; j < MAX_NCH; ++j) I.f_ch[j] = I.b_ch[j];
    }
    p->n_nodes = n_nodes;
    p->n_params = n_params;
    p->D = D;
    p->max_until_b = B.max_until_b;
    p->has_until = B.has_until;
    *out = p;
    return STL_OK;
}

extern "C" stl_status stl_plan_destroy(stl_plan* plan)
{
    delete plan;
    return STL_OK;
}

extern "C" stl_status stl_plan_info(const stl_plan* plan, int32_t* n_nodes, int32_t* n_params)
{
    if (!plan) return fail(STL_E_ARG, "plan is NULL");
    if (n_nodes) *n_nodes = plan->n_nodes;
    if (n_params) *n_params = plan->n_params;
    return STL_OK;
}

extern "C" stl_status stl_lpt_order(const int64_t* host_offsets, int64_t B, int32_t* host_order)
{
    if (!host_offsets || !host_order || B < 0) return fail(STL_E_ARG, "bad arguments");
    std::vector<int32_t> idx((size_t)B);
    for (int64_t i = 0; i < B; ++i) {
        if (host_offsets[i + 1] < host_offsets[i]) return fail(STL_E_ARG, "offsets must be non-decreasing");
        idx[i] = (int32_t)i;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        return host_offsets[a + 1] - host_offsets[a] > host_offsets[b + 1] - host_offsets[b];
    });
    std::memcpy(host_order, idx.data(), sizeof(int32_t) * (size_t)B);
    return STL_OK;
}

