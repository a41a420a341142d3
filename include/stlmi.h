/*
 * stlmi.h -- C ABI of the MI355X (gfx950) STL robustness library.
 *
 * The library evaluates robustness traces of Signal Temporal Logic formulas
 * over batches of trajectories, and their gradients, on the GPU, following
 * the masking formulation of arXiv 2501.04194 ("STLCG++"):
 *
 *   robustness (quantitative semantics) ....... Sec. III-B, eq. (quantitative)
 *   derived Or / Eventually / Always ........... Sec. III-B (after the grammar)
 *   logsumexp smooth max / min ................ Sec. III-C
 *   robustness trace (one value per suffix) ... Sec. III-D, Definition 1
 *   Eventually / Always over [a,b] ............ Sec. IV-B
 *   Until over [a,b] .......................... Sec. IV-C
 *   smooth (sigmoid) time-interval mask ....... Sec. VI, eq. (smooth mask)
 *
 * Conventions shared by every entry point:
 *  - A trajectory of length L has samples 0..L-1; its robustness trace has L
 *    values, value t being the robustness of the suffix starting at t.
 *  - Intervals [a,b] are inclusive offsets in timesteps (b = -1: unbounded,
 *    i.e. up to the last sample).
 *  - Smooth operators use beta = 1/temperature inside the exponent:
 *    smax(V) = (1/beta) log sum exp(beta v), smin(V) = -smax(-V).
 *  - Window positions past the end of a trajectory follow the node's pad
 *    policy (STL_PAD_NEUTRAL drops them; an empty window yields -rho_pad for
 *    Eventually/Or/Until and +rho_pad for Always/And).
 *  - Smooth-mask nodes weight the terms of the logsumexp by
 *    w_k = max(sig(c(k-a)) - sig(c(k-b)) - eps, 0), k = offset >= 0, with
 *    a, b, c, eps read from the device parameter buffer at run time (so they
 *    can be learned or annealed without recompiling the plan).  Their hard
 *    variant takes max/min over the support {k : w_k > 0}.  On Until the
 *    mask weights the Until index i (the psi index) in the outer smooth max;
 *    the running min of phi over [0, i] is unweighted.  On a bounded mask,
 *    STL_PAD_LAST / STL_PAD_CONST give every support offset past the end one
 *    pad copy weighted by w_k (offsets more than 65536 past the end are not
 *    visited; w_k is below eps there unless c is tiny).
 *  - Hard min/max break ties toward the lowest time index (and the lowest
 *    child index for n-ary And/Or; the phi side inside Until's min).
 *
 * Memory and ownership:
 *  - A plan (stl_plan) is opaque, host-resident and immutable after
 *    stl_compile; free it with stl_plan_destroy.  Concurrent calls sharing a
 *    plan are safe if they use distinct workspaces.
 *  - Every array passed to stl_forward / stl_backward is caller-owned device
 *    memory on the current HIP device.  The library never allocates device
 *    memory, never synchronises and launches only on the given stream, so
 *    both calls can be captured in a HIP graph.
 *  - Arguments are validated on the host before any launch; a failure
 *    returns a negative stl_status and sets a thread-local message readable
 *    with stl_last_error().  No call aborts or throws.
 */
#ifndef STLMI_H
#define STLMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STL_OK = 0,
    STL_E_ARG = -1,          /* null pointer, out-of-range index or size */
    STL_E_FORMULA = -2,      /* malformed node array (cycle, dangling child, bad interval) */
    STL_E_UNSUPPORTED = -3,  /* valid formula outside the library's limits */
    STL_E_SHAPE = -4,        /* batch shape inconsistent with the plan */
    STL_E_WORKSPACE = -5,    /* workspace too small */
    STL_E_HIP = -6,          /* a HIP runtime call or kernel launch failed */
    STL_E_NONFINITE = -7     /* reserved: non-finite input detected */
} stl_status;

typedef enum {
    STL_TRUE = 0,            /* constant rho_max (Sec. III-B) */
    STL_PRED_LINEAR = 1,     /* w . x_t - c (Sec. III-A/B, mu(x) - c) */
    STL_PRED_NORM = 2,       /* sign * (||A x_t - p||_2 - r); gradient 0 where A x_t = p */
    STL_NOT = 3,             /* -u_t */
    STL_AND = 4,             /* min / smin over children at the same t */
    STL_OR = 5,              /* max / smax over children at the same t */
    STL_EVENTUALLY = 6,      /* max / smax of the child over the window [t+a, t+b] */
    STL_ALWAYS = 7,          /* min / smin of the child over the window [t+a, t+b] */
    STL_UNTIL = 8            /* max_{i in [a,b]} min(min_{k<=i} phi_{t+k}, psi_{t+i}) */
} stl_op;

typedef enum {
    STL_PAD_NEUTRAL = 0,     /* positions past the end are dropped */
    STL_PAD_LAST = 1,        /* positions past the end read u[L-1] */
    STL_PAD_CONST = 2        /* positions past the end read pad_value */
} stl_pad;

#define STL_MAX_CHILDREN 8
#define STL_MAX_D 16
#define STL_MAX_NODES 48
#define STL_MAX_PREDS 32

/* One formula node.  Children are child_idx[child_off .. child_off+n_child). */
typedef struct {
    int32_t op;              /* stl_op */
    int32_t n_child;         /* NOT/EVENTUALLY/ALWAYS: 1, UNTIL: 2 (phi, psi), AND/OR: 1..8 */
    int32_t child_off;
    int32_t smooth;          /* 0: hard min/max, 1: logsumexp, 2: softmax-weighted mean
                                sum v e^{beta v} / sum e^{beta v} (Sec. III-C): And/Or with
                                up to 4 children and unmasked Eventually/Always only
                                (else STL_E_UNSUPPORTED) */
    int32_t a, b;            /* integer interval (temporal nodes); b = -1: unbounded */
    int32_t mask_param;      /* -1: integer interval; else params[mask_param + 0..3] = (a, b, c, eps) */
    int32_t mask_unbounded;  /* smooth mask with b = +inf (params[mask_param+1] ignored) */
    int32_t beta_param;      /* smooth nodes: index of beta in params; ignored when hard */
    int32_t pred;            /* PRED_*: index into the predicate array */
    int32_t pad;             /* stl_pad (EVENTUALLY / ALWAYS; ignored by unbounded windows) */
    float pad_value;         /* STL_PAD_CONST value */
} stl_node;

/* A predicate mu(x_t) evaluated on the D-dimensional state. */
typedef struct {
    int32_t kind;            /* STL_PRED_LINEAR or STL_PRED_NORM */
    int32_t m;               /* NORM: number of rows of A (1..4) */
    float w[STL_MAX_D];      /* LINEAR: weights */
    float c;                 /* LINEAR: offset */
    float A[4 * STL_MAX_D];  /* NORM: A, m x D row-major */
    float p[4];              /* NORM: centre */
    float r;                 /* NORM: radius */
    float sign;              /* NORM: +1 or -1 */
} stl_pred;

/* A batch of trajectories in device memory. */
typedef struct {
    const float* x;          /* dense: [B, T, D]; ragged: [N_total, D] (rows of trajectory b are
                                offsets[b] .. offsets[b+1]-1) */
    int64_t B;               /* number of trajectories */
    int64_t T;               /* dense: length of every trajectory; ragged: upper bound on the
                                lengths (sizes on-chip buffers; longer trajectories get NaN) */
    int32_t D;               /* state dimension, must equal the plan's */
    int32_t pad0;
    const int64_t* offsets;  /* device int64[B+1]; NULL for a dense batch */
    const int32_t* order;    /* device int32[B]: processing order of the persistent scheduler
                                (e.g. from stl_lpt_order); NULL = 0..B-1 */
} stl_batch;

/* Launch configuration (NULL = library heuristic; see stl_autotune). */
typedef struct {
    int32_t threads;         /* work-group size of the generic executor: 64, 128, 256 or 512 */
    int32_t wg_per_cu;       /* persistent grid size per compute unit (0 = one work-group per
                                trajectory) */
    int32_t global_slots;    /* 1: keep node traces in the workspace instead of LDS */
    int32_t flags;           /* bit 0: generic executor only (no fused path); bit 1: the fp64 fused
                                kernels instead of the matrix-core path (see stl_forward) */
} stl_launch;

typedef struct stl_plan stl_plan;

/*
 * Compile a formula (post-order not required; `root` names the top node)
 * into an execution plan: the bottom-up composition of the formula graph
 * (Sec. III-E, Fig. 2), each node an operator of Sec. III-B / III-C, IV-B,
 * IV-C or VI.  Host only: validates the node array (op codes,
 * child counts and indices, acyclicity, intervals, predicate and parameter
 * indices against n_params), orders nodes topologically, assigns on-chip
 * trace slots by liveness and records the parameter layout.  rho_max is the
 * value of STL_TRUE, rho_pad the magnitude of the empty-window value.
 * Several smooth-mask nodes may name the same (or overlapping) parameter
 * slots (tied bounds): their d/da, d/db are summed into the shared entries.
 * Returns STL_OK and *out, or STL_E_ARG / STL_E_FORMULA / STL_E_UNSUPPORTED.
 */
stl_status stl_compile(const stl_node* nodes, int32_t n_nodes, const int32_t* child_idx,
                       int32_t n_child_idx, int32_t root, const stl_pred* preds, int32_t n_preds,
                       int32_t D, int32_t n_params, float rho_max, float rho_pad, stl_plan** out);

/* Free a plan (NULL is accepted). */
stl_status stl_plan_destroy(stl_plan* plan);

/* Number of formula nodes and parameters the plan was compiled with. */
stl_status stl_plan_info(const stl_plan* plan, int32_t* n_nodes, int32_t* n_params);

/*
 * Device workspace needed by stl_forward and stl_backward for this batch and
 * launch configuration (NULL = heuristic).  Sizes are in bytes.
 */
stl_status stl_workspace_size(const stl_plan* plan, const stl_batch* batch, const stl_launch* cfg,
                              size_t* fwd_bytes, size_t* bwd_bytes);

/*
 * Fused fast paths, for a formula that is a smooth And/Or over up to 4
 * smooth-mask Eventually/Always nodes on linear predicates (or one such
 * node) and a dense batch:
 *  - matrix-core path (one or two bounded masks, D <= 2, any T): the masked
 *    logsumexp windows of Sec. VI as products of Toeplitz weight tiles and
 *    the terms 2^{z - R} on the bf16 matrix cores (each factor split into
 *    two bf16 parts, three products, fp32 accumulation: relative error a few
 *    2^-18 at worst per window sum, far less on average); trajectories whose
 *    exponent range over a chunk of outputs exceeds 200 (log2 units), and
 *    masks wider than the kernel's tiles, go to the generic executor in the
 *    same call;
 *  - otherwise fp64 fused kernels (T <= 2048; one work-group per
 *    trajectory; signal ranges beyond fp64 exponents and mask bands wider
 *    than 512 steps go to the generic executor).  Results agree with the
 *    generic executor to float32 rounding.
 *
 * Robustness traces (Sec. III-D, Definition 1: value t is the robustness of
 * the suffix starting at t), evaluated bottom-up over the plan with the
 * windowed operators of Sec. IV-B / IV-C and the masks of Sec. VI:
 * d_root receives the root trace ([B, T] dense or
 * [N_total] ragged, float32).  d_node_traces, if not NULL, receives every
 * node's trace as [n_nodes][N_total] in the caller's node numbering (debug and
 * tests).  d_params holds the plan's n_params float32 scalars (beta of smooth
 * nodes, (a, b, c, eps) of smooth masks).  Asynchronous on `stream`
 * (a hipStream_t; NULL = default stream).
 */
stl_status stl_forward(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                       float* d_root, float* d_node_traces, void* d_ws, size_t ws_bytes,
                       const stl_launch* cfg, void* stream);

/*
 * Reverse mode through the same plan (the gradients the paper obtains by
 * automatic differentiation of Sec. IV-B / IV-C and of the mask of Sec. VI,
 * here written out per operator): gradients of sum_t G_t * root_t.
 * d_grad_root has the layout of d_root.  d_grad_x (same layout as x) is
 * overwritten; d_grad_params (n_params floats, may be NULL) is overwritten
 * with d/da and d/db of every smooth-mask bound and 0 elsewhere.  The
 * forward node traces are recomputed on chip, not stored.
 */
stl_status stl_backward(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                        const float* d_grad_root, float* d_grad_x, float* d_grad_params,
                        void* d_ws, size_t ws_bytes, const stl_launch* cfg, void* stream);

/*
 * Forward/backward with saved mask-node traces.  The backward of a smooth
 * n-ary root needs every child's trace (Sec. III-C: the logsumexp adjoint
 * weights each child by its softmax share); stl_backward recomputes them on
 * chip, these variants keep them in HBM between the two calls instead
 * (the usual saved-for-backward of an autograd function).
 *
 * stl_saved_size: bytes of the caller-owned device buffer `d_saved` for this
 * batch: a header of B int32 validity flags (padded to 256 bytes) followed by
 * [n_mask][B][T] float32 values when a fused fast path applies (n_mask = the
 * number of smooth-mask children of the root: the fp64 kernels keep the
 * children's traces, the matrix-core kernels log2 of each child's softmax
 * weight at the root minus log2 of its window sum), and for the matrix-core
 * path each trajectory's exponent range and reference ([B][n_mask][3]
 * int32, the total padded to 256 bytes) and 256 bytes of the masks' window
 * geometry; only the header otherwise.  The
 * contents are private to the pair; stl_backward_saved only reads them.
 * A flag is 1 (fp64 fused forward) or 2 (matrix-core forward) where the
 * trajectory's saved data are valid for the backward of the same path.
 *
 * stl_forward_saving: stl_forward that also fills d_saved (saved_bytes must
 * be at least stl_saved_size).  Trajectories the fused kernel does not take
 * are flagged 0 and recomputed by the backward.
 *
 * stl_backward_saved: stl_backward that reads d_saved written by
 * stl_forward_saving with the same plan, batch contents and parameters (the
 * caller guarantees this; the traces are not checked against x).  Results are
 * those of stl_backward to float32 rounding.  Errors as stl_forward.
 */
stl_status stl_saved_size(const stl_plan* plan, const stl_batch* batch, size_t* saved_bytes);
stl_status stl_forward_saving(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                              float* d_root, void* d_saved, size_t saved_bytes, void* d_ws,
                              size_t ws_bytes, const stl_launch* cfg, void* stream);
stl_status stl_backward_saved(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                              const void* d_saved, size_t saved_bytes, const float* d_grad_root,
                              float* d_grad_x, float* d_grad_params, void* d_ws, size_t ws_bytes,
                              const stl_launch* cfg, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): stl_forward
 * whose workspace is a fixed device array inside the library instead of a
 * d_ws argument.  The array holds STL_STATIC_WS_BYTES; each GPU the library
 * runs on keeps its own copy until the process ends.  The call allocates
 * nothing.  A batch whose forward workspace (stl_workspace_size) exceeds the
 * array returns STL_E_WORKSPACE before any launch.  Every call on one GPU
 * shares that GPU's copy, which keeps the previous call's contents (every
 * call writes all the flags and counters it reads): calls that overlap on
 * one GPU, from several streams or host threads, race and must be
 * serialised by the caller.  Results equal stl_forward's bit for bit.
 */
#define STL_STATIC_WS_BYTES ((size_t)16 << 20)
stl_status stl_forward_static(const stl_plan* plan, const stl_batch* batch, const float* d_params, float* d_root,
                              float* d_node_traces, const stl_launch* cfg, void* stream);

/* Message describing the last non-OK status returned on this thread. */
const char* stl_last_error(void);

/*
 * Longest-processing-time order for a ragged batch: host_order[0..B) lists
 * trajectory indices by decreasing length (ties by index), for
 * stl_batch.order.  host_offsets is the host copy of the offsets.
 */
stl_status stl_lpt_order(const int64_t* host_offsets, int64_t B, int32_t* host_order);

/*
 * Time the candidate launch configurations on this batch (forward +
 * backward, on `stream`) and return the fastest in *best (and its time in
 * milliseconds).  Results are cached in memory per (plan, shape) and, when
 * the STLMI_TUNE_CACHE environment variable names a file, in that JSON file.
 * Every candidate computes the same result.  d_ws must be at least the
 * largest workspace of any candidate (stl_workspace_size with cfg = NULL
 * times 2 is enough).
 */
stl_status stl_autotune(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                        float* d_root, const float* d_grad_root, float* d_grad_x,
                        float* d_grad_params, void* d_ws, size_t ws_bytes, void* stream,
                        stl_launch* best, float* best_ms);

/*
 * Capture stl_forward followed by stl_backward (same arguments) into a HIP
 * graph and instantiate it.  Replays read the current contents of every
 * buffer, so new inputs or parameters need no re-capture; a new shape, plan
 * or buffer address does.  The returned handle is freed by stl_graph_destroy.
 */
typedef struct stl_graph stl_graph;
stl_status stl_graph_capture(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                             float* d_root, const float* d_grad_root, float* d_grad_x,
                             float* d_grad_params, void* d_ws, size_t ws_bytes,
                             const stl_launch* cfg, void* stream, stl_graph** out);
stl_status stl_graph_launch(stl_graph* graph, void* stream);
stl_status stl_graph_destroy(stl_graph* graph);

/*
 * Interval-vectorised evaluation (Sec. VI, after eq. (smooth mask): with the
 * masking form, the robustness of one formula for many time-interval
 * values is a batch of independent masked reductions).  For every
 * trajectory b and every interval n it computes the robustness at t = 0 of
 *
 *     op_{mask(a_n, b_n)} (w . x_t - c)        op = STL_ALWAYS or STL_EVENTUALLY
 *
 * where the smooth mask weights offset k by
 * w_k = max(sig(c_mask (k - a_n)) - sig(c_mask (k - b_n)) - eps, 0) (a_n, b_n
 * in timesteps: a_n = a_frac * T for the paper's fractional form).  Smooth:
 * rho = smax_w / smin_w of the trace with weights inside the logsumexp
 * (beta = 1/temperature); hard: max / min over the support {k : w_k > 0}.
 * An interval whose support misses [0, T) yields -rho_pad (Eventually) or
 * +rho_pad (Always).
 *
 * Arguments (device pointers unless noted, all caller-owned):
 *   desc       host struct below; w[0..D) are read from it
 *   d_x        [B][T][D] float32, D innermost
 *   d_a, d_b   [N] float32 interval bounds in timesteps (b > a not required)
 *   d_rho      [B][N] float32 output
 *   d_grad_a, d_grad_b   [B][N] float32 d rho / d a_n, d rho / d b_n, or NULL
 *              (both or neither; zero for the hard variant)
 *   stream     hipStream_t; the call launches one kernel on it and allocates
 *              nothing, so it can be captured in a HIP graph.
 * Limits: 1 <= T <= 4096, 1 <= D <= 16, B, N >= 0, mask_c > 0, mask_eps >= 0,
 * beta > 0 when smooth; otherwise STL_E_ARG / STL_E_SHAPE.  The smooth sums
 * use FP64 terms against the trajectory's largest exponent, and an interval
 * whose support terms all underflow against it is summed again against its
 * own largest exponent.
 */
typedef struct {
    int32_t op;              /* STL_ALWAYS or STL_EVENTUALLY */
    int32_t smooth;          /* 0 hard, 1 logsumexp */
    float beta;              /* smooth only */
    float mask_c, mask_eps;  /* sigmoid steepness (> 0) and tolerance (>= 0) */
    int32_t D;
    float w[16];             /* predicate w . x - c */
    float c;
    float rho_pad;           /* empty-support value magnitude (e.g. 1e6) */
} stl_interval_desc;

stl_status stl_interval_sweep(const stl_interval_desc* desc, const float* d_x, int64_t B, int64_t T,
                              const float* d_a, const float* d_b, int64_t N, float* d_rho, float* d_grad_a,
                              float* d_grad_b, void* stream);

/*
 * Parametric-STL mining by gradient descent over the time interval (Sec. VII-B,
 * the pSTL problem): minimise
 *
 *     L(a, b) = (1/B) sum_i max(-rho_i, 0) + gamma (a - b),
 *     rho_i = robustness at t = 0 of op_{mask(aT, bT)}(w . x_i - c)
 *
 * over a = sig(p_a), b = sig(p_b) (fractions of the horizon T), for `steps`
 * steps of p -= lr dL/dp, with the mask steepness and beta annealed from
 * (c0, beta0) to (c1, beta1) along the sigmoid schedule
 * v_k = v0 + (v1 - v0) / (1 + exp(-12 (k/(steps-1) - 1/2))).
 * The loop runs on the GPU in one launch.
 *
 * Arguments: desc (op, w, c, mask_eps are used; beta and mask_c are taken
 * from the schedules), d_x [B][T][D] float32, d_logits [2] float32 device
 * (p_a, p_b) read and overwritten, d_loss [steps] float32 device (the loss
 * at each step before its update) or NULL, stream.  Limits: 1 <= T <= 1024,
 * B >= 1, B * T <= 12288, steps >= 0, c0, c1, beta0, beta1 > 0; otherwise
 * STL_E_ARG / STL_E_SHAPE.  Allocates nothing.
 */
stl_status stl_pstl_descent(const stl_interval_desc* desc, const float* d_x, int64_t B, int64_t T, float c0,
                            float c1, float beta0, float beta1, int32_t steps, float lr, float gamma,
                            float* d_logits, float* d_loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STLMI_H */
