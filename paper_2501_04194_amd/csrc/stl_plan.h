// Internal execution-plan layout shared by the host plan compiler
// (stl_api.cpp) and the device executor (stl_kernels.hip).  Not part of the
// public ABI.
//
// A plan is a straight-line program over on-chip "slots" (one float per
// timestep of the trajectory being processed): one instruction per formula
// node, in topological order.  The forward kernel runs the instructions in
// order with the forward slot map.  The backward kernel runs them in order
// with the backward slot map (recomputing every trace the adjoints need),
// then runs the adjoint of each instruction in reverse order and finally
// writes d/dx from the predicate adjoints.  The whole program travels to
// the GPU by value as a kernel argument, so a plan needs no device memory.
#pragma once
#include <stdint.h>

namespace stlmi {

enum Kind : int8_t {
    K_TRUE = 0,
    K_LIN = 1,     // linear predicate
    K_NORM = 2,    // norm predicate
    K_NOT = 3,
    K_NARY = 4,    // and / or over up to 4 children
    K_WIN = 5,     // eventually / always over an integer interval
    K_MASK = 6,    // eventually / always with the smooth time mask
    K_UNTIL = 7
};

enum Flag : int8_t {
    F_SMOOTH = 1,
    F_MIN = 2,        // min-type (and, always): evaluated as max on negated values
    F_UNB = 4,        // unbounded integer interval
    F_MASK_UNB = 8,   // smooth mask with b = +inf
    F_SOFT = 16       // smooth form is the softmax-weighted mean (Sec. III-C), not logsumexp
};

constexpr int MAX_INSTR = 48;
constexpr int MAX_COEF = 160;
constexpr int MAX_NCH = 4;
constexpr int MAX_PRED = 32;
constexpr int MAX_MASKS = 16;
constexpr int MAX_D = 16;

struct Instr {                  // 40 bytes
    int8_t kind, flags, nch, pad;
    int8_t f_out, f_in0, f_in1;             // forward slot map
    int8_t b_out, b_in0, b_in1;             // backward slot map (values)
    int8_t g_out, g_in0, g_in1;             // backward slot map (adjoints)
    int8_t beta;                            // parameter index of beta (smooth), -1
    int8_t mask;                            // parameter index of (a,b,c,eps), -1
    int8_t mslot;                           // index of this mask in the d/da,d/db partials
    int8_t f_ch[MAX_NCH], b_ch[MAX_NCH], g_ch[MAX_NCH];
    int16_t node;                           // caller's node index (trace output), -1
    int16_t coef;                           // predicate / pad-value offset into coef[]
    int32_t a, b;                           // integer interval (b < 0: unbounded); K_MASK:
                                            // a = bits of the pad value (no interval)
};
static_assert(sizeof(Instr) == 40, "Instr layout");

// Fused fast path (set by the plan compiler when the formula has the shape
// root = smooth And/Or over up to 4 smooth-mask Eventually/Always nodes, each
// over a linear predicate, or a single such mask node): one kernel computes
// the whole formula per trajectory with fp64 accumulation.
struct FusedDesc {
    int8_t n;                               // number of mask nodes (0: no fused path)
    int8_t root_nary;                       // 1: root is the n-ary node, 0: root is the mask node
    int8_t nary_min;                        // the n-ary node is an And
    int8_t nary_beta;                       // its beta parameter index
    int8_t ins[4];                          // instruction index of each mask node
    int8_t pred[4];                         // instruction index of its linear predicate
};

struct DevPlan {
    int32_t n_ins;
    int32_t n_slots_fwd;
    int32_t n_slots_bwd;
    int32_t D;
    int32_t n_masks;
    int32_t n_params;
    int32_t n_pred;
    int32_t root;                           // instruction index of the root
    float rho_max;
    float rho_pad;
    int16_t pred_ins[MAX_PRED];             // instruction index of each predicate
    int8_t mask_param[MAX_MASKS];           // parameter index of each learnable mask
    FusedDesc fused;
    Instr ins[MAX_INSTR];
    float coef[MAX_COEF];
};

// Predicate coefficient layout in coef[] at offset o:
//   linear: [0] c, [1 .. 1+D) w
//   norm:   [0] m, [1] r, [2] sign, [3..7) p, [7 .. 7+m*D) A (row-major)

// Launch arguments shared by the host launchers and the kernels.
struct MaskTab;

struct Batch {
    const float* x;
    const int64_t* offsets;
    const int32_t* order;
    int64_t B;
    int64_t T;
    int32_t D;
    int32_t Lcap;      // slot capacity (floats per slot)
};

struct KArgs {
    const float* params;
    float* root;           // forward: [N_total]
    float* nodes;          // forward: [n_nodes][N_total] or NULL
    int64_t n_total;
    const float* G;        // backward: upstream gradient [N_total]
    float* dx;             // backward: [N_total, D]
    float* mask_part;      // backward: [B][n_masks][2]
    float* garena;         // global slot arenas (NULL: LDS)
    int64_t arena_floats;  // floats per arena (slots + scratch)
    int* counter;          // persistent scheduler counter
    int persistent;
    int* list_count;       // fused path: number of trajectories sent to the generic executor
    int* list;             // fused path: their indices
    int list_mode;         // generic executor processes list[0 .. *list_count)
    const MaskTab* tabs;   // fused path: per-mask tables (workspace)
    float* saved;          // fused forward: mask-node traces out ([n][B][T]) or NULL
    const float* saved_in; // fused backward: mask-node traces in, or NULL (recompute)
    int* saved_flag;       // [B]: 1 where the saved traces of a trajectory are valid
    const int* scan;       // [B] or NULL: the generic executor takes the trajectories whose flag is set
    int part_stride;       // rows of mask_part per trajectory (1; a caller with more rows per
                           // trajectory has the generic executor clear the others)
};

// Launch arguments of the matrix-core smooth-mask kernels (stl_mx.h).
struct MxHead;
struct MxArgs {
    MxHead* heads;         // [n] per-mask geometry: written by the forward, read by the backward (NULL: derive)
    int moff[2];           // per mask (at most two): offset of its window parameters a, b, c, eps in params
    int munb[2];           //   and whether the window is unbounded (read here, not through the plan)
    int* handed;           // [B] written by every call: 1 where the generic executor takes the trajectory
    int* ranges;           // [B][n][3] floor(min), ceil(max) of O over each trajectory's trace, reference R
    float* part;           // [B][n_masks][2] d/da, d/db partials
};

}  // namespace stlmi
