// C ABI of the STL robustness library: plan compiler, validation, launch
// configuration, persistent scheduling order, autotuner and HIP-graph
// capture.  Kernels live in stl_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/stlmi.h"
#include "stl_plan.h"

namespace stlmi {
size_t scratch_floats(int Lc, int nt, int max_until_b);
hipError_t launch_exec(bool bwd, const DevPlan& plan, const struct Batch& bt, const struct KArgs& ka, int grid,
                       int nt, size_t lds_bytes, hipStream_t s);
hipError_t set_max_lds(size_t bytes);
hipError_t launch_zero_counter(int* c, hipStream_t s);
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t s);
hipError_t launch_reduce_params(const float* part, int64_t B, const DevPlan& plan, float* gp, hipStream_t s);
size_t fused_lds(int Lc, int n, int D, bool bwd);
int fused_max_T();
hipError_t launch_fused(bool bwd, const DevPlan& plan, const struct Batch& bt, const struct KArgs& ka, size_t lds,
                        hipStream_t s);
hipError_t set_max_lds_fused(size_t bytes);
size_t mask_tab_bytes();
size_t mx_lds_bytes(int n, int D, bool bwd);
size_t mx_static_lds();
hipError_t set_max_lds_mx(size_t bytes);
hipError_t launch_mx(bool bwd, const DevPlan& plan, const struct Batch& bt, const struct KArgs& ka,
                     const struct MxArgs& mx, size_t lds, hipStream_t s);
int interval_max_T();
int pstl_max_BT();
hipError_t launch_pstl_descent(const float* x, int B, int T, int D, const float* w, float c, int op_sg, float eps,
                               float c0, float c1, float beta0, float beta1, int steps, float lr, float gamma,
                               float* p, float* loss, hipStream_t s);
hipError_t launch_interval_sweep(int op_sg, int smooth, float beta, float mc, float meps, int D, const float* w,
                                 float c, float rho_pad, const float* x, int64_t B, int T, const float* a,
                                 const float* b, int64_t N, float* rho, float* ga, float* gb, hipStream_t s);

}  // namespace stlmi

using namespace stlmi;

#include "stl_host.h"

// ------------------------------------------------------------------ launch geometry

namespace {

struct DevInfo {
    int cus = 256;
    size_t lds_max = 65536;
    size_t lds_mx = 0;
    bool lds_set = false;
};

std::mutex g_mu;
std::map<int, DevInfo> g_dev;

DevInfo& devinfo()
{
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) return it->second;
    DevInfo di;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) di.cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        di.lds_max = (size_t)v;
    const size_t static_lds = 8192;   // Shared struct + headroom
    di.lds_max = di.lds_max > static_lds ? di.lds_max - static_lds : 0;
    if (set_max_lds(di.lds_max) == hipSuccess) di.lds_set = true;
    (void)set_max_lds_fused(di.lds_max);
    // the matrix-core kernels' static LDS is small and known: they may use the rest
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        di.lds_mx = (size_t)v > mx_static_lds() + 1024 ? (size_t)v - mx_static_lds() - 1024 : 0;
    (void)set_max_lds_mx(di.lds_mx);
    (void)hipGetLastError();
    return g_dev[dev] = di;
}

struct Geom {
    int nt;
    int grid;
    int persistent;
    int Lc;
    bool global;
    size_t arena_floats;
    size_t lds_bytes;
    size_t ws_bytes;        // total workspace
    size_t off_part;        // mask partials (bytes)
    size_t off_arena;       // global arenas (bytes)
    bool fused;             // fused fast path (dense batches of the fused formula shape)
    size_t fused_lds;
    size_t off_list;        // fused: fix-up list (bytes)
    size_t off_tabs;        // fused: per-mask tables (bytes)
    // matrix-core path (replaces the fused kernels where it applies)
    bool mx;
    size_t mx_lds;
    size_t off_handed;      // [B] int
    size_t off_mxtr;        // backward without saved traces: [n][B][T] traces, [B] flags, ranges
    size_t off_mxflag;
    size_t off_mxrange;
    size_t off_mxheads;     // matrix-core forward: per-mask geometry for the backward
};

// The matrix-core path takes dense batches of a root that is a smooth
// And/Or over one or two bounded smooth-mask nodes on linear predicates (or
// one such node), D <= 2, unless the launch asks for another path (flags bit
// 0: generic executor only, bit 1: the fp64 fused kernels).
static bool mx_applies(const DevPlan& dp, const stl_batch* bt, const stl_launch* cfg, bool trace)
{
    if (dp.fused.n < 1 || dp.fused.n > 2 || trace || bt->offsets != nullptr || bt->D > 2) return false;
    if (cfg && (cfg->flags & 3)) return false;
    for (int m = 0; m < dp.fused.n; ++m)
        if (dp.ins[dp.fused.ins[m]].flags & F_MASK_UNB) return false;
    return true;
}

stl_status geometry(const stl_plan* plan, const stl_batch* bt, const stl_launch* cfg, bool bwd, bool trace,
                    Geom* g)
{
    DevInfo& di = devinfo();
    const DevPlan& dp = trace ? plan->dev_trace : plan->dev;
    int nt = cfg && cfg->threads ? cfg->threads : 256;
    if (nt != 64 && nt != 128 && nt != 256 && nt != 512) return fail(STL_E_ARG, "threads must be 64, 128, 256 or 512");
    if (bt->T < 1 || bt->T > (1 << 24)) return fail(STL_E_SHAPE, "T must be in [1, 2^24]");
    int Lc = (int)((bt->T + 3) / 4 * 4);
    const int nslots = bwd ? dp.n_slots_bwd : dp.n_slots_fwd;
    const int ub = plan->has_until ? (int)std::min<int64_t>(plan->max_until_b, bt->T) : 0;
    size_t arena = (size_t)nslots * Lc + scratch_floats(Lc, nt, ub);
    size_t lds = arena * sizeof(float);
    bool global = (cfg && cfg->global_slots) || lds > di.lds_max;
    if (!(cfg && cfg->threads) && bt->B < di.cus) {
        // fewer trajectories than compute units (one work-group each): size
        // the work-group to the trajectory (measured on MI355X: 64 threads
        // for T <= 64, 128 up to 128, 256 up to 256, 512 beyond), but keep
        // 256 where the larger Until checkpoint area of 512 threads would
        // push the arena out of LDS
        const int want = bt->T <= 64 ? 64 : bt->T <= 128 ? 128 : bt->T <= 256 ? 256 : 512;
        const size_t a2 = (size_t)nslots * Lc + scratch_floats(Lc, want, ub);
        const bool g2 = (cfg && cfg->global_slots) || a2 * sizeof(float) > di.lds_max;
        if (want < 256 || g2 == global) {
            nt = want;
            arena = a2;
            lds = a2 * sizeof(float);
            global = g2;
        }
    }
    int persistent = cfg ? (cfg->wg_per_cu > 0) : 0;
    int grid;
    if (global) {
        int per_cu = cfg && cfg->wg_per_cu > 0 ? cfg->wg_per_cu : 4;
        persistent = 1;
        grid = di.cus * per_cu;
    } else if (persistent) {
        grid = di.cus * cfg->wg_per_cu;
    } else {
        grid = (int)std::min<int64_t>(bt->B, 1 << 30);
    }
    if (persistent && grid > bt->B) grid = (int)std::max<int64_t>(1, bt->B);
    g->nt = nt;
    g->grid = std::max(grid, 1);
    g->persistent = persistent;
    g->Lc = Lc;
    g->global = global;
    g->arena_floats = arena;
    g->lds_bytes = global ? 0 : lds;
    g->mx = false;
    g->mx_lds = 0;
    g->off_handed = g->off_mxtr = g->off_mxflag = g->off_mxrange = g->off_mxheads = 0;
    if (mx_applies(dp, bt, cfg, trace)) {
        // (a backward without saved traces runs the forward kernel first, with the same LDS size)
        const size_t lds = bwd ? std::max(mx_lds_bytes(dp.fused.n, bt->D, false), mx_lds_bytes(dp.fused.n, bt->D, true))
                               : mx_lds_bytes(dp.fused.n, bt->D, false);
        if (lds <= di.lds_mx) {
            g->mx = true;
            g->mx_lds = lds;
        }
    }
    const int64_t prow = 1;     // partial rows per trajectory
    size_t off = 256;   // counter
    g->off_part = off;
    if (bwd) off += (size_t)bt->B * prow * std::max(dp.n_masks, 1) * 2 * sizeof(float);
    off = (off + 255) / 256 * 256;
    g->off_arena = off;
    g->fused = false;
    g->fused_lds = 0;
    g->off_list = 0;
    g->off_tabs = 0;
    if (g->mx) {
        // fix-up grid of the generic executor (it takes the trajectories whose
        // hand-off flag is set), hand-off flags
        g->persistent = 0;
        g->grid = (int)std::max<int64_t>(1, std::min<int64_t>(bt->B, di.cus / 4));
        g->off_handed = off;
        off += (size_t)bt->B * sizeof(int);
        off = (off + 255) / 256 * 256;
        g->off_mxheads = off;
        off += 256;
        if (bwd) {
            // the backward without saved traces first runs the forward into these
            g->off_mxtr = off;
            off += (size_t)dp.fused.n * bt->B * bt->T * sizeof(float);
            off = (off + 255) / 256 * 256;
            g->off_mxflag = off;
            off += (size_t)bt->B * sizeof(int);
            off = (off + 255) / 256 * 256;
            g->off_mxrange = off;
            off += (size_t)bt->B * dp.fused.n * 3 * sizeof(int);
            off = (off + 255) / 256 * 256;
        }
        g->off_arena = off;
    }
    const bool want_fused = !g->mx && dp.fused.n > 0 && !trace && bt->offsets == nullptr &&
                            bt->T <= fused_max_T() && !(cfg && (cfg->flags & 1));
    if (want_fused) {
        const size_t fl = fused_lds((int)((bt->T + 3) / 4 * 4), dp.fused.n, bt->D, bwd);
        if (fl <= di.lds_max) {
            g->fused = true;
            g->fused_lds = fl;
            // the generic executor handles the fix-up list with a small persistent grid
            if (!global) {
                g->persistent = 1;
                g->grid = (int)std::max<int64_t>(1, std::min<int64_t>(bt->B, di.cus / 4));
            } else {
                g->grid = (int)std::max<int64_t>(1, std::min<int64_t>(bt->B, di.cus / 4));
            }
            g->off_list = off;
            off += (size_t)bt->B * sizeof(int);
            off = (off + 255) / 256 * 256;
            g->off_tabs = off;
            off += (size_t)dp.fused.n * mask_tab_bytes();
            off = (off + 255) / 256 * 256;
            g->off_arena = off;
        }
    }
    if (global) off += (size_t)g->grid * arena * sizeof(float);
    g->ws_bytes = off;
    return STL_OK;
}

stl_status check_batch(const stl_plan* plan, const stl_batch* bt)
{
    if (!plan) return fail(STL_E_ARG, "plan is NULL");
    if (!bt) return fail(STL_E_ARG, "batch is NULL");
    if (bt->B < 0) return fail(STL_E_SHAPE, "B < 0");
    if (bt->B > 0 && !bt->x) return fail(STL_E_ARG, "x is NULL");
    if (bt->D != plan->D) return fail(STL_E_SHAPE, "batch D=%d but the plan was compiled for D=%d", bt->D, plan->D);
    if (bt->T < 1) return fail(STL_E_SHAPE, "T must be >= 1");
    return STL_OK;
}

}  // namespace

extern "C" stl_status stl_workspace_size(const stl_plan* plan, const stl_batch* batch, const stl_launch* cfg,
                                         size_t* fwd_bytes, size_t* bwd_bytes)
{
    stl_status s = check_batch(plan, batch);
    if (s != STL_OK) return s;
    Geom gf, gb, gt;
    if ((s = geometry(plan, batch, cfg, false, false, &gf)) != STL_OK) return s;
    if ((s = geometry(plan, batch, cfg, false, true, &gt)) != STL_OK) return s;
    if ((s = geometry(plan, batch, cfg, true, false, &gb)) != STL_OK) return s;
    if (fwd_bytes) *fwd_bytes = std::max(gf.ws_bytes, gt.ws_bytes);
    if (bwd_bytes) *bwd_bytes = gb.ws_bytes;
    return STL_OK;
}

static size_t saved_header(int64_t B) { return ((size_t)B * sizeof(int32_t) + 255) / 256 * 256; }

// saved buffer: B int32 flags (padded to 256 bytes), [n][B][T] float32 per
// mask node and output when a fused path applies (the fp64 kernels: the
// node's trace; the matrix-core kernels: log2 of the root's softmax weight of
// the node minus lg2 of its window sum), and for the matrix-core path each
// trajectory's exponent range and reference ([B][n][3] int32)
static size_t saved_traces_bytes(const stl_plan* plan, const stl_batch* bt)
{
    return (size_t)plan->dev.fused.n * bt->B * bt->T * sizeof(float);
}

// matrix-core path: after the ranges (256-aligned) the per-mask geometry the
// saving forward derived (256 bytes)
static size_t saved_heads_offset(const stl_plan* plan, const stl_batch* bt)
{
    const size_t e = saved_header(bt->B) + saved_traces_bytes(plan, bt) +
                     (size_t)bt->B * plan->dev.fused.n * 3 * sizeof(int32_t);
    return (e + 255) / 256 * 256;
}

static size_t saved_bytes_needed(const stl_plan* plan, const stl_batch* bt)
{
    const int n = plan->dev.fused.n;
    const bool mx = mx_applies(plan->dev, bt, nullptr, false);
    const bool fusable = n > 0 && bt->offsets == nullptr && (bt->T <= fused_max_T() || mx);
    if (mx) return saved_heads_offset(plan, bt) + 256;
    return saved_header(bt->B) + (fusable ? saved_traces_bytes(plan, bt) : 0);
}

// saved: 0 none, 1 forward writes d_saved, 2 backward reads it
static stl_status run(const stl_plan* plan, const stl_batch* bt, const float* params, bool bwd, float* root,
                      float* nodes, const float* G, float* dx, float* gparams, void* ws, size_t ws_bytes,
                      const stl_launch* cfg, void* stream, int saved = 0, void* d_saved = nullptr,
                      size_t saved_bytes = 0)
{
    stl_status s = check_batch(plan, bt);
    if (s != STL_OK) return s;
    if (saved && bt->B > 0) {
        if (!d_saved) return fail(STL_E_ARG, "saved buffer is NULL");
        const size_t need = saved_bytes_needed(plan, bt);
        if (saved_bytes < need)
            return fail(STL_E_ARG, "saved buffer too small: need %zu bytes, got %zu", need, saved_bytes);
    }
    if (plan->n_params > 0 && !params) return fail(STL_E_ARG, "params is NULL");
    if (!bwd && bt->B > 0 && !root) return fail(STL_E_ARG, "root output is NULL");
    if (bwd && bt->B > 0 && (!G || !dx)) return fail(STL_E_ARG, "grad_root / grad_x is NULL");
    const bool trace = !bwd && nodes != nullptr;
    Geom g;
    if ((s = geometry(plan, bt, cfg, bwd, trace, &g)) != STL_OK) return s;
    if (!ws || ws_bytes < g.ws_bytes)
        return fail(STL_E_WORKSPACE, "workspace too small: need %zu bytes, got %zu", g.ws_bytes, ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    const DevPlan& dp = trace ? plan->dev_trace : plan->dev;
    if (bt->B == 0) {
        if (bwd && gparams) {
            if (launch_reduce_params(nullptr, 0, dp, gparams, st) != hipSuccess)
                return fail(STL_E_HIP, "launch failed: %s", hipGetErrorString(hipGetLastError()));
        }
        return STL_OK;
    }
    Batch b;
    b.x = bt->x;
    b.offsets = bt->offsets;
    b.order = bt->order;
    b.B = bt->B;
    b.T = bt->T;
    b.D = bt->D;
    b.Lcap = g.Lc;
    KArgs ka;
    std::memset(&ka, 0, sizeof ka);
    char* wsb = (char*)ws;
    ka.params = params;
    ka.root = root;
    ka.nodes = nodes;
    ka.n_total = 0;
    ka.G = G;
    ka.dx = dx;
    ka.mask_part = (float*)(wsb + g.off_part);
    ka.garena = g.global ? (float*)(wsb + g.off_arena) : nullptr;
    ka.arena_floats = (int64_t)g.arena_floats;
    ka.counter = (int*)wsb;
    ka.persistent = g.persistent;
    // dense node traces are [n_nodes][B*T]; a ragged batch's N_total (offsets[B])
    // is read by the kernel itself
    if (nodes && !bt->offsets) ka.n_total = bt->B * bt->T;
    ka.list_count = (int*)wsb + 1;
    ka.list = (g.fused || g.mx) ? (int*)(wsb + g.off_list) : nullptr;
    ka.tabs = g.fused ? (const MaskTab*)(wsb + g.off_tabs) : nullptr;
    ka.list_mode = 0;
    ka.part_stride = 1;
    if (g.mx) {
        // each matrix-core kernel derives its tables from the parameters and
        // writes every trajectory's hand-off flag; the generic executor then
        // takes the flagged ones
        MxArgs mx;
        for (int m = 0; m < 2; ++m) {
            const bool has = m < dp.fused.n;
            mx.moff[m] = has ? dp.ins[dp.fused.ins[m]].mask : 0;
            mx.munb[m] = has ? ((dp.ins[dp.fused.ins[m]].flags & F_MASK_UNB) != 0) : 0;
        }
        mx.heads = (MxHead*)(wsb + g.off_mxheads);
        mx.handed = (int*)(wsb + g.off_handed);
        mx.part = ka.mask_part;
        mx.ranges = nullptr;
        ka.list = nullptr;
        hipError_t e;
        if (saved) {
            float* traces = (float*)((char*)d_saved + saved_header(bt->B));
            ka.saved_flag = (int*)d_saved;
            mx.ranges = (int*)((char*)traces + saved_traces_bytes(plan, bt));
            mx.heads = (MxHead*)((char*)d_saved + saved_heads_offset(plan, bt));
            if (saved == 1) ka.saved = traces;
            else ka.saved_in = traces;
        }
        if (!bwd || saved == 2) {
            e = launch_mx(bwd, dp, b, ka, mx, g.mx_lds, st);
        } else {
            // no saved traces: the forward fills workspace copies first
            KArgs kf = ka;
            MxArgs mf = mx;
            kf.root = nullptr;
            kf.saved = (float*)(wsb + g.off_mxtr);
            kf.saved_flag = (int*)(wsb + g.off_mxflag);
            mf.ranges = (int*)(wsb + g.off_mxrange);
            e = launch_mx(false, dp, b, kf, mf, g.mx_lds, st);
            if (e == hipSuccess) {
                KArgs kb = ka;
                kb.saved_in = kf.saved;
                kb.saved_flag = kf.saved_flag;
                e = launch_mx(true, dp, b, kb, mf, g.mx_lds, st);
            }
        }
        if (e != hipSuccess) return fail(STL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        KArgs kx = ka;
        kx.scan = mx.handed;
        kx.persistent = 0;
        kx.saved = nullptr;
        kx.saved_in = nullptr;
        e = launch_exec(bwd, dp, b, kx, g.grid, g.nt, g.lds_bytes, st);
        if (e != hipSuccess) return fail(STL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        if (bwd && gparams) {
            e = launch_reduce_params(ka.mask_part, bt->B, dp, gparams, st);
            if (e != hipSuccess) return fail(STL_E_HIP, "launch failed: %s", hipGetErrorString(e));
        }
        return STL_OK;
    }
    if (saved) {
        int* flags = (int*)d_saved;
        float* traces = (float*)((char*)d_saved + saved_header(bt->B));
        ka.saved_flag = flags;
        if (saved == 1 && g.fused) ka.saved = traces;
        if (saved == 2 && g.fused) ka.saved_in = traces;
        // a forward that does not take the fused path leaves nothing to reuse
        if (saved == 1 && !g.fused && launch_fill_int(flags, bt->B, 0, st) != hipSuccess)
            return fail(STL_E_HIP, "launch failed: %s", hipGetErrorString(hipGetLastError()));
        // (matrix-core layout: geometry marked unusable, so that a matrix-core
        // backward hands every trajectory to the generic executor)
        if (saved == 1 && mx_applies(plan->dev, bt, nullptr, false) &&
            launch_fill_int((int*)((char*)d_saved + saved_heads_offset(plan, bt)), 64, 0, st) != hipSuccess)
            return fail(STL_E_HIP, "launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    // (the fused path's table kernel resets the counters itself)
    if (g.persistent && !g.fused && launch_zero_counter(ka.counter, st) != hipSuccess)
        return fail(STL_E_HIP, "launch failed: %s", hipGetErrorString(hipGetLastError()));
    hipError_t e;
    if (g.fused) {
        e = launch_fused(bwd, dp, b, ka, g.fused_lds, st);
        if (e != hipSuccess) return fail(STL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        // trajectories the fused kernel could not take (signal range beyond
        // fp64 exponents, very wide mask bands) go through the generic executor
        KArgs kf = ka;
        kf.list_mode = 1;
        kf.persistent = 1;
        e = launch_exec(bwd, dp, b, kf, g.grid, g.nt, g.lds_bytes, st);
    } else {
        e = launch_exec(bwd, dp, b, ka, g.grid, g.nt, g.lds_bytes, st);
    }
    if (e != hipSuccess) return fail(STL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    if (bwd && gparams) {
        e = launch_reduce_params(ka.mask_part, bt->B, dp, gparams, st);
        if (e != hipSuccess) return fail(STL_E_HIP, "launch failed: %s", hipGetErrorString(e));
    }
    return STL_OK;
}

extern "C" stl_status stl_forward(const stl_plan* plan, const stl_batch* batch, const float* d_params, float* d_root,
                                  float* d_node_traces, void* d_ws, size_t ws_bytes, const stl_launch* cfg,
                                  void* stream)
{
    return run(plan, batch, d_params, false, d_root, d_node_traces, nullptr, nullptr, nullptr, d_ws, ws_bytes, cfg,
               stream);
}

extern "C" stl_status stl_backward(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                                   const float* d_grad_root, float* d_grad_x, float* d_grad_params, void* d_ws,
                                   size_t ws_bytes, const stl_launch* cfg, void* stream)
{
    return run(plan, batch, d_params, true, nullptr, nullptr, d_grad_root, d_grad_x, d_grad_params, d_ws, ws_bytes,
               cfg, stream);
}

extern "C" stl_status stl_saved_size(const stl_plan* plan, const stl_batch* batch, size_t* saved_bytes)
{
    stl_status s = check_batch(plan, batch);
    if (s != STL_OK) return s;
    if (!saved_bytes) return fail(STL_E_ARG, "saved_bytes is NULL");
    *saved_bytes = saved_bytes_needed(plan, batch);
    return STL_OK;
}

extern "C" stl_status stl_forward_saving(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                                         float* d_root, void* d_saved, size_t saved_bytes, void* d_ws,
                                         size_t ws_bytes, const stl_launch* cfg, void* stream)
{
    return run(plan, batch, d_params, false, d_root, nullptr, nullptr, nullptr, nullptr, d_ws, ws_bytes, cfg, stream,
               1, d_saved, saved_bytes);
}

extern "C" stl_status stl_backward_saved(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                                         const void* d_saved, size_t saved_bytes, const float* d_grad_root,
                                         float* d_grad_x, float* d_grad_params, void* d_ws, size_t ws_bytes,
                                         const stl_launch* cfg, void* stream)
{
    return run(plan, batch, d_params, true, nullptr, nullptr, d_grad_root, d_grad_x, d_grad_params, d_ws, ws_bytes,
               cfg, stream, 2, const_cast<void*>(d_saved), saved_bytes);
}

// ------------------------------------------------------------------ forward with a static workspace

namespace {

// The workspace of stl_forward_static.  In host code `scratch` names a host
// stand-in, not device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device (one copy per GPU).
static __device__ __align__(256) unsigned char scratch[STL_STATIC_WS_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;     // device -> its copy of `scratch`

stl_status scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(STL_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return STL_OK;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return fail(STL_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    *out = p;
    return STL_OK;
}

}  // namespace

extern "C" stl_status stl_forward_static(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                                         float* d_root, float* d_node_traces, const stl_launch* cfg, void* stream)
{
    stl_status s = check_batch(plan, batch);
    if (s != STL_OK) return s;
    Geom g;
    if ((s = geometry(plan, batch, cfg, false, d_node_traces != nullptr, &g)) != STL_OK) return s;
    if (g.ws_bytes > STL_STATIC_WS_BYTES)
        return fail(STL_E_WORKSPACE, "stl_forward_static: this batch needs %zu bytes of workspace, more than the "
                                     "static %zu", g.ws_bytes, (size_t)STL_STATIC_WS_BYTES);
    void* ws = nullptr;
    if ((s = scratch_ptr(&ws)) != STL_OK) return s;
    return run(plan, batch, d_params, false, d_root, d_node_traces, nullptr, nullptr, nullptr, ws,
               STL_STATIC_WS_BYTES, cfg, stream);
}

// ------------------------------------------------------------------ autotuner

namespace {

struct TuneKey {
    const stl_plan* plan;
    int64_t B, T;
    int D;
    bool ragged;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(plan, B, T, D, ragged) < std::tie(o.plan, o.B, o.T, o.D, o.ragged);
    }
};
std::map<TuneKey, std::pair<stl_launch, float>> g_tune;

std::string plan_signature(const stl_plan* p, const stl_batch* bt)
{
    // stable text key for the on-disk cache: program shape plus batch shape
    unsigned long long h = 1469598103934665603ull;
    const unsigned char* c = (const unsigned char*)&p->dev;
    for (size_t i = 0; i < sizeof(DevPlan); ++i) h = (h ^ c[i]) * 1099511628211ull;
    char buf[160];
    snprintf(buf, sizeof buf, "%016llx_B%lld_T%lld_D%d_%s", h, (long long)bt->B, (long long)bt->T, bt->D,
             bt->offsets ? "ragged" : "dense");
    return buf;
}

bool cache_lookup(const std::string& key, stl_launch* out, float* ms)
{
    const char* path = std::getenv("STLMI_TUNE_CACHE");
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[200];
        int a, b2, c;
        float m;
        // one JSON object per line: {"key": "...", "threads": a, "wg_per_cu": b, "global_slots": c, "ms": m}
        if (std::sscanf(line, " {\"key\": \"%199[^\"]\", \"threads\": %d, \"wg_per_cu\": %d, \"global_slots\": %d, \"ms\": %f",
                        k, &a, &b2, &c, &m) == 5 &&
            key == k) {
            out->threads = a;
            out->wg_per_cu = b2;
            out->global_slots = c;
            out->flags = 0;
            *ms = m;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string& key, const stl_launch& l, float ms)
{
    const char* path = std::getenv("STLMI_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"wg_per_cu\": %d, \"global_slots\": %d, \"ms\": %.6f}\n",
                 key.c_str(), l.threads, l.wg_per_cu, l.global_slots, ms);
    std::fclose(f);
}

}  // namespace

extern "C" stl_status stl_autotune(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                                   float* d_root, const float* d_grad_root, float* d_grad_x, float* d_grad_params,
                                   void* d_ws, size_t ws_bytes, void* stream, stl_launch* best, float* best_ms)
{
    stl_status s = check_batch(plan, batch);
    if (s != STL_OK) return s;
    if (!best) return fail(STL_E_ARG, "best is NULL");
    TuneKey key{plan, batch->B, batch->T, batch->D, batch->offsets != nullptr};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return STL_OK;
        }
    }
    const std::string sig = plan_signature(plan, batch);
    float cms = 0;
    if (cache_lookup(sig, best, &cms)) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tune[key] = {*best, cms};
        if (best_ms) *best_ms = cms;
        return STL_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    std::vector<stl_launch> cands;
    for (int nt : {128, 256, 512})
        for (int wpc : {0, 1, 2, 4, 8})
            cands.push_back(stl_launch{nt, wpc, 0, 0});
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(STL_E_HIP, "hipEventCreate failed");
    float bestt = 1e30f;
    stl_launch bl{256, 0, 0, 0};
    bool any = false;
    for (const stl_launch& c : cands) {
        size_t fw = 0, bw = 0;
        if (stl_workspace_size(plan, batch, &c, &fw, &bw) != STL_OK) continue;
        if (std::max(fw, bw) > ws_bytes) continue;
        Geom g;
        if (geometry(plan, batch, &c, true, false, &g) != STL_OK) continue;
        if (g.global && !(c.global_slots)) {
            // candidates that do not fit LDS all degrade to the same global layout
        }
        bool ok = true;
        float tsum = 0;
        for (int rep = 0; rep < 3 && ok; ++rep) {
            hipEventRecord(e0, st);
            ok = stl_forward(plan, batch, d_params, d_root, nullptr, d_ws, ws_bytes, &c, stream) == STL_OK &&
                 stl_backward(plan, batch, d_params, d_grad_root, d_grad_x, d_grad_params, d_ws, ws_bytes, &c,
                              stream) == STL_OK;
            hipEventRecord(e1, st);
            hipEventSynchronize(e1);
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) tsum += ms;   // first rep is a warm-up
        }
        if (!ok) continue;
        any = true;
        float t = tsum / 2;
        if (t < bestt) { bestt = t; bl = c; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!any) return fail(STL_E_WORKSPACE, "no launch candidate fits the workspace");
    *best = bl;
    if (best_ms) *best_ms = bestt;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tune[key] = {bl, bestt};
    }
    cache_store(sig, bl, bestt);
    return STL_OK;
}

// ------------------------------------------------------------------ graphs

struct stl_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" stl_status stl_graph_capture(const stl_plan* plan, const stl_batch* batch, const float* d_params,
                                        float* d_root, const float* d_grad_root, float* d_grad_x,
                                        float* d_grad_params, void* d_ws, size_t ws_bytes, const stl_launch* cfg,
                                        void* stream, stl_graph** out)
{
    if (!out) return fail(STL_E_ARG, "out is NULL");
    *out = nullptr;
    stl_status s = check_batch(plan, batch);
    if (s != STL_OK) return s;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(STL_E_HIP, "stream create failed");
    // order the capture after the caller's pending work
    hipEvent_t ev;
    hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    hipEventRecord(ev, (hipStream_t)stream);
    hipStreamWaitEvent(cs, ev, 0);
    hipStreamSynchronize(cs);
    hipEventDestroy(ev);
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        hipStreamDestroy(cs);
        return fail(STL_E_HIP, "hipStreamBeginCapture failed");
    }
    stl_status s1 = stl_forward(plan, batch, d_params, d_root, nullptr, d_ws, ws_bytes, cfg, cs);
    stl_status s2 = s1 == STL_OK ? stl_backward(plan, batch, d_params, d_grad_root, d_grad_x, d_grad_params, d_ws,
                                                ws_bytes, cfg, cs)
                                 : s1;
    std::string err = stl_last_error();
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    hipStreamDestroy(cs);
    if (s2 != STL_OK) {
        if (graph) hipGraphDestroy(graph);
        stlmi_set_error(err.c_str());
        return s2;
    }
    if (ec != hipSuccess || !graph) return fail(STL_E_HIP, "hipStreamEndCapture failed");
    stl_graph* gr = new (std::nothrow) stl_graph();
    if (!gr) { hipGraphDestroy(graph); return fail(STL_E_ARG, "out of host memory"); }
    gr->graph = graph;
    if (hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        hipGraphDestroy(graph);
        delete gr;
        return fail(STL_E_HIP, "hipGraphInstantiate failed");
    }
    *out = gr;
    return STL_OK;
}

extern "C" stl_status stl_graph_launch(stl_graph* graph, void* stream)
{
    if (!graph) return fail(STL_E_ARG, "graph is NULL");
    hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(STL_E_HIP, "hipGraphLaunch failed: %s", hipGetErrorString(e));
    return STL_OK;
}

extern "C" stl_status stl_graph_destroy(stl_graph* graph)
{
    if (!graph) return STL_OK;
    if (graph->exec) hipGraphExecDestroy(graph->exec);
    if (graph->graph) hipGraphDestroy(graph->graph);
    delete graph;
    return STL_OK;
}

// ------------------------------------------------------------------ interval sweep

extern "C" stl_status stl_interval_sweep(const stl_interval_desc* desc, const float* d_x, int64_t B, int64_t T,
                                         const float* d_a, const float* d_b, int64_t N, float* d_rho,
                                         float* d_grad_a, float* d_grad_b, void* stream)
{
    if (!desc) return fail(STL_E_ARG, "desc is NULL");
    if (desc->op != STL_ALWAYS && desc->op != STL_EVENTUALLY)
        return fail(STL_E_ARG, "op must be STL_ALWAYS or STL_EVENTUALLY");
    if (desc->D < 1 || desc->D > 16) return fail(STL_E_ARG, "D must be in [1, 16]");
    if (!(desc->mask_c > 0.f)) return fail(STL_E_ARG, "mask_c must be > 0");
    if (!(desc->mask_eps >= 0.f)) return fail(STL_E_ARG, "mask_eps must be >= 0");
    if (desc->smooth && !(desc->beta > 0.f)) return fail(STL_E_ARG, "beta must be > 0");
    if (B < 0 || N < 0) return fail(STL_E_SHAPE, "B and N must be >= 0");
    if (T < 1 || T > interval_max_T()) return fail(STL_E_SHAPE, "T must be in [1, %d]", interval_max_T());
    if ((d_grad_a == nullptr) != (d_grad_b == nullptr)) return fail(STL_E_ARG, "pass both gradients or neither");
    if (B == 0 || N == 0) return STL_OK;
    if (!d_x || !d_a || !d_b || !d_rho) return fail(STL_E_ARG, "null device pointer");
    hipError_t e = launch_interval_sweep(desc->op == STL_EVENTUALLY ? 1 : -1, desc->smooth ? 1 : 0, desc->beta,
                                         desc->mask_c, desc->mask_eps, desc->D, desc->w, desc->c, desc->rho_pad, d_x,
                                         B, (int)T, d_a, d_b, N, d_rho, d_grad_a, d_grad_b, (hipStream_t)stream);
    if (e != hipSuccess) return fail(STL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return STL_OK;
}

extern "C" stl_status stl_pstl_descent(const stl_interval_desc* desc, const float* d_x, int64_t B, int64_t T, float c0,
                                       float c1, float beta0, float beta1, int32_t steps, float lr, float gamma,
                                       float* d_logits, float* d_loss, void* stream)
{
    if (!desc) return fail(STL_E_ARG, "desc is NULL");
    if (desc->op != STL_ALWAYS && desc->op != STL_EVENTUALLY)
        return fail(STL_E_ARG, "op must be STL_ALWAYS or STL_EVENTUALLY");
    if (desc->D < 1 || desc->D > 16) return fail(STL_E_ARG, "D must be in [1, 16]");
    if (!(desc->mask_eps >= 0.f)) return fail(STL_E_ARG, "mask_eps must be >= 0");
    if (!(c0 > 0.f && c1 > 0.f && beta0 > 0.f && beta1 > 0.f)) return fail(STL_E_ARG, "schedules must be > 0");
    if (steps < 0 || !std::isfinite(lr) || !std::isfinite(gamma)) return fail(STL_E_ARG, "bad steps, lr or gamma");
    if (T < 1 || T > 1024) return fail(STL_E_SHAPE, "T must be in [1, 1024]");
    if (B < 1 || B * T > pstl_max_BT()) return fail(STL_E_SHAPE, "need B >= 1 and B * T <= %d", pstl_max_BT());
    if (!d_x || !d_logits) return fail(STL_E_ARG, "null device pointer");
    hipError_t e = launch_pstl_descent(d_x, (int)B, (int)T, desc->D, desc->w, desc->c,
                                       desc->op == STL_EVENTUALLY ? 1 : -1, desc->mask_eps, c0, c1, beta0, beta1,
                                       steps, lr, gamma, d_logits, d_loss, (hipStream_t)stream);
    if (e != hipSuccess) return fail(STL_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return STL_OK;
}
