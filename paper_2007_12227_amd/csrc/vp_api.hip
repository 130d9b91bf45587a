// vp_api.hip -- host runtime of libvp: handles, validation, per-step plans,
// launch lists, HIP graphs, batching and the tile autotuner.  See include/vp.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/vp.h"
#include "vp_internal.h"

using namespace vp;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(VP_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

constexpr int kMinTile = 8;
constexpr size_t kDefaultLds = 64 * 1024;
size_t g_max_lds = kDefaultLds;  // raised once per process to what the device allows (160 KiB on gfx950)
std::once_flag g_lds_once;

// Let the deposit kernels use the device's full LDS per workgroup.
void raise_lds_limit() {
    std::call_once(g_lds_once, [] {
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return;
        if (lim <= (int)kDefaultLds) return;
        for (int basis : {kBasisTent, kBasisQuadratic, kBasisCubic})
            if (hipFuncSetAttribute(deposit_kernel(basis), hipFuncAttributeMaxDynamicSharedMemorySize, lim - 1024) !=
                hipSuccess)
                return;
        g_max_lds = (size_t)(lim - 1024);
    });
}
constexpr int kGraphSteps = 16;

// HIP events destroyed with their holder (also on an early error return).
struct Events {
    std::vector<hipEvent_t> ev;
    explicit Events(size_t n) : ev(n, nullptr) {}
    Events(const Events&) = delete;
    Events& operator=(const Events&) = delete;
    ~Events() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    hipError_t create() {
        for (auto& e : ev)
            if (hipError_t r = hipEventCreate(&e); r != hipSuccess) return r;
        return hipSuccess;
    }
    hipEvent_t& operator[](size_t k) { return ev[k]; }
};

bool axis_ok(const vp_axis* a) {
    return a && a->n >= 4 && a->n <= (1 << 16) && isfinite(a->lo) && isfinite(a->hi) && a->hi > a->lo;
}

double spacing(const vp_axis& a) { return (a.hi - a.lo) / (a.periodic ? a.n : a.n - 1); }

// The kernels and the box planner do their cell arithmetic in 32-bit
// integers: a step whose drift, or whose pendulum kick, moves a node by more
// than 2^20 cells is refused (the exact rotation stays within the lattice;
// the FEL kick is bounded by its field, which the planner takes per step).
constexpr double kMaxCellsPerStep = 1048576.0;
bool step_too_large(const vp_axis& x, const vp_axis& p, const vp_hamiltonian& h, double dt) {
    if (h.kind == VP_H_SHO_EXACT) return false;
    const double v = std::max(fabs(p.lo), fabs(p.hi)) + (h.kind == VP_H_FEL ? fabs(h.fel_delta) : 0.0);
    const double drift = fabs(dt) * v / spacing(x);
    const double kick = h.kind == VP_H_PENDULUM ? fabs(dt * h.a) / spacing(p) : 0.0;
    return !(drift <= kMaxCellsPerStep && kick <= kMaxCellsPerStep);
}

// Workspace layout: every piece 256-byte aligned.
struct Layout {
    size_t w0, w1, b, tab_x, tab_p, fel_ex, fel_eq, fel_state, partials, counters,
        inst, off, moments, boxes, map_f, map_k, total;
    size_t partial_doubles;
};

Layout layout(int nx, int np) {
    Layout L{};
    size_t n = (size_t)nx * np, o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.w0 = take(n * 4);
    L.w1 = take(n * 4);
    L.b = take(n * 4);
    L.tab_x = take((size_t)nx * 16);
    L.tab_p = take((size_t)np * 16);
    L.fel_ex = take((size_t)nx * 16);
    L.fel_eq = take((size_t)np * 16);
    L.fel_state = take(kFelStateLen * 8);
    // solve tiles (FEL bunching partials) and reduction blocks
    size_t tiles = (size_t)((nx + kSegX - 1) / kSegX) * ((np + kSegP - 1) / kSegP);
    L.partial_doubles = std::max((size_t)kReduceBlocks * kMoments, kPartialsPerTile * tiles);
    L.partials = take(L.partial_doubles * 8);
    L.counters = take(4 * sizeof(uint32_t));
    L.inst = take(sizeof(VpInst));
    L.off = take(8 * sizeof(int32_t));
    L.moments = take(kMoments * 8);
    L.boxes = take(box_capacity(nx, np) * sizeof(int4));
    L.map_f = take(n * sizeof(float2));  // the cached push of a static Hamiltonian
    L.map_k = take(n * sizeof(int32_t));
    L.total = o;
    return L;
}

// A list of instances launched together: one instance for a grid, many for a batch.
struct LaunchList {
    VpInst* d_inst = nullptr;
    int32_t* d_off1 = nullptr;  // deposit tiles
    int32_t* d_off2 = nullptr;  // solve tiles
    int ninst = 0, total1 = 0, total2 = 0;
    bool has_fel = false;  // an FEL instance: the field kernel follows the solve
    bool has_rk4 = false;  // a Runge-Kutta FEL instance: its stage sums precede the deposit
    // one Runge-Kutta instance whose deposit sums the stage partials itself
    // (stage_fusable): no field launch between the stage sums and the deposit
    bool fuse_stage = false;
    int basis = kBasisTent;  // of every instance in the list
    int solve = kSolveTent;  // the solve kernel serving every instance in the list
    size_t lds1 = 0;
    int threads1 = 256;  // deposit workgroup size
    int grid1 = 0;       // deposit workgroups: 0 = one per tile, else that many looping over the tiles
    hipStream_t stream = nullptr;
    // graphs of r steps (r = 1 .. kGraphSteps), by the relative parity they start at
    hipGraphExec_t exec[kGraphSteps + 1][2] = {};
    // the launch's range word (device) and its host copy, refreshed after
    // every run (pinned, read without waiting for the stream)
    uint32_t* d_any = nullptr;
    volatile uint32_t* h_any = nullptr;

    void drop_graphs() {
        for (auto& row : exec)
            for (auto& e : row)
                if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
    }
    LaunchArgs args(const int32_t* off, int total, int parity, int mode = 0) const {
        return LaunchArgs{d_inst, off, ninst, total, parity, mode, d_any};
    }
    // the kernels of one step: {kernel, off, total (= grid), lds, threads, mode}
    struct K { const void* fn; const int32_t* off; int total; size_t lds; int threads; int mode; int grid = 0; };
    int dep_grid() const { return grid1 > 0 && grid1 < total1 ? grid1 : total1; }
    int kernels(K (&k)[5]) const {
        int n = 0;
        if (has_rk4) {
            k[n++] = K{fel_stage_kernel(), d_off2, total2, 0, kStageThreads, 0};
            if (!fuse_stage) k[n++] = K{fel_field_kernel(), d_off2, ninst, 0, kFieldThreads, 1};
        }
        k[n++] = K{deposit_kernel(basis), d_off1, total1, lds1, threads1, fuse_stage ? 1 : 0, dep_grid()};
        k[n++] = K{solve_kernel(solve), d_off2, total2, 0, solve_threads(solve), 0};
        if (has_fel) k[n++] = K{fel_field_kernel(), d_off2, ninst, 0, kFieldThreads, 0};
        return n;
    }
    int enqueue_step(int parity) const {
        if (has_rk4) {
            HIP_TRY(launch_fel_stage(args(d_off2, total2, parity), total2, stream));
            if (!fuse_stage) HIP_TRY(launch_fel_field(args(d_off2, ninst, parity, 1), stream));
        }
        HIP_TRY(launch_deposit(args(d_off1, total1, parity, fuse_stage ? 1 : 0), dep_grid(), lds1, threads1, stream,
                               basis));
        HIP_TRY(launch_solve(args(d_off2, total2, parity), total2, stream, solve));
        if (has_fel) HIP_TRY(launch_fel_field(args(d_off2, ninst, parity), stream));
        return VP_OK;
    }
    int build_graph(int rel_parity, int steps) {
        hipGraph_t graph;
        HIP_TRY(hipGraphCreate(&graph, 0));
        hipGraphNode_t prev = nullptr;
        std::vector<LaunchArgs> keep;
        keep.reserve(5 * steps);
        K ks[5];
        const int nk = kernels(ks);
        for (int s = 0; s < steps; ++s) {
            for (int ki = 0; ki < nk; ++ki) {
                const K& k = ks[ki];
                keep.push_back(args(k.off, k.total, (rel_parity + s) & 1, k.mode));
                void* kp[1] = {&keep.back()};
                hipKernelNodeParams p{};
                p.func = const_cast<void*>(k.fn);
                p.gridDim = dim3(k.grid > 0 ? k.grid : k.total);
                p.blockDim = dim3(k.threads);
                p.sharedMemBytes = (unsigned)k.lds;
                p.kernelParams = kp;
                p.extra = nullptr;
                hipGraphNode_t node;
                hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
                if (e != hipSuccess) {
                    (void)hipGraphDestroy(graph);
                    return fail(VP_EHIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
                }
                prev = node;
            }
        }
        hipError_t e = hipGraphInstantiate(&exec[steps][rel_parity], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(VP_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        return VP_OK;
    }
    // A deposit cell sum left the fixed-point range in a run whose copy of the
    // range word has arrived (a run still in flight reports on a later call).
    bool range_seen() const { return h_any && *h_any != 0u; }
    // Copy the range word to the host behind the work just enqueued.
    int post_range_copy() const {
        if (h_any) HIP_TRY(hipMemcpyAsync((void*)h_any, d_any, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        return VP_OK;
    }
    // Run n steps starting at relative parity rp.
    // With use_graph: whole graphs of kGraphSteps steps, then one graph of
    // the remaining steps (the graphs of every length are built on first use
    // and kept; 16 is even, so the remainder starts at parity rp too).
    int run(int64_t n, int rp, bool use_graph) {
        int64_t done = 0;
        if (use_graph) {
            auto launch = [&](int steps) -> int {
                if (!exec[steps][rp]) {
                    int rc = build_graph(rp, steps);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(exec[steps][rp], stream));
                return VP_OK;
            };
            for (; done + kGraphSteps <= n; done += kGraphSteps)
                if (int rc = launch(kGraphSteps)) return rc;
            if (done < n) {
                if (int rc = launch((int)(n - done))) return rc;
                done = n;
            }
        }
        for (; done < n; ++done) {
            int rc = enqueue_step((int)((rp + done) & 1));
            if (rc) return rc;
        }
        return post_range_copy();
    }
    // Run n steps from relative parity rp with direct launches and HIP events
    // attached to the dispatches: us[0] the mean duration of the deposit
    // phase (for the Runge-Kutta FEL from the stage sums before it), us[1]
    // of the solve phase (for the FEL up to the field update after it).
    // Waits for the stream.
    int timed(int64_t n, int rp, double us[2]) {
        Events ev((size_t)(4 * n));
        HIP_TRY(ev.create());
        for (int64_t s = 0; s < n; ++s) {
            const int par = (int)((rp + s) & 1);
            hipEvent_t* e = &ev[4 * s];
            if (has_rk4) {
                HIP_TRY(launch_fel_stage(args(d_off2, total2, par), total2, stream, e[0], nullptr));
                if (!fuse_stage) HIP_TRY(launch_fel_field(args(d_off2, ninst, par, 1), stream));
            }
            HIP_TRY(launch_deposit(args(d_off1, total1, par, fuse_stage ? 1 : 0), dep_grid(), lds1, threads1, stream,
                                   basis, has_rk4 ? nullptr : e[0], e[1]));
            HIP_TRY(launch_solve(args(d_off2, total2, par), total2, stream, solve, e[2], has_fel ? nullptr : e[3]));
            if (has_fel) HIP_TRY(launch_fel_field(args(d_off2, ninst, par), stream, nullptr, e[3]));
        }
        HIP_TRY(hipEventSynchronize(ev[4 * n - 1]));
        double t[2] = {0.0, 0.0};
        for (int64_t s = 0; s < n; ++s)
            for (int k = 0; k < 2; ++k) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev[4 * s + 2 * k], ev[4 * s + 2 * k + 1]));
                t[k] += ms;
            }
        for (int k = 0; k < 2; ++k) us[k] = 1000.0 * t[k] / n;
        return post_range_copy();
    }
};

// One Runge-Kutta instance on tents with at most kStageFuseTiles solve tiles
// and deposit workgroups of at least kFieldThreads threads: each deposit
// workgroup sums the stage partials itself (at most 32 KB of reads), which
// saves the launch of the one-workgroup field kernel between the stage sums
// and the deposit.
bool stage_fusable(const LaunchList& L) {
    return L.has_rk4 && L.ninst == 1 && L.basis == kBasisTent && L.total2 <= kStageFuseTiles &&
           L.threads1 >= kFieldThreads;
}

// Small pinned host word for a launch list's range flag.
int alloc_host_flag(volatile uint32_t** out) {
    void* p = nullptr;
    HIP_TRY(hipHostMalloc(&p, 64, hipHostMallocDefault));
    *reinterpret_cast<uint32_t*>(p) = 0u;
    *out = reinterpret_cast<volatile uint32_t*>(p);
    return VP_OK;
}
void free_host_flag(volatile uint32_t** p) {
    if (*p) (void)hipHostFree((void*)*p);
    *p = nullptr;
}

}  // namespace

namespace vp {
// The calling thread's error message for a failure reported by another
// source file of the library (the 2D2V runtime).
int set_error(int code, const char* msg) {
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}
}  // namespace vp

struct vp_grid {
    vp_axis x{}, p{};
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L{};
    VpInst inst{};  // host copy of the device descriptor
    LaunchList list;
    vp_hamiltonian ham{};
    bool has_ham = false, has_density = false;
    bool plan_valid = false, bunch_valid = false;
    double bunch_dz = 0.0;  // the FEL step size the bunching in the device state belongs to
    double plan_dt = 0.0;
    int parity = 0;
    int64_t step = 0;
    double N0 = 0.0;
    vp_tiles tiles{};
    bool use_graph = true;
    bool use_map = false;  // cache the push of a static Hamiltonian (k_map); off: it does not pay here
    bool in_batch = false;
    int basis = kBasisTent;

    template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

struct vp_batch {
    std::vector<vp_grid*> grids;
    std::vector<double> dt;
    LaunchList list;
    int64_t steps_done = 0;
};

namespace {

int validate_tiles(int basis, const vp_tiles& t) {
    if (t.k1_tx < kMinTile || t.k1_ty < 1)
        return fail(VP_EINVAL, "deposit tile below the minimum (k1_tx >= %d, k1_ty >= 1)", kMinTile);
    if (t.k1_tx > 4096 || t.k1_ty > 1024) return fail(VP_EINVAL, "deposit tile too large");
    const int max_threads = basis == kBasisCubic ? kDepositCubicThreads : kDepositMaxThreads;
    if (t.k1_threads < 64 || t.k1_threads > max_threads || t.k1_threads % 64)
        return fail(VP_EINVAL, "deposit threads %d: need a multiple of 64 in [64, %d]", t.k1_threads, max_threads);
    if (deposit_lds_bytes(t.k1_tx, t.k1_ty, basis) > g_max_lds)
        return fail(VP_EINVAL, "deposit tile %dx%d needs %zu bytes of LDS (limit %zu)", t.k1_tx, t.k1_ty,
                    deposit_lds_bytes(t.k1_tx, t.k1_ty, basis), g_max_lds);
    return VP_OK;
}

// Starting deposit shape by lattice size: the largest of the timed shapes
// that still gives every compute unit a tile (256 of them), since larger
// tiles rescan fewer halo sources and keep more waves per compute unit.
// (The 64 x 64 x 512 rung took the served mix from 6.0e10 to 6.8e10
// node-steps/s; 512 threads for the smallest tiles too helped it a little
// more but slowed a batch of 256 small grids by 21%.)
vp_tiles default_tiles(int nx, int np, int basis = kBasisTent) {
    const double nodes = (double)nx * np;
    // (the cubic basis's 8-cell border leaves a 128 x 128 tile without room;
    // 128 x 64 is the timed best for it at 2048^2)
    if (nodes >= 256.0 * 128 * 128) return basis == kBasisCubic ? vp_tiles{128, 64, 768} : vp_tiles{128, 128, 1024};
    if (nodes >= 256.0 * 128 * 64) return vp_tiles{128, 64, 512};
    if (nodes >= 256.0 * 64 * 64) return vp_tiles{64, 64, 512};
    return vp_tiles{64, 32, 256};
}

vp_tiles clip_tiles(const vp_grid* g, vp_tiles t) {
    t.k1_tx = std::min(t.k1_tx, g->x.n);
    t.k1_ty = std::min(t.k1_ty, g->p.n);
    return t;
}

// Upload the host descriptor and tile offsets of a single grid.
int upload_inst(vp_grid* g) {
    VpInst& I = g->inst;
    const vp_tiles t = clip_tiles(g, g->tiles);
    I.k1_tx = t.k1_tx;
    I.k1_ty = t.k1_ty;
    I.k1_tiles_x = (g->x.n + t.k1_tx - 1) / t.k1_tx;
    I.k1_tiles = I.k1_tiles_x * ((g->p.n + t.k1_ty - 1) / t.k1_ty);
    I.k2_tiles = solve_tiles(g->x.n, g->p.n, g->basis);
    I.parity0 = 0;
    // source boxes of a push that does not depend on the state: planned here
    // once, instead of by one thread of every deposit tile at every step
    I.boxes = nullptr;
    std::vector<int4> boxes;
    if (I.push.kind != kFel && (size_t)I.k1_tiles <= box_capacity(g->x.n, g->p.n)) {
        boxes.resize(I.k1_tiles);
        for (int t2 = 0; t2 < I.k1_tiles; ++t2) {
            const int tyi = t2 / I.k1_tiles_x, txi = t2 - tyi * I.k1_tiles_x;
            const int X0 = txi * I.k1_tx, Y0 = tyi * I.k1_ty;
            int b[4];
            source_box(I.push, X0, std::min(X0 + I.k1_tx, g->x.n), Y0, std::min(Y0 + I.k1_ty, g->p.n), b);
            boxes[t2] = make_int4(b[0], b[1], b[2], b[3]);
        }
        I.boxes = g->at<int4>(g->L.boxes);
        HIP_TRY(hipMemcpyAsync(g->at<int4>(g->L.boxes), boxes.data(), boxes.size() * sizeof(int4),
                               hipMemcpyHostToDevice, g->stream));
    }
    // a push that does not depend on the state is the same every step: form
    // it once into the map the deposit reads instead of pushing
    const bool map = g->use_map && I.push.kind != kFel;
    I.map_f = map ? g->at<float2>(g->L.map_f) : nullptr;
    I.map_k = map ? g->at<int32_t>(g->L.map_k) : nullptr;
    int32_t off[4] = {0, I.k1_tiles, 0, I.k2_tiles};
    HIP_TRY(hipMemcpyAsync(g->list.d_inst, &I, sizeof(VpInst), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->list.d_off1, off, sizeof off, hipMemcpyHostToDevice, g->stream));
    if (map) HIP_TRY(launch_map(g->list.d_inst, (long)g->x.n * g->p.n, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    // the graphs hold launch shapes and kernel choices, not the descriptor
    // (it is read from device memory): keep them while those stay the same
    LaunchList& L = g->list;
    const auto shape = std::make_tuple(L.ninst, L.has_fel, L.has_rk4, L.total1, L.total2, L.lds1, L.basis, L.solve,
                                       L.threads1);
    L.ninst = 1;
    L.has_fel = I.push.kind == kFel;
    L.has_rk4 = I.push.kind == kFel && I.push.rk4;
    L.total1 = I.k1_tiles;
    L.total2 = I.k2_tiles;
    L.lds1 = deposit_lds_bytes(t.k1_tx, t.k1_ty, g->basis);
    L.basis = g->basis;
    L.solve = solve_kind(g->basis, g->x.n, g->p.n, g->x.periodic != 0);
    L.threads1 = t.k1_threads;
    L.fuse_stage = stage_fusable(L);
    if (shape != std::make_tuple(L.ninst, L.has_fel, L.has_rk4, L.total1, L.total2, L.lds1, L.basis, L.solve,
                                 L.threads1))
        L.drop_graphs();
    return VP_OK;
}

// Push parameters in cell units for step dt (FEL: the kick amplitudes alpha,
// beta come from the device field at each step; kick_re/kick_im fill them in
// for host-side planning).
PushParams push_params(const vp_axis& x, const vp_axis& p, const vp_hamiltonian& H, double dt, int basis,
                       double kick_re = 0.0, double kick_im = 0.0) {
    const double hx = spacing(x), hp = spacing(p);
    PushParams P{};
    P.kind = H.kind;
    P.wide = basis;  // the overlaps reach `basis` cells further than tents
    P.nx = x.n;
    P.np = p.n;
    P.x_periodic = x.periodic ? 1 : 0;
    P.x_lo = (float)x.lo;
    P.hx = (float)hx;
    P.p_lo = (float)p.lo;
    P.hp = (float)hp;
    if (H.kind == VP_H_SHO_EXACT) {
        P.c = (float)cos(H.omega * dt);
        P.s = (float)sin(H.omega * dt);
        return P;
    }
    const double delta = H.kind == VP_H_FEL ? H.fel_delta : 0.0;
    P.drift0 = (float)((delta + p.lo) * dt / hx);
    P.drift1 = (float)(hp * dt / hx);
    P.q0 = (float)(0.5 * dt * (delta + p.lo));
    P.q1 = (float)(0.5 * dt * hp);
    P.kd = H.kind == VP_H_FREE ? 0.0f : (float)(hp * dt / (2.0 * hx));
    if (H.kind == VP_H_PENDULUM) P.beta = (float)(-H.a * dt / hp);
    if (H.kind == VP_H_FEL) {
        const double kick = -2.0 * dt / hp;
        P.alpha = (float)(kick * kick_re);
        P.beta = (float)(-kick * kick_im);
        P.rk4 = H.integrator == VP_FEL_RK4 ? 1 : 0;
    }
    return P;
}

TableParams table_params(const vp_axis& x, const vp_axis& p, const vp_hamiltonian& H, double dt) {
    TableParams T{};
    T.kind = H.kind;
    T.x_lo = x.lo;
    T.hx = spacing(x);
    T.p_lo = p.lo;
    T.hp = spacing(p);
    T.dt = dt;
    T.delta = H.kind == VP_H_FEL ? H.fel_delta : 0.0;
    T.omega = H.omega;
    return T;
}

// Per-step tables of the push for step dt (FP64 on the host, stored FP32),
// and the FP64 phase tables of the FEL bunching.
int plan(vp_grid* g, double dt) {
    const int nx = g->x.n, np = g->p.n;
    const double hp = spacing(g->p);
    const vp_hamiltonian& H = g->ham;
    std::vector<float4> tx(nx), tp(np);
    std::vector<double2> ex(nx), eq(np);
    g->inst.push = push_params(g->x, g->p, H, dt, g->basis);
    const TableParams T = table_params(g->x, g->p, H, dt);
    for (int i = 0; i < nx; ++i) table_x(T, i, tx[i], ex[i]);
    for (int j = 0; j < np; ++j) table_p(T, j, tp[j], eq[j]);
    VpInst& I = g->inst;
    I.fel_kick = -2.0 * dt / hp;
    I.fel_sigma2 = (float)H.fel_sigma2;
    I.fel_dz = dt;
    HIP_TRY(hipMemcpyAsync(g->at<float4>(g->L.tab_x), tx.data(), nx * sizeof(float4), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->at<float4>(g->L.tab_p), tp.data(), np * sizeof(float4), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->at<double2>(g->L.fel_ex), ex.data(), nx * sizeof(double2), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->at<double2>(g->L.fel_eq), eq.data(), np * sizeof(double2), hipMemcpyHostToDevice, g->stream));
    int rc = upload_inst(g);  // synchronises, so the host vectors may go
    if (rc) return rc;
    g->plan_dt = dt;
    g->plan_valid = true;
    return VP_OK;
}

int launch_reduce_on(vp_grid* g, int mode, double dt) {
    ReduceArgs R{};
    R.w = g->at<float>(g->parity ? g->L.w1 : g->L.w0);
    R.nx = g->x.n;
    R.np = g->p.n;
    R.kind = g->ham.kind;
    R.mode = mode;
    R.x_lo = g->x.lo;
    R.hx = spacing(g->x);
    R.p_lo = g->p.lo;
    R.hp = spacing(g->p);
    R.a = g->ham.a;
    R.inv_n0 = g->N0 != 0.0 ? 1.0 / g->N0 : 0.0;
    R.fel_ex = g->at<double2>(g->L.fel_ex);
    R.fel_eq = g->at<double2>(g->L.fel_eq);
    R.partials = g->at<double>(g->L.partials);
    R.counter = g->at<uint32_t>(g->L.counters) + 1;
    R.out = mode == 1 ? g->at<double>(g->L.fel_state) : g->at<double>(g->L.moments);
    R.dz = dt;
    // integrals of p^2 and cos x over a basis function (per unit of spacing):
    // the B-spline of degree d (d = 1 the tent) is d + 1 unit boxes
    // convolved, so its variance is (d + 1)/12 and its transform sinc^(d+1)
    const double y = 0.5 * R.hx, sc = y == 0.0 ? 1.0 : sin(y) / y;
    const int degree = g->basis + 1;
    R.var_c = (degree + 1) / 12.0;
    R.cos_fac = pow(sc, degree + 1);
    HIP_TRY(launch_reduce(R, g->stream));
    return VP_OK;
}

// Prepare a grid for stepping with dt: plan and, for the FEL, the bunching of
// the current state at the half-drift phases of this dz.
int prepare(vp_grid* g, double dt) {
    if (!g->has_ham || !g->has_density)
        return fail(VP_ESTATE, "set the Hamiltonian and the density before stepping");
    if (!isfinite(dt)) return fail(VP_EINVAL, "dt must be finite");
    if (step_too_large(g->x, g->p, g->ham, dt))
        return fail(VP_EINVAL, "dt %g moves nodes by more than 2^20 cells per step", dt);
    if (g->ham.kind == VP_H_FEL && !(g->N0 != 0.0))
        return fail(VP_ESTATE, "the FEL needs a nonzero sum of the initial weights (N0 normalises the bunching)");
    if (!g->plan_valid || g->plan_dt != dt) {
        int rc = plan(g, dt);
        if (rc) return rc;
    }
    // the FEL bunching at the half-drift phases of this dz: the solve's
    // epilogue keeps it current while dz stays; otherwise reduce the state
    if (g->ham.kind == VP_H_FEL && (!g->bunch_valid || g->bunch_dz != dt)) {
        int rc = launch_reduce_on(g, 1, dt);
        if (rc) return rc;
        g->bunch_valid = true;
        g->bunch_dz = dt;
    }
    return VP_OK;
}

// (Re)build a batch's launch list from its grids as they are planned now:
// the descriptors, the tile offsets, one deposit workgroup size and LDS size
// for the launch, one solve kernel.  The graphs are rebuilt on next use.
int fill_batch(vp_batch* b) {
    const int n = (int)b->grids.size();
    std::vector<VpInst> insts(n);
    std::vector<int32_t> off1(n + 1, 0), off2(n + 1, 0);
    size_t lds1 = 0;
    // one workgroup size serves every tile of the launch (the deposit loops
    // stride by it): the one most of the tiles were planned with (a small
    // grid timed alone may pick a large workgroup for its few tiles)
    std::map<int, long> tiles_at;
    for (auto* g : b->grids) tiles_at[g->list.threads1] += g->inst.k1_tiles;
    int threads1 = tiles_at.begin()->first;
    for (auto& kv : tiles_at)
        if (kv.second > tiles_at[threads1]) threads1 = kv.first;
    LaunchList& L = b->list;
    L.has_fel = L.has_rk4 = L.fuse_stage = false;  // a batch keeps the stage field launch
    L.solve = kSolveTent;
    for (int k = 0; k < n; ++k) {
        vp_grid* g = b->grids[k];
        insts[k] = g->inst;
        insts[k].parity0 = g->parity;
        off1[k + 1] = off1[k] + insts[k].k1_tiles;
        off2[k + 1] = off2[k] + insts[k].k2_tiles;
        lds1 = std::max(lds1, deposit_lds_bytes(insts[k].k1_tx, insts[k].k1_ty, g->basis));
        L.has_fel |= insts[k].push.kind == kFel;
        L.has_rk4 |= insts[k].push.kind == kFel && insts[k].push.rk4;
        // one solve kernel for the launch: the narrow-lattice one if any grid needs it
        L.solve = std::max(L.solve, g->list.solve);
    }
    L.total1 = off1[n];
    L.total2 = off2[n];
    L.lds1 = lds1;
    L.threads1 = threads1;
    L.basis = b->grids[0]->basis;
    L.drop_graphs();
    hipStream_t s = L.stream;
    HIP_TRY(hipMemcpyAsync(L.d_inst, insts.data(), sizeof(VpInst) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(L.d_off1, off1.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(L.d_off2, off2.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    // the parities now stand relative to the grids' own
    b->steps_done = 0;
    return VP_OK;
}

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, long, int>, vp_tiles> g_tune_cache;  // shape class -> tiles

}  // namespace

extern "C" {

size_t vp_workspace_bytes(const vp_axis* x, const vp_axis* p) {
    if (!axis_ok(x) || !axis_ok(p)) return 0;
    return layout(x->n, p->n).total;
}

int vp_create_grid(const vp_grid_desc* d, vp_grid** out) {
    if (!d || !out) return fail(VP_EINVAL, "null argument");
    *out = nullptr;
    if (!axis_ok(&d->x) || !axis_ok(&d->p)) return fail(VP_EINVAL, "invalid axis (need n >= 4, hi > lo, finite)");
    if (d->p.periodic) return fail(VP_EUNSUPPORTED, "the momentum axis must be open");
    Layout L = layout(d->x.n, d->p.n);
    if (!d->workspace) return fail(VP_ENOMEM, "no workspace");
    if (d->workspace_bytes < L.total)
        return fail(VP_ENOMEM, "workspace of %zu bytes, need %zu", d->workspace_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(d->workspace) % 256)
        return fail(VP_EINVAL, "workspace must be 256-byte aligned");
    raise_lds_limit();
    vp_grid* g = new vp_grid();
    g->x = d->x;
    g->p = d->p;
    g->stream = reinterpret_cast<hipStream_t>(d->stream);
    g->ws = reinterpret_cast<char*>(d->workspace);
    g->L = L;
    g->tiles = default_tiles(d->x.n, d->p.n);
    g->list.stream = g->stream;
    g->list.d_inst = g->at<VpInst>(L.inst);
    g->list.d_off1 = g->at<int32_t>(L.off);
    g->list.d_off2 = g->at<int32_t>(L.off) + 2;
    g->list.d_any = g->at<uint32_t>(L.counters) + kRangeFlag;
    if (alloc_host_flag(&g->list.h_any) != VP_OK) {
        delete g;
        return VP_EHIP;
    }
    VpInst& I = g->inst;
    I.w[0] = g->at<float>(L.w0);
    I.w[1] = g->at<float>(L.w1);
    I.b = g->at<float>(L.b);
    I.tab_x = g->at<float4>(L.tab_x);
    I.tab_p = g->at<float4>(L.tab_p);
    I.fel_ex = g->at<double2>(L.fel_ex);
    I.fel_eq = g->at<double2>(L.fel_eq);
    I.fel_state = g->at<double>(L.fel_state);
    I.partials = g->at<double>(L.partials);
    I.counters = g->at<uint32_t>(L.counters);
    std::vector<double> st(kFelStateLen, 0.0);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(g->at<double>(L.fel_state), st.data(), st.size() * 8, hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->at<uint32_t>(L.counters), 0, 4 * sizeof(uint32_t), g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        free_host_flag(&g->list.h_any);
        delete g;
        return fail(VP_EHIP, "grid initialisation: %s", hipGetErrorString(e));
    }
    *out = g;
    return VP_OK;
}

int vp_destroy_grid(vp_grid* g) {
    if (!g) return VP_OK;
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    (void)hipStreamSynchronize(g->stream);
    g->list.drop_graphs();
    free_host_flag(&g->list.h_any);
    delete g;
    return VP_OK;
}

int vp_set_hamiltonian(vp_grid* g, const vp_hamiltonian* h) {
    if (!g || !h) return fail(VP_EINVAL, "null argument");
    if (h->kind < VP_H_FREE || h->kind > VP_H_FEL) return fail(VP_EINVAL, "unknown Hamiltonian kind %d", h->kind);
    if (!isfinite(h->a) || !isfinite(h->omega) || !isfinite(h->fel_delta) || !isfinite(h->fel_sigma2) ||
        !isfinite(h->A_re) || !isfinite(h->A_im))
        return fail(VP_EINVAL, "non-finite Hamiltonian parameter");
    if (h->kind == VP_H_SHO_EXACT && g->x.periodic)
        return fail(VP_EUNSUPPORTED, "the exact rotation needs an open x axis");
    if (h->integrator != VP_FEL_DKD && !(h->kind == VP_H_FEL && h->integrator == VP_FEL_RK4))
        return fail(VP_EINVAL, "integrator %d: only the FEL takes VP_FEL_RK4", h->integrator);
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    g->ham = *h;
    g->has_ham = true;
    g->plan_valid = false;
    g->bunch_valid = false;
    if (h->kind == VP_H_FEL) {
        double A[2] = {h->A_re, h->A_im};
        HIP_TRY(hipMemcpyAsync(g->at<double>(g->L.fel_state) + kA, A, sizeof A, hipMemcpyHostToDevice, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
    }
    return VP_OK;
}

int vp_set_density(vp_grid* g, const float* w, int32_t on_device) {
    if (!g || !w) return fail(VP_EINVAL, "null argument");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    const size_t bytes = (size_t)g->x.n * g->p.n * sizeof(float);
    float* dst = g->at<float>(g->parity ? g->L.w1 : g->L.w0);
    HIP_TRY(hipMemcpyAsync(dst, w, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, g->stream));
    int rc = launch_reduce_on(g, 2, 0.0);
    if (rc) return rc;
    double m[kMoments];
    HIP_TRY(hipMemcpyAsync(m, g->at<double>(g->L.moments), sizeof m, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    if (m[9] > 0.0) {
        // the deposit's fixed-point taps would drop a non-finite weight silently
        g->has_density = false;
        return fail(VP_ENONFINITE, "%lld non-finite weights in the density", (long long)m[9]);
    }
    g->N0 = m[0];
    {
        // fixed-point scale of the deposit cell sums: 2^(40 - e), max|w0| < 2^e
        const double wmax = m[8];
        int e = 0;
        if (wmax > 0.0 && isfinite(wmax)) {
            (void)frexp(wmax, &e);  // wmax = f 2^e, f in [0.5, 1)
            e = std::max(e, kFixBits - 126);
        }
        g->inst.fix_scale = ldexpf(1.0f, kFixBits - e);
        g->inst.fix_inv = ldexpf(1.0f, e - kFixBits);
        g->plan_valid = false;
    }
    HIP_TRY(hipMemcpyAsync(g->at<double>(g->L.fel_state) + kN0, &g->N0, sizeof(double), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemsetAsync(g->at<uint32_t>(g->L.counters) + kRangeFlag, 0, sizeof(uint32_t), g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    *g->list.h_any = 0u;  // every copy of the old word has arrived
    g->has_density = true;
    g->bunch_valid = false;
    g->step = 0;
    return VP_OK;
}

int vp_get_density(vp_grid* g, float* w, int32_t on_device) {
    if (!g || !w) return fail(VP_EINVAL, "null argument");
    if (!g->has_density) return fail(VP_ESTATE, "no density set");
    const size_t bytes = (size_t)g->x.n * g->p.n * sizeof(float);
    HIP_TRY(hipMemcpyAsync(w, g->at<float>(g->parity ? g->L.w1 : g->L.w0), bytes,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream));
    int rc = g->list.post_range_copy();
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(g->stream));
    if (g->list.range_seen())
        return fail(VP_ERANGE, "a deposit cell sum exceeded 2^6 x 2^e (fixed-point range): the weights are not valid");
    return VP_OK;
}

int vp_step(vp_grid* g, double dt, int64_t nsteps) {
    if (!g) return fail(VP_EINVAL, "null grid");
    if (nsteps < 0) return fail(VP_EINVAL, "negative step count");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    if (g->list.range_seen())
        return fail(VP_ERANGE, "an earlier step left the deposit's fixed-point range; set a density again");
    int rc = prepare(g, dt);
    if (rc) return rc;
    if (nsteps == 0) return VP_OK;
    rc = g->list.run(nsteps, g->parity, g->use_graph);
    if (rc) return rc;
    g->parity = (int)((g->parity + nsteps) & 1);
    g->step += nsteps;
    return VP_OK;
}

int vp_step_timed(vp_grid* g, double dt, int64_t nsteps, double us[2]) {
    if (!g || !us) return fail(VP_EINVAL, "null argument");
    if (nsteps <= 0) return fail(VP_EINVAL, "need at least one step");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    int rc = prepare(g, dt);
    if (rc) return rc;
    rc = g->list.timed(nsteps, g->parity, us);
    if (rc) return rc;
    g->parity = (int)((g->parity + nsteps) & 1);
    g->step += nsteps;
    return VP_OK;
}

int vp_moments(vp_grid* g, vp_moments_t* out) {
    if (!g || !out) return fail(VP_EINVAL, "null argument");
    if (!g->has_density) return fail(VP_ESTATE, "no density set");
    int rc = launch_reduce_on(g, 0, 0.0);
    if (rc) return rc;
    double m[kMoments], st[kFelStateLen];
    uint32_t flags[4];
    HIP_TRY(hipMemcpyAsync(m, g->at<double>(g->L.moments), sizeof m, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(st, g->at<double>(g->L.fel_state), sizeof st, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(flags, g->at<uint32_t>(g->L.counters), sizeof flags, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    const double cell = spacing(g->x) * spacing(g->p);
    memset(out, 0, sizeof *out);
    out->sum_w = m[0];
    out->mass = cell * m[0];
    out->neg_mass = -cell * m[1];
    out->l1 = cell * m[2];
    out->entropy = -cell * m[3];
    out->mean_p = m[0] != 0.0 ? m[4] / m[0] : 0.0;
    out->energy = cell * m[5];
    out->step = g->step;
    out->nonfinite = (int64_t)m[9];
    if (g->has_ham && g->ham.kind == VP_H_FEL) {
        const double n0 = g->N0 != 0.0 ? g->N0 : 1.0;
        out->A_re = st[kA];
        out->A_im = st[kA + 1];
        out->bunch_re = m[6] / n0;
        out->bunch_im = m[7] / n0;
        out->fel_invariant = st[kA] * st[kA] + st[kA + 1] * st[kA + 1] + m[4] / n0;
    }
    if (out->nonfinite) return fail(VP_ENONFINITE, "%lld non-finite weights", (long long)out->nonfinite);
    if (flags[kRangeFlag])
        return fail(VP_ERANGE, "a deposit cell sum exceeded 2^6 x 2^e, max|w0| < 2^e (fixed-point range)");
    return VP_OK;
}

int vp_set_fixed_point(vp_grid* g, int32_t e) {
    if (!g) return fail(VP_EINVAL, "null grid");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    if (!g->has_density) return fail(VP_ESTATE, "set the density first (it picks the default exponent)");
    // the scale 2^(40 - e) and its inverse must be normal floats
    if (e < kFixBits - 126 || e > 127) return fail(VP_EINVAL, "fixed-point exponent %d outside [%d, 127]", e, kFixBits - 126);
    g->inst.fix_scale = ldexpf(1.0f, kFixBits - e);
    g->inst.fix_inv = ldexpf(1.0f, e - kFixBits);
    g->plan_valid = false;
    return VP_OK;
}

int vp_get_run_state(vp_grid* g, vp_run_state* out) {
    if (!g || !out) return fail(VP_EINVAL, "null argument");
    if (!g->has_density) return fail(VP_ESTATE, "no density set");
    double st[kFelStateLen];
    HIP_TRY(hipMemcpyAsync(st, g->at<double>(g->L.fel_state), sizeof st, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    memset(out, 0, sizeof *out);
    out->fix_exponent = kFixBits - ilogbf(g->inst.fix_scale);
    out->step = g->step;
    out->n0 = g->N0;
    out->bunch_dz = g->bunch_valid ? g->bunch_dz : NAN;
    static_assert(sizeof(out->fel) == sizeof st, "the FEL state fits the record");
    memcpy(out->fel, st, sizeof st);
    return VP_OK;
}

int vp_set_run_state(vp_grid* g, const vp_run_state* s) {
    if (!g || !s) return fail(VP_EINVAL, "null argument");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    if (!g->has_density) return fail(VP_ESTATE, "set the density first");
    const int32_t e = s->fix_exponent;
    if (e < kFixBits - 126 || e > 127) return fail(VP_EINVAL, "fixed-point exponent %d outside [%d, 127]", e, kFixBits - 126);
    for (double v : s->fel)
        if (!isfinite(v)) return fail(VP_EINVAL, "non-finite FEL state");
    if (!isfinite(s->n0) || s->step < 0) return fail(VP_EINVAL, "invalid normalisation or step");
    double st[kFelStateLen];
    memcpy(st, s->fel, sizeof st);
    st[kN0] = s->n0;
    HIP_TRY(hipMemcpyAsync(g->at<double>(g->L.fel_state), st, sizeof st, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->N0 = s->n0;
    g->inst.fix_scale = ldexpf(1.0f, kFixBits - e);
    g->inst.fix_inv = ldexpf(1.0f, e - kFixBits);
    g->step = s->step;
    g->bunch_valid = isfinite(s->bunch_dz);
    g->bunch_dz = g->bunch_valid ? s->bunch_dz : 0.0;
    g->plan_valid = false;
    return VP_OK;
}

int vp_set_basis(vp_grid* g, int32_t basis) {
    if (!g) return fail(VP_EINVAL, "null grid");
    if (basis < VP_BASIS_TENT || basis > VP_BASIS_CUBIC) return fail(VP_EINVAL, "unknown basis %d", basis);
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    // the deposit tile must still fit the LDS with the basis's border
    if (validate_tiles(basis, g->tiles) != VP_OK) g->tiles = default_tiles(g->x.n, g->p.n, basis);
    g->basis = basis;
    g->plan_valid = false;
    return VP_OK;
}

int vp_set_tiles(vp_grid* g, const vp_tiles* t) {
    if (!g || !t) return fail(VP_EINVAL, "null argument");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    vp_tiles n = g->tiles;
    if (t->k1_tx) n.k1_tx = t->k1_tx;
    if (t->k1_ty) n.k1_ty = t->k1_ty;
    if (t->k1_threads) n.k1_threads = t->k1_threads;
    int rc = validate_tiles(g->basis, n);
    if (rc) return rc;
    g->tiles = n;
    g->plan_valid = false;
    return VP_OK;
}

int vp_get_tiles(const vp_grid* g, vp_tiles* t) {
    if (!g || !t) return fail(VP_EINVAL, "null argument");
    *t = g->tiles;
    return VP_OK;
}

int vp_set_map_cache(vp_grid* g, int32_t on) {
    if (!g) return fail(VP_EINVAL, "null grid");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    g->use_map = on != 0;
    g->plan_valid = false;
    return VP_OK;
}

int vp_set_launch(vp_grid* g, int32_t use_graph) {
    if (!g) return fail(VP_EINVAL, "null grid");
    g->use_graph = use_graph != 0;
    return VP_OK;
}

int vp_autotune(vp_grid* g, double dt, double* best_us) {
    if (!g) return fail(VP_EINVAL, "null grid");
    if (g->in_batch) return fail(VP_ESTATE, "grid belongs to a live batch");
    int rc = prepare(g, dt);
    if (rc) return rc;
    // shape class: kind, half-octave buckets of the axis lengths and of the
    // largest displacement in cells
    const double hx = spacing(g->x), hp = spacing(g->p);
    const double disp = fabs(dt) * (std::max(fabs(g->p.lo), fabs(g->p.hi)) / hx + fabs(g->ham.a) / hp);
    const auto key = std::make_tuple((int)g->ham.kind, (int)lround(2.0 * log2((double)g->x.n)),
                                     (int)lround(2.0 * log2((double)g->p.n)), (long)lround(2.0 * log2(1.0 + disp)),
                                     g->basis);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && !best_us) {
            g->tiles = it->second;
            g->plan_valid = false;
            return prepare(g, dt);
        }
    }
    // save the state (weights, FEL scalars, parity, step) to restore afterwards
    const size_t n = (size_t)g->x.n * g->p.n;
    std::vector<float> saved(n);
    std::vector<double> saved_st(kFelStateLen);
    HIP_TRY(hipMemcpyAsync(saved.data(), g->at<float>(g->parity ? g->L.w1 : g->L.w0), n * 4, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipMemcpyAsync(saved_st.data(), g->at<double>(g->L.fel_state), kFelStateLen * 8, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    const int saved_parity = g->parity;
    const int64_t saved_step = g->step;
    const bool saved_graph = g->use_graph;
    Events ev(2);
    HIP_TRY(ev.create());
    hipEvent_t e0 = ev[0], e1 = ev[1];
    auto time_tiles = [&](const vp_tiles& t, float* us) -> int {
        if (validate_tiles(g->basis, t)) return VP_EINVAL;
        g->tiles = t;
        g->plan_valid = false;
        int r = prepare(g, dt);
        if (r) return r;
        // the fastest of three trials of eight steps: one trial alone varies by
        // ~2% between runs, enough to flip near-tied shapes
        const int reps = 8, trials = 3;
        r = g->list.run(2, g->parity, false);
        if (r) return r;
        *us = 1e30f;
        for (int k = 0; k < trials; ++k) {
            HIP_TRY(hipEventRecord(e0, g->stream));
            r = g->list.run(reps, g->parity, false);
            if (r) return r;
            HIP_TRY(hipEventRecord(e1, g->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            *us = std::min(*us, 1000.f * ms / reps);
        }
        return VP_OK;
    };
    const int k1c[][3] = {{64, 16, 256},  {64, 32, 256},  {64, 64, 256},  {128, 32, 256},   {64, 64, 512},
                          {128, 64, 512}, {128, 64, 640}, {128, 64, 768}, {128, 64, 1024}, {128, 128, 1024},
                          {256, 64, 1024}};
    vp_tiles best = g->tiles;
    float best_t = 1e30f;
    for (auto& c : k1c) {
        vp_tiles t = best;
        t.k1_tx = c[0];
        t.k1_ty = c[1];
        t.k1_threads = c[2];
        float us;
        // a candidate must beat the incumbent by 2%, so that near-ties (timing
        // noise) do not flip the choice from run to run
        if (time_tiles(t, &us) == VP_OK && us < 0.98f * best_t) { best_t = us; best = t; }
    }
    g->tiles = best;
    g->plan_valid = false;
    g->parity = saved_parity;
    g->step = saved_step;
    g->use_graph = saved_graph;
    HIP_TRY(hipMemcpyAsync(g->at<float>(g->parity ? g->L.w1 : g->L.w0), saved.data(), n * 4, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->at<double>(g->L.fel_state), saved_st.data(), kFelStateLen * 8, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->bunch_valid = false;
    rc = prepare(g, dt);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (best_us) *best_us = best_t;
    return VP_OK;
}

int vp_batch_create(vp_grid* const* grids, int32_t n, const double* dt, vp_batch** out) {
    if (!grids || !dt || !out || n <= 0) return fail(VP_EINVAL, "invalid batch arguments");
    *out = nullptr;
    hipStream_t s = grids[0] ? grids[0]->stream : nullptr;
    for (int k = 0; k < n; ++k) {
        if (!grids[k]) return fail(VP_EINVAL, "null grid %d", k);
        if (grids[k]->in_batch) return fail(VP_ESTATE, "grid %d already belongs to a batch", k);
        if (grids[k]->stream != s) return fail(VP_EINVAL, "grid %d is on another stream than grid 0", k);
        if (grids[k]->basis != grids[0]->basis)
            return fail(VP_EUNSUPPORTED, "grid %d has another basis than grid 0 (a batch runs one basis)", k);
        for (int q = 0; q < k; ++q)
            if (grids[q] == grids[k]) return fail(VP_EINVAL, "grid %d listed twice", k);
    }
    for (int k = 0; k < n; ++k) {
        int rc = prepare(grids[k], dt[k]);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(grids[k]->stream));
    }
    vp_batch* b = new vp_batch();
    b->grids.assign(grids, grids + n);
    b->dt.assign(dt, dt + n);
    LaunchList& L = b->list;
    L.stream = s;
    L.ninst = n;
    hipError_t e = hipMalloc(&L.d_inst, sizeof(VpInst) * n);
    // tile offsets of both kernels, then the batch's range word
    if (e == hipSuccess) e = hipMalloc(&L.d_off1, sizeof(int32_t) * (2 * (n + 1) + 1));
    L.d_off2 = L.d_off1 + (n + 1);
    L.d_any = reinterpret_cast<uint32_t*>(L.d_off2 + (n + 1));
    if (e == hipSuccess && alloc_host_flag(&L.h_any) != VP_OK) e = hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMemsetAsync(L.d_any, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int rc = e == hipSuccess ? fill_batch(b) : fail(VP_EHIP, "batch setup: %s", hipGetErrorString(e));
    if (rc) {
        (void)hipFree(L.d_inst);
        (void)hipFree(L.d_off1);
        free_host_flag(&L.h_any);
        delete b;
        return rc;
    }
    for (auto* g : b->grids) g->in_batch = true;
    *out = b;
    return VP_OK;
}

int vp_batch_autotune(vp_batch* b, double* best_us) {
    if (!b) return fail(VP_EINVAL, "null batch");
    LaunchList& L = b->list;
    const int n = (int)b->grids.size();
    // composition class: the multiset of (kind, basis, half-octave axis lengths)
    std::vector<std::tuple<int, int, int, int>> comp;
    for (auto* g : b->grids)
        comp.emplace_back((int)g->ham.kind, g->basis, (int)lround(2.0 * log2((double)g->x.n)),
                          (int)lround(2.0 * log2((double)g->p.n)));
    std::sort(comp.begin(), comp.end());
    // candidates: every grid keeps its own shape (as planned), or every grid
    // takes one shape (cut to the lattice); each with one workgroup per tile
    // or a persistent launch (as many workgroups as fit the device at once,
    // looping over the tiles)
    const int shapes[][3] = {{0, 0, 0}, {64, 32, 256}, {64, 64, 256}, {128, 32, 256}, {128, 64, 512}, {128, 64, 1024},
                             {128, 128, 1024}};
    constexpr int kShapes = sizeof(shapes) / sizeof(shapes[0]);
    auto apply = [&](int si, bool persistent, const std::vector<vp_tiles>& own) -> int {
        for (int k = 0; k < n; ++k) {
            vp_grid* g = b->grids[k];
            vp_tiles t = own[k];
            if (si > 0) {
                t = vp_tiles{shapes[si][0], shapes[si][1], shapes[si][2]};
                if (validate_tiles(g->basis, t) != VP_OK) t = own[k];
            }
            g->tiles = t;
            g->plan_valid = false;
            int rc = prepare(g, b->dt[k]);
            if (rc) return rc;
        }
        int rc = fill_batch(b);
        if (rc) return rc;
        L.grid1 = 0;
        if (persistent) {
            int dev = 0, cus = 0, per = 0;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, deposit_kernel(L.basis), L.threads1, L.lds1));
            L.grid1 = std::max(1, cus * per);
        }
        return VP_OK;
    };
    std::vector<vp_tiles> own(n);
    for (int k = 0; k < n; ++k) own[k] = b->grids[k]->tiles;
    using Key = std::vector<std::tuple<int, int, int, int>>;
    static std::mutex mu;
    static std::map<Key, std::pair<int, bool>> cache;
    if (!best_us) {
        std::pair<int, bool> choice;
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cache.find(comp);
            if (it == cache.end()) return fail(VP_ESTATE, "no tuned choice for this batch composition yet");
            choice = it->second;
        }
        return apply(choice.first, choice.second, own);
    }
    // save the states (weights and FEL scalars) to restore after timing
    size_t bytes = 0;
    std::vector<size_t> at(n);
    for (int k = 0; k < n; ++k) {
        at[k] = bytes;
        bytes += align_up((size_t)b->grids[k]->x.n * b->grids[k]->p.n * 4) + kFelStateLen * 8;
    }
    char* save = nullptr;
    HIP_TRY(hipMalloc(&save, bytes));
    auto copy_states = [&](bool to_save) -> int {
        for (int k = 0; k < n; ++k) {
            vp_grid* g = b->grids[k];
            const size_t wb = (size_t)g->x.n * g->p.n * 4;
            char* w = reinterpret_cast<char*>(g->at<float>(g->parity ? g->L.w1 : g->L.w0));
            char* st = reinterpret_cast<char*>(g->at<double>(g->L.fel_state));
            char* sw = save + at[k];
            char* ss = save + at[k] + align_up(wb);
            HIP_TRY(hipMemcpyAsync(to_save ? sw : w, to_save ? w : sw, wb, hipMemcpyDeviceToDevice, L.stream));
            HIP_TRY(hipMemcpyAsync(to_save ? ss : st, to_save ? st : ss, kFelStateLen * 8, hipMemcpyDeviceToDevice,
                                   L.stream));
        }
        return VP_OK;
    };
    int rc = copy_states(true);
    Events ev(2);
    if (rc == VP_OK && ev.create() != hipSuccess) rc = fail(VP_EHIP, "hipEventCreate failed");
    double best = 1e300;
    int best_si = 0;
    bool best_p = false;
    for (int si = 0; si < kShapes && rc == VP_OK; ++si)
        for (int pers = 0; pers < 2 && rc == VP_OK; ++pers) {
            rc = apply(si, pers != 0, own);
            if (rc) break;
            // the fastest of three trials of eight steps (even: the grids'
            // parities come back), as for one grid
            const int reps = 8, trials = 3;
            rc = L.run(2, 0, false);
            if (rc) break;
            double us = 1e300;
            for (int k = 0; k < trials && rc == VP_OK; ++k) {
                if (hipEventRecord(ev[0], L.stream) != hipSuccess) { rc = fail(VP_EHIP, "hipEventRecord"); break; }
                rc = L.run(reps, 0, false);
                if (rc) break;
                float ms = 0.f;
                if (hipEventRecord(ev[1], L.stream) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                    hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
                    rc = fail(VP_EHIP, "batch timing events");
                    break;
                }
                us = std::min(us, 1000.0 * ms / reps);
            }
            if (rc) break;
            // a candidate must beat the incumbent by 2% (timing noise)
            if (us < 0.98 * best) {
                best = us;
                best_si = si;
                best_p = pers != 0;
            }
            rc = copy_states(false);
        }
    if (rc == VP_OK) rc = copy_states(false);
    if (rc == VP_OK) rc = apply(best_si, best_p, own);
    (void)hipStreamSynchronize(L.stream);
    (void)hipFree(save);
    if (rc) return rc;
    for (auto* g : b->grids) g->bunch_valid = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        cache[comp] = {best_si, best_p};
    }
    *best_us = best;
    return VP_OK;
}

int vp_batch_config(const vp_batch* b, int32_t* deposit_grid, int32_t* deposit_threads, int32_t* tiles) {
    if (!b || !deposit_grid || !deposit_threads || !tiles) return fail(VP_EINVAL, "null argument");
    *deposit_grid = b->list.grid1;
    *deposit_threads = b->list.threads1;
    *tiles = b->list.total1;
    return VP_OK;
}

int vp_batch_step(vp_batch* b, int64_t nsteps) {
    if (!b) return fail(VP_EINVAL, "null batch");
    if (nsteps < 0) return fail(VP_EINVAL, "negative step count");
    if (b->list.range_seen())
        return fail(VP_ERANGE, "a deposit cell sum of a batched grid left the fixed-point range "
                               "(vp_moments names the grid)");
    if (nsteps == 0) return VP_OK;
    int rc = b->list.run(nsteps, (int)(b->steps_done & 1), true);
    if (rc) return rc;
    b->steps_done += nsteps;
    for (auto* g : b->grids) {
        g->parity = (int)((g->parity + nsteps) & 1);
        g->step += nsteps;
    }
    return VP_OK;
}

int vp_batch_step_timed(vp_batch* b, int64_t nsteps, double us[2]) {
    if (!b || !us) return fail(VP_EINVAL, "null argument");
    if (nsteps <= 0) return fail(VP_EINVAL, "need at least one step");
    if (b->list.range_seen())
        return fail(VP_ERANGE, "a deposit cell sum of a batched grid left the fixed-point range "
                               "(vp_moments names the grid)");
    int rc = b->list.timed(nsteps, (int)(b->steps_done & 1), us);
    if (rc) return rc;
    b->steps_done += nsteps;
    for (auto* g : b->grids) {
        g->parity = (int)((g->parity + nsteps) & 1);
        g->step += nsteps;
    }
    return VP_OK;
}

int vp_batch_destroy(vp_batch* b) {
    if (!b) return VP_OK;
    (void)hipStreamSynchronize(b->list.stream);
    b->list.drop_graphs();
    (void)hipFree(b->list.d_inst);
    (void)hipFree(b->list.d_off1);
    free_host_flag(&b->list.h_any);
    for (auto* g : b->grids) g->in_batch = false;
    delete b;
    return VP_OK;
}

int vp_step_noalloc(const vp_axis* x, const vp_axis* p, const vp_hamiltonian* h, int32_t basis, double dt,
                    int64_t nsteps, const float* w_in, float* w_out, double fel_n0, double* fel_A, int32_t* status,
                    void* stream) {
    if (!x || !p || !h || !w_in || !w_out) return fail(VP_EINVAL, "null argument");
    if (!axis_ok(x) || !axis_ok(p)) return fail(VP_EINVAL, "invalid axis (need n >= 4, hi > lo, finite)");
    if (p->periodic) return fail(VP_EUNSUPPORTED, "the momentum axis must be open");
    if (h->kind < VP_H_FREE || h->kind > VP_H_FEL) return fail(VP_EINVAL, "unknown Hamiltonian kind %d", h->kind);
    if (!isfinite(h->a) || !isfinite(h->omega) || !isfinite(h->fel_delta) || !isfinite(h->fel_sigma2))
        return fail(VP_EINVAL, "non-finite Hamiltonian parameter");
    if (h->kind == VP_H_SHO_EXACT && x->periodic) return fail(VP_EUNSUPPORTED, "the exact rotation needs an open x axis");
    if (h->integrator != VP_FEL_DKD && !(h->kind == VP_H_FEL && h->integrator == VP_FEL_RK4))
        return fail(VP_EINVAL, "integrator %d: only the FEL takes VP_FEL_RK4", h->integrator);
    if (basis < VP_BASIS_TENT || basis > VP_BASIS_CUBIC) return fail(VP_EINVAL, "unknown basis %d", basis);
    if (!isfinite(dt)) return fail(VP_EINVAL, "dt must be finite");
    if (step_too_large(*x, *p, *h, dt)) return fail(VP_EINVAL, "dt %g moves nodes by more than 2^20 cells per step", dt);
    if (nsteps < 0) return fail(VP_EINVAL, "negative step count");
    const bool fel = h->kind == VP_H_FEL;
    if (fel && (!fel_A || !(fel_n0 != 0.0) || !isfinite(fel_n0)))
        return fail(VP_ESTATE, "the FEL needs its field (fel_A) and a nonzero finite N0");
    const int nx = x->n, np = p->n;
    if ((long)nx * np > kNoAllocMaxNodes)
        return fail(VP_ENOMEM, "%d x %d nodes: the allocation-free step takes at most %ld", nx, np, kNoAllocMaxNodes);
    const Layout L = layout(nx, np);
    const size_t need = L.boxes - L.b;  // b .. the moments: everything but the state and the host boxes
    if (need > kNoAllocScratchBytes)
        return fail(VP_ENOMEM, "%zu bytes of scratch needed, %zu available", need, kNoAllocScratchBytes);
    raise_lds_limit();
    hipError_t e = hipSuccess;
    char* scr = static_cast<char*>(noalloc_scratch(&e));
    if (!scr) return fail(VP_EHIP, "scratch address: %s", hipGetErrorString(e));
    auto at = [&](size_t off) { return scr + (off - L.b); };
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // the descriptor of a grid of this shape, as upload_inst builds it, with
    // the state in w_out (read and written in place: the deposit reads it into
    // b, the solve writes it back) and the source boxes planned in the kernel
    VpInst I{};
    I.push = push_params(*x, *p, *h, dt, basis);
    vp_tiles t = default_tiles(nx, np, basis);
    t.k1_tx = std::min(t.k1_tx, nx);
    t.k1_ty = std::min(t.k1_ty, np);
    I.k1_tx = t.k1_tx;
    I.k1_ty = t.k1_ty;
    I.k1_tiles_x = (nx + t.k1_tx - 1) / t.k1_tx;
    I.k1_tiles = I.k1_tiles_x * ((np + t.k1_ty - 1) / t.k1_ty);
    I.k2_tiles = solve_tiles(nx, np, basis);
    I.fel_kick = -2.0 * dt / spacing(*p);
    I.fel_sigma2 = (float)h->fel_sigma2;
    I.fel_dz = dt;
    I.w[0] = I.w[1] = w_out;
    I.b = reinterpret_cast<float*>(at(L.b));
    I.tab_x = reinterpret_cast<float4*>(at(L.tab_x));
    I.tab_p = reinterpret_cast<float4*>(at(L.tab_p));
    I.fel_ex = reinterpret_cast<double2*>(at(L.fel_ex));
    I.fel_eq = reinterpret_cast<double2*>(at(L.fel_eq));
    I.fel_state = reinterpret_cast<double*>(at(L.fel_state));
    I.partials = reinterpret_cast<double*>(at(L.partials));
    I.counters = reinterpret_cast<uint32_t*>(at(L.counters));
    I.boxes = nullptr;
    NoAllocSetup S{};
    S.inst = I;
    S.inst_out = reinterpret_cast<VpInst*>(at(L.inst));
    S.off_out = reinterpret_cast<int32_t*>(at(L.off));
    S.tables = table_params(*x, *p, *h, dt);
    S.tab_x = const_cast<float4*>(I.tab_x);
    S.tab_p = const_cast<float4*>(I.tab_p);
    S.fel_ex = const_cast<double2*>(I.fel_ex);
    S.fel_eq = const_cast<double2*>(I.fel_eq);
    S.fel_state = I.fel_state;
    S.counters = I.counters;
    S.fel_A = fel ? fel_A : nullptr;
    S.n0 = fel ? fel_n0 : 0.0;
    double* moments = reinterpret_cast<double*>(at(L.moments));

    const size_t bytes = (size_t)nx * np * sizeof(float);
    if (w_out != w_in) HIP_TRY(hipMemcpyAsync(w_out, w_in, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_noalloc_setup(S, nx, np, s));
    ReduceArgs R{};
    R.w = w_out;
    R.nx = nx;
    R.np = np;
    R.kind = h->kind;
    R.mode = 2;
    R.x_lo = x->lo;
    R.hx = spacing(*x);
    R.p_lo = p->lo;
    R.hp = spacing(*p);
    R.inv_n0 = fel ? 1.0 / fel_n0 : 0.0;
    R.fel_ex = I.fel_ex;
    R.fel_eq = I.fel_eq;
    R.partials = I.partials;
    R.counter = I.counters + 1;
    R.out = moments;
    R.dz = dt;
    HIP_TRY(launch_reduce(R, s));
    HIP_TRY(launch_noalloc_scale(S.inst_out, moments, s));
    if (fel) {  // the bunching of the starting state at the half-drift phases
        R.mode = 1;
        R.out = I.fel_state;
        HIP_TRY(launch_reduce(R, s));
    }
    LaunchList LL;
    LL.d_inst = S.inst_out;
    LL.d_off1 = S.off_out;
    LL.d_off2 = S.off_out + 2;
    LL.d_any = I.counters + kRangeFlag;
    LL.ninst = 1;
    LL.total1 = I.k1_tiles;
    LL.total2 = I.k2_tiles;
    LL.has_fel = fel;
    LL.has_rk4 = fel && h->integrator == VP_FEL_RK4;
    LL.basis = basis;
    LL.solve = solve_kind(basis, nx, np, x->periodic != 0);
    LL.lds1 = deposit_lds_bytes(t.k1_tx, t.k1_ty, basis);
    LL.threads1 = t.k1_threads;
    LL.fuse_stage = stage_fusable(LL);
    LL.stream = s;
    for (int64_t k = 0; k < nsteps; ++k) {
        int rc = LL.enqueue_step((int)(k & 1));
        if (rc) return rc;
    }
    HIP_TRY(launch_noalloc_finish(moments, I.fel_state, I.counters, fel ? fel_A : nullptr, status, s));
    return VP_OK;
}

const char* vp_status_string(int s) {
    switch (s) {
    case VP_OK: return "ok";
    case VP_EINVAL: return "invalid argument";
    case VP_ENOMEM: return "workspace missing or too small";
    case VP_ESTATE: return "call out of order";
    case VP_EHIP: return "HIP runtime error";
    case VP_EUNSUPPORTED: return "unsupported configuration";
    case VP_ENONFINITE: return "non-finite state";
    case VP_ERANGE: return "deposit fixed-point range exceeded";
    default: return "unknown status";
    }
}

const char* vp_last_error(void) { return g_err; }

int vp_plan_source_box(const vp_axis* x, const vp_axis* p, const vp_hamiltonian* h, int32_t basis, double dt,
                       double kick_re, double kick_im, int32_t bx0, int32_t bx1, int32_t by0, int32_t by1,
                       int32_t box[4]) {
    if (!axis_ok(x) || !axis_ok(p) || !h || !box) return fail(VP_EINVAL, "invalid argument");
    if (basis < VP_BASIS_TENT || basis > VP_BASIS_CUBIC) return fail(VP_EINVAL, "unknown basis %d", basis);
    PushParams P = push_params(*x, *p, *h, dt, basis, kick_re, kick_im);
    int b[4];
    source_box(P, bx0, bx1, by0, by1, b);
    for (int k = 0; k < 4; ++k) box[k] = b[k];
    return VP_OK;
}

}  // extern "C"
