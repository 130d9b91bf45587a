// vp_internal.h -- data layout shared by the host runtime and the gfx950 kernels of libvp.
//
// One step of the method (Edelen & Webb, Sec. "An Algorithm Based on Phase
// Space Density Conservation", eqs. 6-10) runs as two kernels (plus, for the
// FEL, a one-workgroup field update, k_fel_field):
//   k_deposit: every lattice node is pushed (its position is its index, so
//              nothing but w is read) and its weight is scattered onto the
//              4x4 lattice taps of its moved tent with cubic B-spline weights
//              (the tent-tent overlap of eq. 9).  A workgroup owns one
//              destination tile held in LDS and scans the box of source nodes
//              that can reach it; the tile is written to b once.
//   k_solve:   w_out = (M_x^{-1} (x) M_p^{-1}) b, the tent mass matrix of
//              eq. 8, M = tridiag(1/6, 2/3, 1/6), cyclic on a periodic axis.  A
//              wavefront owns a 32x64 output tile and solves the 64x96 window
//              around it (a 16-node halo per side makes the tile independent of
//              its neighbours to within (2-sqrt 3)^16 ~ 7e-10), columns then
//              rows, one line per lane.  For the FEL its epilogue also forms
//              the FP64 bunching partials of the new state, which k_fel_field
//              sums to advance the FEL field.
// With quadratic or cubic B-spline basis functions in place of tents (the
// smoother basis the paper's discussion proposes) the overlaps are B-splines
// of degree 5 or 7: k_deposit scatters 6x6 or 8x8 taps per node, and
// k_solve_spline solves the banded mass matrix ((1/120)[1, 26, 66, 26, 1] or
// (1/5040)[1, 120, 1191, 2416, 1191, 120, 1]) along both axes.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#ifndef __HIP_DEVICE_COMPILE__
#include <cmath>
#endif

namespace vp {

enum Kind : int32_t { kFree = 0, kSho = 1, kPendulum = 2, kFel = 3 };

constexpr int kHalo = 16;         // warm-up nodes on each side of a solve tile
constexpr int kEdge = 32;         // nodes from an open edge whose LU coefficients are tabulated
constexpr int kPad = 4;           // trash border of a deposit tile (per side)
constexpr int kFixBits = 40;      // deposit cell sums: 64-bit fixed point at 2^-40 of 2^e > max|w0|
constexpr int kDepositMaxThreads = 1024;  // deposit workgroup: a multiple of 64 up to this
// The cubic basis's deposit is compiled for at most 768 threads per workgroup:
// its row pairs' taps then fit the registers (158 VGPRs) without spilling.
constexpr int kDepositCubicThreads = 768;
constexpr int kSegX = 32;                  // solve tile: kSegX columns by kSegP rows (kept nodes)
constexpr int kSegP = 64;
constexpr int kLineX = kSegX + 2 * kHalo;  // window line along x: the kept segment plus both halos
constexpr int kLineP = kSegP + 2 * kHalo;  // window line along p
constexpr int kSolveThreads = 64;          // solve: one wavefront (a window column, then a kept row, per lane)
constexpr int kFieldThreads = 256;       // FEL field update: one workgroup per instance
constexpr int kStageThreads = 256;       // FEL Runge-Kutta stage sums: four wavefronts per solve tile
constexpr int kStageFuseTiles = 1024;    // FEL Runge-Kutta: a single grid's deposit sums the stage partials up to this many solve tiles
constexpr int kReduceBlocks = 256;
constexpr int kReduceThreads = 256;
constexpr int kMoments = 10;      // FP64 sums produced by the reduction kernel

// Basis functions of the expansion: tents (eq. 4), or B-splines of degree 2 or
// 3 (degree = basis + 1; the overlaps reach `basis` cells further than tents).
enum Basis : int32_t { kBasisTent = 0, kBasisQuadratic = 1, kBasisCubic = 2 };
constexpr int kPadQ = 6;          // quadratic basis: trash border of a deposit tile (5 taps past it, even for alignment)
constexpr int kPadC = 8;          // cubic basis: the same for 7 taps past it
constexpr int kLineQ = 128;       // spline bases: window line of a solve tile (both axes)
constexpr int kPitchQ = kLineQ + 1;         // LDS row pitch of the window (odd: rows and columns are conflict-free)
constexpr int kSolveQThreads = kLineQ;      // one window line per thread
constexpr int kEdgeQ = 24;        // nodes from an open edge whose LDL^T coefficients are tabulated
// warm-up nodes per side of a solve tile, by band (2: quadratic, 3: cubic):
// the slowest decay of the inverse mass matrix, 0.4306 and 0.5353 per node,
// reaches ~1.6e-9 over the halo
constexpr int spline_halo(int band) { return band == 2 ? 24 : 34; }
constexpr int spline_seg(int band) { return kLineQ - 2 * spline_halo(band); }  // kept nodes per axis
constexpr int kHaloQ = spline_halo(2), kSegQ = spline_seg(2);  // quadratic: 80 x 80 tiles
constexpr int kHaloC = spline_halo(3), kSegC = spline_seg(3);  // cubic: 60 x 60 tiles

// Parameters of the push in cell units and of the source-box bound.
//  FREE / PENDULUM / FEL: node (i, j) moves by
//     dv = alpha cos(phi_i + q_j) + beta sin(phi_i + q_j)
//     du = drift_j + kd * dv
//  with phi_i = x_lo + i hx, q_j = q0 + j q1, drift_j = drift0 + j drift1.
//  SHO: (x, p) -> (x c + p s, -x s + p c).
struct PushParams {
    int32_t kind;
    int32_t nx, np, x_periodic;
    float x_lo, hx, p_lo, hp;
    float drift0, drift1;
    float q0, q1;
    float alpha, beta;
    float kd;
    float c, s;
    int32_t rk4;  // FEL by Runge-Kutta (the deposit reads its stage constants; alpha bounds |dv|)
    int32_t wide; // the basis (Basis): its overlaps reach `wide` cells further than tents (4 + 2 wide taps per axis)
};

__host__ __device__ inline float vp_floor(float v) {
#ifdef __HIP_DEVICE_COMPILE__
    return floorf(v);
#else
    return std::floor(v);
#endif
}
__host__ __device__ inline float vp_sin(float v) {
#ifdef __HIP_DEVICE_COMPILE__
    return sinf(v);
#else
    return std::sin(v);
#endif
}

// Range [lo, hi] of sin over the interval [a, b], a <= b.
__host__ __device__ inline void sin_range(float a, float b, float* lo, float* hi) {
    const float two_pi = 6.28318530717958647f, half_pi = 1.57079632679489662f;
    if (!(b - a < two_pi)) {
        *lo = -1.0f;
        *hi = 1.0f;
        return;
    }
    float sa = vp_sin(a), sb = vp_sin(b);
    float l = sa < sb ? sa : sb, h = sa < sb ? sb : sa;
    float kmax = vp_floor((b - half_pi) / two_pi);  // largest k with pi/2 + 2k pi <= b
    if (half_pi + two_pi * kmax >= a) h = 1.0f;
    float kmin = vp_floor((b + half_pi) / two_pi);  // largest k with -pi/2 + 2k pi <= b
    if (-half_pi + two_pi * kmin >= a) l = -1.0f;
    // guard against rounding of the endpoint values
    *lo = l - 1e-6f;
    *hi = h + 1e-6f;
}

// Push tables of one step, formed in FP64 and stored as the kernels read them
// (the host planner and the allocation-free entry point's device set-up use
// the same code).  Column i, tab_x: sin and cos of x_i, or for the exact
// rotation the x terms of the displacement in cells as hi + lo float pairs;
// fel_ex: e^{i x_i} in FP64.  Row j, tab_p: the drift p_j dt / h_x in cells as
// a hi + lo pair and sin, cos of the half-drift phase q_j = (delta + p_j) dt/2
// (rotation: the p terms as pairs); fel_eq: e^{i q_j} in FP64.
struct TableParams {
    int32_t kind;
    double x_lo, hx, p_lo, hp, dt, delta, omega;
};
__host__ __device__ inline void split_pair(double v, float& hi, float& lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
}
__host__ __device__ inline void table_x(const TableParams& T, int i, float4& tx, double2& ex) {
    const double x = T.x_lo + i * T.hx;
    if (T.kind == kSho) {
        const double th = T.omega * T.dt, s = sin(th), cm1 = -2.0 * sin(0.5 * th) * sin(0.5 * th);
        split_pair(x * cm1 / T.hx, tx.x, tx.y);
        split_pair(-x * s / T.hp, tx.z, tx.w);
        ex = make_double2(0.0, 0.0);
    } else {
        tx = make_float4((float)sin(x), (float)cos(x), 0.f, 0.f);
        ex = make_double2(cos(x), sin(x));
    }
}
__host__ __device__ inline void table_p(const TableParams& T, int j, float4& tp, double2& eq) {
    const double p = T.p_lo + j * T.hp;
    if (T.kind == kSho) {
        const double th = T.omega * T.dt, s = sin(th), cm1 = -2.0 * sin(0.5 * th) * sin(0.5 * th);
        split_pair(p * s / T.hx, tp.x, tp.y);
        split_pair(p * cm1 / T.hp, tp.z, tp.w);
        eq = make_double2(0.0, 0.0);
    } else {
        const double v = T.delta + p;  // drift velocity of row j
        const double q = 0.5 * T.dt * v;
        split_pair(v * T.dt / T.hx, tp.x, tp.y);
        tp.z = (float)sin(q);
        tp.w = (float)cos(q);
        eq = make_double2(cos(q), sin(q));
    }
}

__host__ __device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__host__ __device__ inline int ifloor(float v) { return (int)vp_floor(v); }
__host__ __device__ inline int iceil(float v) { return -(int)vp_floor(-v); }

// Box of source nodes [x0,x1) x [y0,y1) (columns unwrapped on a periodic axis)
// whose moved basis functions can deposit into destination columns [bx0,bx1)
// and rows [by0,by1).  A moved tent at cell position (u, v) touches columns
// floor(u)-1 .. floor(u)+2, so it reaches the tile only if u in
// [bx0-2, bx1+1) and v in [by0-2, by1+1) (a quadratic basis function, columns
// floor(u)-2 .. floor(u)+3: one cell more on each side).  The displacement is
// bounded by interval arithmetic over the candidate box, then the bound is
// tightened once with the phase range of that box.  Each end of the column
// range carries a margin of 1e-3 cells plus 2^-20 of the magnitudes involved,
// for the FP32 rounding of this bound and of the push.  The row range keeps
// two more cells per side: rows as tight as the columns were measured no
// faster with 128-row tiles and 10-14% slower with 32-row tiles (the cause,
// in the scheduling of the four-row work units, is not established).
__host__ __device__ inline float box_margin(float a, float b) {
    return 1e-3f + 9.5367431640625e-7f * ((a < 0 ? -a : a) + (b < 0 ? -b : b));
}
__host__ __device__ inline void source_box(const PushParams& P, int bx0, int bx1, int by0, int by1,
                                           int box[4]) {
    const float reach = (float)P.wide;
    const float ulo = (float)bx0 - 2.0f - reach, uhi = (float)bx1 + 1.0f + reach;
    const float vlo = (float)by0 - 3.0f - reach, vhi = (float)by1 + 2.0f + reach;
    int x0, x1, y0, y1;
    if (P.kind == kSho) {
        // preimage of the dest rectangle under the rotation: rotate its corners back
        float X[2] = {P.x_lo + ulo * P.hx, P.x_lo + uhi * P.hx};
        float Pm[2] = {P.p_lo + vlo * P.hp, P.p_lo + vhi * P.hp};
        float xmn = 3.4e38f, xmx = -3.4e38f, pmn = 3.4e38f, pmx = -3.4e38f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                float x = X[a] * P.c - Pm[b] * P.s, p = X[a] * P.s + Pm[b] * P.c;
                xmn = x < xmn ? x : xmn;
                xmx = x > xmx ? x : xmx;
                pmn = p < pmn ? p : pmn;
                pmx = p > pmx ? p : pmx;
            }
        x0 = ifloor((xmn - P.x_lo) / P.hx) - 1;
        x1 = iceil((xmx - P.x_lo) / P.hx) + 2;
        y0 = ifloor((pmn - P.p_lo) / P.hp) - 1;
        y1 = iceil((pmx - P.p_lo) / P.hp) + 2;
    } else {
        float R = P.kind == kFree ? 0.0f : sqrtf(P.alpha * P.alpha + P.beta * P.beta);
        float dvmin = -R, dvmax = R;
        x0 = x1 = y0 = y1 = 0;
        for (int pass = 0; pass < 2; ++pass) {
            y0 = ifloor(vlo - dvmax) - 1;
            y1 = iceil(vhi - dvmin) + 1;
            y0 = y0 < 0 ? 0 : y0;
            y1 = y1 > P.np ? P.np : y1;
            if (y1 <= y0) break;
            float da = P.drift0 + (float)y0 * P.drift1, db = P.drift0 + (float)(y1 - 1) * P.drift1;
            float dmin = da < db ? da : db, dmax = da < db ? db : da;
            float va = dvmax > -dvmin ? dvmax : -dvmin;
            float kk = P.kd < 0 ? -P.kd : P.kd;
            float umin = dmin - kk * va, umax = dmax + kk * va;
            x0 = iceil(ulo - umax - box_margin(ulo, umax));
            x1 = iceil(uhi - umin + box_margin(uhi, umin));
            // (the Runge-Kutta push has no single phase to tighten with)
            if (pass == 1 || R == 0.0f || P.rk4) break;
            // tighten dv with the phase range phi + q over the candidate box
            float qa = P.q0 + (float)y0 * P.q1, qb = P.q0 + (float)(y1 - 1) * P.q1;
            float qmin = qa < qb ? qa : qb, qmax = qa < qb ? qb : qa;
            float th0 = atan2f(P.alpha, P.beta);  // dv = R sin(phi + q + th0)
            float pa = P.x_lo + (float)x0 * P.hx + qmin + th0;
            float pb = P.x_lo + (float)(x1 - 1) * P.hx + qmax + th0;
            float slo, shi;
            sin_range(pa, pb, &slo, &shi);
            dvmin = R * slo;
            dvmax = R * shi;
        }
    }
    if (!P.x_periodic) {
        x0 = x0 < 0 ? 0 : x0;
        x1 = x1 > P.nx ? P.nx : x1;
    }
    y0 = y0 < 0 ? 0 : y0;
    y1 = y1 > P.np ? P.np : y1;
    if (x1 < x0) x1 = x0;
    if (y1 < y0) y1 = y0;
    box[0] = x0;
    box[1] = x1;
    box[2] = y0;
    box[3] = y1;
}

// One grid instance as the kernels see it.  A single grid is a batch of one.
struct VpInst {
    PushParams push;
    int32_t k1_tx, k1_ty, k1_tiles_x, k1_tiles;
    int32_t k2_tiles;        // solve tiles: kSegX x kSegP nodes
    int32_t pad2;
    int32_t parity0;         // index of the current state buffer when the launch list was built
    int32_t pad0;
    float fix_scale, fix_inv;  // deposit fixed-point scale 2^(40-e), max|w0| < 2^e, and its inverse
    float fel_sigma2;
    float pad1;
    double fel_kick;           // -2 dz / h_eta (cells per unit field), FP64: the field coupling
    double fel_dz;
    float* w[2];
    float* b;
    const float4* tab_x;     // per column push table
    const float4* tab_p;     // per row push table
    const double2* fel_ex;   // (cos phi_i, sin phi_i)
    const double2* fel_eq;   // (cos q_j, sin q_j), q_j the half drift of row j
    double* fel_state;       // [A_re, A_im, b_re, b_im, N0, dz_b, ...]
    double* partials;        // per solve tile: bunching partial (re, im)
    uint32_t* counters;      // [1]: reduction, [kRangeFlag]: deposit range
    const int4* boxes;       // per deposit tile: source box (x0, x1, y0, y1) planned on the host,
                             // or null: the deposit plans it (the FEL kick depends on the field)
    float2* map_f;           // cached push of a static Hamiltonian (k_map): fractions (fu, fv) per
    int32_t* map_k;          // node, whole cells ku | kv << 16; null: the deposit pushes
};

// Host-planned source boxes: room for one per deposit tile of 32 x 16 nodes
// (smaller tiles plan their boxes in the kernel).
constexpr int kBoxTileX = 32, kBoxTileY = 16;
inline size_t box_capacity(int nx, int np) {
    return (size_t)((nx + kBoxTileX - 1) / kBoxTileX) * ((np + kBoxTileY - 1) / kBoxTileY);
}

constexpr int kRangeFlag = 2;  // counters slot set when a deposit cell sum leaves half its range

// fel_state slots
//   A: field; Bn: bunching at the half-drift phases (the exact-kick step's,
//   and the Runge-Kutta step's stage 2); B1, B3, B4: the Runge-Kutta stages'
//   bunchings at the lattice phases and at stages 3 and 4; An: the field after
//   the Runge-Kutta step in progress
enum { kA = 0, kBn = 2, kN0 = 4, kDzB = 5, kB1 = 6, kB3 = 8, kB4 = 10, kAn = 12, kFelStateLen = 16 };
constexpr int kPartialsPerTile = 4;  // per solve tile: two complex FP64 bunching sums

struct LaunchArgs {
    const VpInst* inst;
    const int32_t* off;  // [ninst+1] exclusive prefix of tile counts
    int32_t ninst;
    int32_t total;
    int32_t parity;      // step parity relative to each instance's parity0
    int32_t mode;        // k_fel_field: 0 after the solve, 1 after the Runge-Kutta stage sums
    uint32_t* any_range; // set (with the instance's own flag) by a deposit cell out of range:
                         // one word for the whole launch list, polled by the host
};

struct ReduceArgs {
    const float* w;
    int32_t nx, np, kind, mode;   // mode 0: moments, 1: FEL bunching, 2: sum, max|w| and non-finite count
    double x_lo, hx, p_lo, hp, a;
    double inv_n0;
    const double2* fel_ex;
    const double2* fel_eq;
    double* partials;             // [kReduceBlocks][kMoments]
    uint32_t* counter;
    double* out;                  // moments: [kMoments]; bunching: fel_state
    double dz;
    double var_c;                 // integral of s^2 over the basis function of unit width: 1/6 tent, 1/4 quadratic
    double cos_fac;               // integral of cos over the basis function of width h_x, per h_x: sinc(h_x/2)^(2 or 3)
};

// Allocation-free stepping (vp_step_noalloc): one lattice's scratch (b, the
// push tables, FEL state, per-tile partials, counters, descriptor and tile
// offsets) in a static device array of this size, for at most this many nodes.
constexpr size_t kNoAllocScratchBytes = (size_t)20 << 20;
constexpr long kNoAllocMaxNodes = 1l << 22;

struct NoAllocSetup {
    VpInst inst;            // the descriptor, pointers into the scratch
    VpInst* inst_out;       // where the kernels read it
    int32_t* off_out;       // tile offsets {0, deposit tiles, 0, solve tiles}
    TableParams tables;
    float4* tab_x;
    float4* tab_p;
    double2* fel_ex;
    double2* fel_eq;
    double* fel_state;
    uint32_t* counters;
    const double* fel_A;    // FEL field at the start (device), or null
    double n0;              // FEL normalisation
};
// Device address of the allocation-free scratch on the current device (looked
// up once per device); null with the error in *err on failure.
void* noalloc_scratch(hipError_t* err);
hipError_t launch_noalloc_setup(const NoAllocSetup& S, int nx, int np, hipStream_t s);
// fixed-point scale from max|w| (moments[8]); a non-finite input (moments[9])
// zeroes the scale, so nothing is deposited
hipError_t launch_noalloc_scale(VpInst* inst, const double* moments, hipStream_t s);
// the field back to the caller, the status word (VP_OK, VP_ENONFINITE, VP_ERANGE)
hipError_t launch_noalloc_finish(const double* moments, const double* fel_state, const uint32_t* counters,
                                 double* fel_A, int32_t* status, hipStream_t s);

// Record msg as the calling thread's last error (vp_last_error) and return code.
int set_error(int code, const char* msg);

// launchers (vp_kernels.hip)
// (optional events e0, e1: recorded at the kernel's start and end, for timing)
hipError_t launch_deposit(const LaunchArgs& a, int grid, size_t lds, int threads, hipStream_t s, int basis,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_solve(const LaunchArgs& a, int grid, hipStream_t s, int kind, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_fel_field(const LaunchArgs& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_fel_stage(const LaunchArgs& a, int grid, hipStream_t s, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
// the cached push map of a static Hamiltonian (inst: the device descriptor)
hipError_t launch_map(const VpInst* inst, long nodes, hipStream_t s);
const void* deposit_kernel(int basis);
// Solve kernels: tents (k_solve); spline bases (k_solve_spline), each with a
// variant for lattices with an open axis shorter than a window line.
enum SolveKind : int32_t { kSolveTent = 0, kSolveQuad = 1, kSolveQuadNarrow = 2, kSolveCubic = 3, kSolveCubicNarrow = 4 };
inline int solve_kind(int basis, int nx, int np, bool x_periodic) {
    if (basis == kBasisTent) return kSolveTent;
    const bool narrow = np < kLineQ || (!x_periodic && nx < kLineQ);
    return (basis == kBasisQuadratic ? kSolveQuad : kSolveCubic) + (narrow ? 1 : 0);
}
const void* solve_kernel(int kind);
inline int solve_threads(int kind) { return kind == kSolveTent ? kSolveThreads : kSolveQThreads; }
inline int solve_tiles(int nx, int np, int basis) {
    if (basis != kBasisTent) {
        const int seg = basis == kBasisQuadratic ? kSegQ : kSegC;
        return ((nx + seg - 1) / seg) * ((np + seg - 1) / seg);
    }
    return ((nx + kSegX - 1) / kSegX) * ((np + kSegP - 1) / kSegP);
}
const void* fel_field_kernel();
const void* fel_stage_kernel();

// Deposit LDS image: the tile and its border, (tx + 2 pad) x (ty + 2 pad) 64-bit cells.
inline size_t deposit_lds_bytes(int tx, int ty, int basis) {
    const int pad = basis == kBasisQuadratic ? kPadQ : basis == kBasisCubic ? kPadC : kPad;
    return sizeof(int64_t) * (size_t)(tx + 2 * pad) * (ty + 2 * pad);
}

}  // namespace vp
