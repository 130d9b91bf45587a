// vp4_internal.h -- data layout shared by the host runtime and the gfx950
// kernels of the four-dimensional (2D2V) phase space.
#pragma once

#include "vp_internal.h"

namespace vp {

// ---------------------------------------------------------------------------
// Four-dimensional phase space (x, y, p_x, p_y), tensor-product tents: the
// weights are [n_py][n_px][n_y][n_x] (x fastest); x and y periodic, the
// momenta open.  One step: k_deposit4 (push and the 4^4 B3 taps of every
// node into LDS destination tiles), then one line-solve launch per axis.
// ---------------------------------------------------------------------------
enum Push4 : int32_t { kPush4Free = 0, kPush4Potential = 2 };
constexpr int kDeposit4Threads = 1024;
constexpr int kDeposit4Pad = 4;  // LDS cells before and after the deposit tile's image (x taps past a row's ends)
constexpr int kDeposit4RowPad = 3;  // LDS cells after each x row of the deposit tile (taps past its ends)
constexpr int kSolve4Threads = 256;
constexpr int kSolve4Halo = 16;  // periodic lines: warm-up nodes (wrapped) per side
constexpr int kSolve4XLines = 64;  // k_solve4_x: lines along x staged in LDS per workgroup
constexpr int kSolve4XMax = 120;   // k_solve4_x: longest x line (two padded copies of 64 lines within 64 KiB)

struct Vp4Inst {
    int32_t n[4];        // nodes along x, y, px, py
    int32_t T[4];        // deposit tile along each axis (nodes)
    int32_t tiles[4];    // tiles along each axis
    int32_t total_tiles;
    int32_t kind;        // Push4
    int32_t parity0;
    int32_t pad0;
    // kick in cells: dv_px = -(ax sin xh + cx sin(xh - yh)), dv_py = -(by sin yh - cy sin(xh - yh));
    // drift in cells: du_x = drift_x(p_x) + kdx dv_px, du_y = drift_y(p_y) + kdy dv_py
    float ax, cx, by, cy, kdx, kdy;
    float fix_scale, fix_inv;   // deposit fixed point: 2^(40-e) and its inverse, max|w0| < 2^e
    const float4* tab[4];       // x, y: (sin, cos) of the node; px, py: (drift hi, drift lo, sin q, cos q)
    const int4* boxes;          // per tile: (x0, x1, y0, y1), (px0, px1, py0, py1) source ranges, x and y unwrapped
    float* w[2];
    uint32_t* counters;         // [kRangeFlag]: deposit range
};

struct Launch4Args {
    const Vp4Inst* inst;
    int32_t parity;    // step parity relative to parity0 (the deposit reads w[parity0 ^ parity])
    int32_t axis;      // k_solve4: the axis of the lines (0 x, 1 y, 2 px, 3 py)
    int32_t push;      // k_deposit4: Push4 kind (chooses the instantiation)
    int32_t total;     // deposit: tiles; solve: lines
    int32_t inst_nx;   // solve: n_x (the launch shape of the x lines)
    const float* src;  // solve: input array
    float* dst;        // deposit, solve: output array
};

struct Reduce4Args {
    const float* w;
    int32_t n[4];
    int32_t mode;                 // 0: moments, 2: sum, max|w| and non-finite count
    double lo[4], h[4];
    double a, b, c;               // potential (energy)
    double sinc2[2];              // sinc^2(h/2) along x and y (tent integrals of cos)
    double* partials;             // [kReduceBlocks][kMoments]
    uint32_t* counter;
    double* out;                  // [kMoments]
};

hipError_t launch_deposit4(const Launch4Args& a, size_t lds, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
hipError_t launch_solve4(const Launch4Args& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_reduce4(const Reduce4Args& a, hipStream_t s);
const void* deposit4_kernel(int push);

}  // namespace vp
