// vp_device.h -- device helpers shared by the kernel sources of libvp: the
// push's error-free sums and cell split, the B-spline tap weights, the exact
// fixed-point encoding of the deposit sums, index wrapping, global-memory
// views, XCD-aware tile order and the LU factors of tridiag(1, 4, 1).
#pragma once

#include "vp_internal.h"

namespace vp {

namespace {

// 2 - sqrt(3): interior LU multiplier of tridiag(1,4,1), equal to 1/d_inf.
constexpr float kMinf = 0.267949192431122706f;

__device__ inline void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Integer part and fraction of hi + lo, |lo| small: the fraction of hi plus
// lo lies in [-1, 2), and its own floor moves the carry into the integer part
// (no branches).  The fraction is in [0, 1], reaching 1 only when a tiny
// negative fraction rounds up; the taps of t = 1 at cell k are those of
// t = 0 at cell k + 1, so either form deposits the same weights.
__device__ inline void split_cell(float hi, float lo, int& k, float& t) {
    const float f = floorf(hi);
    const float r = (hi - f) + lo;
    const float g = floorf(r);
    k = (int)(f + g);
    t = r - g;
}

// Cubic B-spline tap weights B3(t+1), B3(t), B3(1-t), B3(2-t) for t in [0,1),
// in FP64 (eq. 9).  The second tap is one minus the other three, so the taps
// sum to one to FP64 rounding (the partition of unity behind the conservation
// argument of eqs. 11-12), far below the 2^-40 fixed-point grid the products
// are rounded to.
// Every fused multiply-add is written out and the compiler forms no other:
// the taps are the same bits in every inlined copy, so the deposit's exact
// sums do not depend on which copy (kind of push, wrap mode) pushed a node.
__device__ inline void bspline_taps(float tf, double (&b)[4]) {
#pragma clang fp contract(off)
    const double sixth = 1.0 / 6.0;
    const double t = (double)tf, s = 1.0 - t, t2 = t * t;
    b[0] = (s * sixth) * (s * s);
    const double t3 = (t * sixth) * t2;
    b[3] = t3;
    b[2] = fma(-3.0, t3, fma(0.5, fma(t, t, t), sixth));
    b[1] = 1.0 - ((b[0] + b[3]) + b[2]);
}

// Quintic B-spline tap weights B5(t+2), B5(t+1), B5(t), B5(1-t), B5(2-t),
// B5(3-t) for t in [0,1): the overlaps of a quadratic B-spline basis function
// moved to cell position k + t with those of nodes k-2 .. k+3.  Each piece as
// a polynomial in s = 1 - t or in t, times 120:
//   s^5,  1 + 5s + 10s^2 + 10s^3 + 5s^4 - 5s^5,  26 + 50s + 20s^2 - 20s^3 - 20s^4 + 10s^5,
// and the same in t from the other end; the tap at cell k is one minus the
// others (partition of unity), as for the cubic taps.
__device__ inline void quintic_taps(float tf, double (&b)[6]) {
#pragma clang fp contract(off)
    const double c = 1.0 / 120.0;
    const double t = (double)tf, s = 1.0 - t;
    auto near = [](double v) {  // 1 + 5v + 10v^2 + 10v^3 + 5v^4 - 5v^5
        return fma(fma(fma(fma(fma(-5.0, v, 5.0), v, 10.0), v, 10.0), v, 5.0), v, 1.0);
    };
    auto mid = [](double v) {  // 26 + 50v + 20v^2 - 20v^3 - 20v^4 + 10v^5
        return fma(fma(fma(fma(fma(10.0, v, -20.0), v, -20.0), v, 20.0), v, 50.0), v, 26.0);
    };
    const double s2 = s * s, t2 = t * t;
    b[0] = ((s2 * s2) * s) * c;
    b[1] = near(s) * c;
    b[3] = mid(t) * c;
    b[4] = near(t) * c;
    b[5] = ((t2 * t2) * t) * c;
    b[2] = 1.0 - ((((b[0] + b[5]) + (b[1] + b[4])) + b[3]));
}

// Septic B-spline tap weights B7(t+3) .. B7(4-t) for t in [0,1): the
// overlaps of a cubic B-spline basis function moved to cell position k + t
// with those of nodes k-3 .. k+4.  Each piece as a polynomial in s = 1 - t or
// in t, times 5040:
//   v^7,  1 + 7v + 21v^2 + 35v^3 + 35v^4 + 21v^5 + 7v^6 - 7v^7,
//   120 + 392v + 504v^2 + 280v^3 - 84v^5 - 42v^6 + 21v^7,
//   1191 + 1715v + 315v^2 - 665v^3 - 315v^4 + 105v^5 + 105v^6 - 35v^7,
// the tap at cell k (the fourth) one minus the others.
__device__ inline void septic_taps(float tf, double (&b)[8]) {
#pragma clang fp contract(off)
    const double c = 1.0 / 5040.0;
    const double t = (double)tf, s = 1.0 - t;
    auto p1 = [](double v) {
        return fma(fma(fma(fma(fma(fma(fma(-7.0, v, 7.0), v, 21.0), v, 35.0), v, 35.0), v, 21.0), v, 7.0), v, 1.0);
    };
    auto p2 = [](double v) {
        return fma(fma(fma(fma(fma(fma(fma(21.0, v, -42.0), v, -84.0), v, 0.0), v, 280.0), v, 504.0), v, 392.0), v,
                   120.0);
    };
    auto p3 = [](double v) {
        return fma(fma(fma(fma(fma(fma(fma(-35.0, v, 105.0), v, 105.0), v, -315.0), v, -665.0), v, 315.0), v, 1715.0),
                   v, 1191.0);
    };
    const double s2 = s * s, t2 = t * t, s4 = s2 * s2, t4 = t2 * t2;
    b[0] = ((s4 * s2) * s) * c;
    b[1] = p1(s) * c;
    b[2] = p2(s) * c;
    b[4] = p3(t) * c;
    b[5] = p2(t) * c;
    b[6] = p1(t) * c;
    b[7] = ((t4 * t2) * t) * c;
    b[3] = 1.0 - ((((b[0] + b[7]) + (b[1] + b[6])) + (b[2] + b[5])) + b[4]);
}

template <int TAPS>
__device__ inline void basis_taps(float t, double (&b)[TAPS]) {
    if constexpr (TAPS == 4) bspline_taps(t, b);
    else if constexpr (TAPS == 6) quintic_taps(t, b);
    else septic_taps(t, b);
}

// 1.5 * 2^52: adding it to a value of magnitude below 2^51 leaves the value
// rounded to the nearest integer in the low bits of the sum's encoding,
// two's complement on top of the constant's encoding 0x4338 << 48.
constexpr double kFixMagic = 6755399441055744.0;

// Encoding of round(a * b) + 1.5 * 2^52, |a b| < 2^47: the FMA rounds the
// exact product once, straight onto the integer grid.  Summed as 64-bit
// integers, n such words give n (0x4338 << 48) + sum of the integers, whose
// low 48 bits are the sum itself modulo 2^48: exact while |sum| < 2^47
// (fix48_value), with no per-tap subtraction of the constant.
__device__ inline unsigned long long fix48_word(double a, double b) {
    return (unsigned long long)__double_as_longlong(fma(a, b, kFixMagic));
}
__device__ inline long long fix48_value(long long sum) { return (long long)((unsigned long long)sum << 16) >> 16; }

// Locate the instance of a flattened tile index (thread 0 only).
__device__ inline int find_instance(const int32_t* off, int ninst, int item) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline int wrap_index(int i, int n, float inv_n) {
    int q = (int)floorf(((float)i + 0.5f) * inv_n);
    int r = i - q * n;
    r += r < 0 ? n : 0;
    r -= r >= n ? n : 0;
    return r;
}

// Global-memory views of device pointers (loads through them are global, not
// flat, loads) and a 32-bit offset pinned to a vector register: a running
// row offset then costs one register and one add per row, instead of one
// precomputed 64-bit address per row.
#ifdef __HIP_DEVICE_COMPILE__
#define VP_GLOBAL __attribute__((address_space(1)))
#else
#define VP_GLOBAL
#endif
typedef VP_GLOBAL const float gfloat;
typedef VP_GLOBAL const float4 gfloat4;
typedef VP_GLOBAL float gfloat_out;
__device__ inline gfloat* as_global(const float* p) { return (gfloat*)p; }
__device__ inline gfloat4* as_global(const float4* p) { return (gfloat4*)p; }
// Stores through a global (not flat) pointer: a flat store also counts on
// the LDS counter, so a later wait for an LDS read would wait for it too.
__device__ inline gfloat_out* as_global_out(float* p) { return (gfloat_out*)p; }
__device__ inline unsigned in_vgpr(unsigned v) {
    asm volatile("" : "+v"(v));
    return v;
}
// Make a wave-uniform value available here (its scalar load waited for
// before a loop, not inside it: there the wait would also drain every LDS
// operation in flight, since both share one counter).
template <class T>
__device__ inline void settle(T v) {
    asm volatile("" ::"s"(v));
}

// s_waitcnt immediate that waits for every vector-memory load (vmcnt 0) and
// nothing else (expcnt 7, lgkmcnt 15).
constexpr int kWaitVmcnt0 = 0x0F70;

// Fourth word of a raw buffer resource (gfx9 family): 32-bit data format,
// no range check beyond the 2^32-byte window the resource spans.
constexpr int kBufferWord3 = 0x00020000;

// Workgroups are dispatched to the 8 XCDs round-robin.  When the grid has
// one workgroup per tile, give each XCD a contiguous run of tiles, so that
// neighbouring tiles (which share halo and source data) meet in one L2.
constexpr int kXcds = 8;
__device__ inline int xcd_tile(int b, int total) {
    const int xcd = b % kXcds, k = b / kXcds, q = total / kXcds, r = total % kXcds;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}
__device__ inline int tile_of(int item, int total) {
    return (int)gridDim.x == total ? xcd_tile(item, total) : item;
}

// LU coefficients of T = tridiag(1, 4, 1) on a line that starts at an open
// edge: d_0 = 4, m_k = 1/d_{k-1}, d_k = 4 - m_k.  They converge to the interior
// constants m = 1/d = 2 - sqrt 3 well within kEdge nodes.  Computed at compile
// time in FP64 and rounded once, so an unrolled solve folds them into its
// instructions (no table, no registers).
struct LuEdge {
    float m[kEdge], dinv[kEdge];
};
constexpr LuEdge lu_edge_table() {
    LuEdge t{};
    double dprev = 0.0;
    for (int k = 0; k < kEdge; ++k) {
        const double m = k == 0 ? 0.0 : 1.0 / dprev;
        const double d = 4.0 - m;
        t.m[k] = (float)m;
        t.dinv[k] = (float)(1.0 / d);
        dprev = d;
    }
    return t;
}
constexpr LuEdge kLuEdge = lu_edge_table();

// Coefficients at position k of a line (a compile-time index once unrolled):
// the edge values on a line that starts at an open edge (EDGE), the interior
// constant elsewhere and on every line that starts at a cut.
template <bool EDGE>
__device__ inline float lu_m(int k) { return (EDGE && k < kEdge) ? kLuEdge.m[k] : kMinf; }
template <bool EDGE>
__device__ inline float lu_dinv(int k) { return (EDGE && k < kEdge) ? kLuEdge.dinv[k] : kMinf; }

// Solve M y = b, M = tridiag(1/6, 2/3, 1/6), along one line of N values
// v[] (registers), written as
//     y = b - T^{-1} (D2 b),   T = 6 M = tridiag(1, 4, 1),  D2 b = b[k-1] - 2 b[k] + b[k+1]
// (T = 6 I + D2, so 6 T^{-1} = I - T^{-1} D2).  The LU recursions of T then only
// carry the correction T^{-1} D2 b, so their FP32 rounding (whose fixed point
// is biased on slowly varying data) acts on a term much smaller than b: the
// mass a line carries is kept to ~1e-10 per step instead of ~1e-8.
// Neighbours outside the line count as zero: exact at an open edge (the
// truncated M), and a cut inside the lattice only disturbs the halo.
// MASKED: the lattice line is shorter than N; v[k] is zero for k >= n
// and the recursion ends at n (an open edge).  Otherwise every index
// condition is a compile-time one.  The solution replaces v[LO..N); the
// backward sweep stops at LO, below which the caller keeps nothing (the
// values there are left as they were), so z[k < LO] and v[k < LO] are dead
// after the forward sweep and hold no registers.
template <int N, int LO, bool EDGE, bool MASKED>
__device__ inline void line_solve(float (&v)[N], int n) {
    float z[N];
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float r = ((k > 0 ? v[k - 1] : 0.0f) + (k + 1 < N ? v[k + 1] : 0.0f)) - 2.0f * v[k];
        acc = fmaf(-lu_m<EDGE>(k), acc, r);
        if (MASKED) acc = k < n ? acc : 0.0f;
        z[k] = acc;
    }
    float c = 0.0f;
#pragma unroll
    for (int k = N - 1; k >= LO; --k) {
        c = (z[k] - c) * lu_dinv<EDGE>(k);
        v[k] -= c;
    }
}

// The same solve on a line that starts at an open edge (or is a whole short
// line, MASKED) with the forward sweep's z of the first NL nodes kept in LDS
// (zs[k * stride]) rather than in registers: not much more than one line of
// registers is live, where v and z would take two.  For the few windows that need it; the backward sweep's LDS reads do not
// depend on the recursion, so they are issued ahead of it.
template <int N, int NL, bool MASKED>
__device__ inline void line_solve_lds(float (&v)[N], int n, float* zs, int stride) {
    float zr[N - NL];  // z of the nodes past the first NL
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float r = ((k > 0 ? v[k - 1] : 0.0f) + (k + 1 < N ? v[k + 1] : 0.0f)) - 2.0f * v[k];
        acc = fmaf(-lu_m<true>(k), acc, r);
        if (MASKED) acc = k < n ? acc : 0.0f;
        if (k < NL) zs[k * stride] = acc;
        else zr[k - NL] = acc;
    }
    asm volatile("" ::: "memory");  // read z back from LDS (not forwarded from the stores)
    float c = 0.0f;
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        c = ((k < NL ? zs[k * stride] : zr[k - NL]) - c) * lu_dinv<true>(k);
        v[k] -= c;
    }
}

// Start of the window of `line` nodes around a segment starting at s0 on an
// open axis of n nodes: kHalo before the segment, shifted to lie inside
// [0, n) so that a window near an edge ends exactly at it (0 when n < line).
__device__ inline int open_window(int s0, int n, int line) { return max(0, min(s0 - kHalo, n - line)); }

}  // namespace

}  // namespace vp
