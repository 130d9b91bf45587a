// vp4_kernels.hip -- gfx950 kernels of the four-dimensional (2D2V) phase
// space: the 256-tap deposit, the per-axis line solves and the moments.
#include <hip/hip_ext.h>

#include "vp4_internal.h"
#include "vp_device.h"

namespace vp {

// ---------------------------------------------------------------------------
// Four-dimensional phase space: the same step with tensor-product tents on
// (x, y, p_x, p_y) (the closing remark of the algorithm section: only Lambda
// and Delta depend on the dimension).  The overlap of two 4-D tents is the
// product of four B3 factors (eq. 9), the mass matrix the Kronecker product of
// four tridiagonal ones (eq. 8).
// ---------------------------------------------------------------------------

// Wrap an index into [0, n) (any integer, small multiples of n away).
__device__ inline int wrap4(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// A periodic index into [0, n): one conditional step for an index within a
// period of the range, the remainder for any other (rare) value.
__device__ inline int wrap_once4(int i, int n) {
    i -= i >= n ? n : 0;
    i += i < 0 ? n : 0;
    return (unsigned)i < (unsigned)n ? i : wrap4(i, n);
}

// The push of one source into whole cells and fractions along x, y (drift)
// and p_x, p_y (kick), from the per-axis tables.
template <int PUSH>
__device__ inline void push4(const Vp4Inst& I, float4 X, float4 Y, float4 PX, float4 PY, int& ku0, float& fu0,
                             int& ku1, float& fu1, int& kv0, float& fv0, int& kv1, float& fv1) {
#pragma clang fp contract(off)
    float dvx = 0.0f, dvy = 0.0f;
    if (PUSH == kPush4Potential) {
        // phases at the half drift: x + q_px, y + q_py, from the tables
        const float sxh = fmaf(X.x, PX.w, X.y * PX.z), cxh = fmaf(X.y, PX.w, -(X.x * PX.z));
        const float syh = fmaf(Y.x, PY.w, Y.y * PY.z), cyh = fmaf(Y.y, PY.w, -(Y.x * PY.z));
        const float sd = fmaf(sxh, cyh, -(cxh * syh));  // sin(xh - yh)
        dvx = -fmaf(I.ax, sxh, I.cx * sd);
        dvy = -fmaf(I.by, syh, -(I.cy * sd));
    }
    float su, eu;
    two_sum(PX.x, dvx * I.kdx, su, eu);
    split_cell(su, eu + PX.y, ku0, fu0);
    two_sum(PY.x, dvy * I.kdy, su, eu);
    split_cell(su, eu + PY.y, ku1, fu1);
    split_cell(dvx, 0.0f, kv0, fv0);
    split_cell(dvy, 0.0f, kv1, fv1);
}

// The sources of one tile's box.  Thread k takes sources k, k + blockDim.x,
// ... of the box in x-fastest order; its box coordinates advance by the
// stride's own coordinates with one carry per axis (no division per source).
// NEAR: the tile is at least 3 cells short of spanning each periodic axis,
// so a tap before its origin never wraps into it and a node's four x taps
// are four consecutive LDS cells (one address per block of four, immediate
// offsets, no branch): an x tap outside the tile adds the fixed-point zero
// (a word whose low 48 bits are zero; a cell's sum is the sign-extended low
// 48 bits) to the cell it addresses, one of the kDeposit4RowPad cells that
// end every x row of the LDS image (a tap before the row's start lands in the
// previous row's, or in the kDeposit4Pad cells before the image), never on a
// cell that real taps add to.  Otherwise a tap before the origin wraps to the
// axis's end.
template <int PUSH, bool NEAR>
__device__ inline void scan_box4(const Vp4Inst& I, long long* acc4, gfloat* __restrict__ w_in, int4 ba,
                                 int4 bb, int B0, int B1, int B2, int B3, int O0, int O1, int O2, int O3, int E0,
                                 int E1, int E2, int E3) {
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    const int T1 = I.T[1], T2 = I.T[2];
    const int S1 = I.T[0] + kDeposit4RowPad, S2 = S1 * T1, S3 = S2 * T2;  // LDS strides (padded x rows)
    gfloat4* __restrict__ tx = as_global(I.tab[0]);
    gfloat4* __restrict__ ty = as_global(I.tab[1]);
    gfloat4* __restrict__ tpx = as_global(I.tab[2]);
    gfloat4* __restrict__ tpy = as_global(I.tab[3]);
    const float scale = I.fix_scale;
    // the thread's first source and the stride, as box coordinates
    const int st = (int)blockDim.x, BB = B0 * B1;
    const int st0 = st % B0, st1 = (st / B0) % B1, st2 = (st / BB) % B2, st3 = st / (BB * B2);
    const int k = (int)threadIdx.x;
    int i0 = k % B0, i1 = (k / B0) % B1, i2 = (k / BB) % B2, i3 = k / (BB * B2);
    for (; i3 < B3;) {
        const int ix = wrap_once4(ba.x + i0, n0), iy = wrap_once4(ba.z + i1, n1);
        const int ipx = bb.x + i2, ipy = bb.z + i3;
        const unsigned node = (__umul24(__umul24(ipy, n2) + ipx, n1) + iy) * (unsigned)n0 + ix;
        const float wv = w_in[node];
        const float4 X = tx[ix], Y = ty[iy], PX = tpx[ipx], PY = tpy[ipy];
        // the next source's box coordinates
        i0 += st0;
        int c = i0 >= B0;
        i0 -= c ? B0 : 0;
        i1 += st1 + c;
        c = i1 >= B1;
        i1 -= c ? B1 : 0;
        i2 += st2 + c;
        c = i2 >= B2;
        i2 -= c ? B2 : 0;
        i3 += st3 + c;
        if (wv == 0.0f) continue;
        int ku0, ku1, kv0, kv1;
        float fu0, fu1, fv0, fv1;
        push4<PUSH>(I, X, Y, PX, PY, ku0, fu0, ku1, fu1, kv0, fv0, kv1, fv1);
        // first tap of each axis relative to the tile origin (periodic axes
        // wrapped into [-3, n - 3))
        const int r0 = wrap_once4(ix + ku0 + 2 - O0, n0) - 3;
        const int r1 = wrap_once4(iy + ku1 + 2 - O1, n1) - 3;
        const int r2 = ipx + kv0 - 1 - O2, r3 = ipy + kv1 - 1 - O3;
        if (r0 < -3 || r0 >= E0 || r1 < -3 || r1 >= E1 || r2 < -3 || r2 >= E2 || r3 < -3 || r3 >= E3) continue;
        double bx[4], byy[4], bpx[4], bpy[4];
        bspline_taps(fu0, bx);
        bspline_taps(fu1, byy);
        bspline_taps(fv0, bpx);
        bspline_taps(fv1, bpy);
        const double ws = (double)(wv * scale);
        // tap positions in the tile along x and y; on a periodic axis a tap
        // before the origin wraps to the axis's end (only a tile within 3
        // cells of spanning the axis can take it)
        int p0[4], p1[4];
        double bxm[4];  // NEAR: the x taps, zero outside the tile
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            p0[q] = NEAR ? r0 + q : r0 + q + (r0 + q < 0 ? n0 : 0);
            p1[q] = NEAR ? r1 + q : r1 + q + (r1 + q < 0 ? n1 : 0);
            bxm[q] = (unsigned)(r0 + q) < (unsigned)E0 ? bx[q] : 0.0;
        }
        const int lane = NEAR ? r1 * S1 + r0 : 0;  // cell (r0, r1) of the lane's first taps, relative
#pragma unroll
        for (int q3 = 0; q3 < 4; ++q3) {
            if ((unsigned)(r3 + q3) >= (unsigned)E3) continue;
            const double w3 = ws * bpy[q3];
#pragma unroll
            for (int q2 = 0; q2 < 4; ++q2) {
                if ((unsigned)(r2 + q2) >= (unsigned)E2) continue;
                const double w2 = w3 * bpx[q2];
                const int plane = (r3 + q3) * S3 + (r2 + q2) * S2;
#pragma unroll
                for (int q1 = 0; q1 < 4; ++q1) {
                    if ((unsigned)p1[q1] >= (unsigned)E1) continue;
                    const double w1 = w2 * byy[q1];
                    if (NEAR) {
                        unsigned long long* row = (unsigned long long*)(acc4 + (lane + plane + q1 * S1));
#pragma unroll
                        for (int q0 = 0; q0 < 4; ++q0) atomicAdd(row + q0, fix48_word(w1, bxm[q0]));
                    } else {
                        unsigned long long* row = (unsigned long long*)(acc4 + plane + p1[q1] * S1);
#pragma unroll
                        for (int q0 = 0; q0 < 4; ++q0)
                            if ((unsigned)p0[q0] < (unsigned)E0) atomicAdd(row + p0[q0], fix48_word(w1, bx[q0]));
                    }
                }
            }
        }
    }
}

// k_deposit4: a workgroup owns one destination tile of T0 x T1 x T2 x T3
// lattice nodes held in LDS (no border: every tap is tested against the tile
// and the blocks of taps that miss it are skipped), scans the host-planned
// source box, pushes each source and adds its 4^4 B3 taps as exact
// fixed-point integers (the 2-D deposit's encoding), then writes the tile of
// b once.  The blocks of taps along p_y, p_x and y are skipped when the
// lane's taps there miss the tile; along x a tap outside the tile adds the
// fixed-point zero to a pad cell (or, in a tile within 3 cells of spanning a
// periodic axis, is its own test).
template <int PUSH>
__global__ __launch_bounds__(kDeposit4Threads) void k_deposit4(Launch4Args A) {
    extern __shared__ __align__(16) long long lds4d[];
    long long* acc4 = lds4d + kDeposit4Pad;  // the tile's image, between the padding cells
    const Vp4Inst& I = *A.inst;
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2], n3 = I.n[3];
    const int T0 = I.T[0], T1 = I.T[1], T2 = I.T[2], T3 = I.T[3];
    const int cells = T0 * T1 * T2 * T3;
    const int P0 = T0 + kDeposit4RowPad, lds_cells = P0 * T1 * T2 * T3;  // the LDS image: padded x rows
    const int par = (I.parity0 + A.parity) & 1;
    gfloat* __restrict__ w_in = as_global(I.w[par]);
    for (int t = blockIdx.x; t < A.total; t += gridDim.x) {
        int q = t;
        const int c0 = q % I.tiles[0];
        q /= I.tiles[0];
        const int c1 = q % I.tiles[1];
        q /= I.tiles[1];
        const int c2 = q % I.tiles[2];
        const int c3 = q / I.tiles[2];
        const int O0 = c0 * T0, O1 = c1 * T1, O2 = c2 * T2, O3 = c3 * T3;
        const int E0 = min(T0, n0 - O0), E1 = min(T1, n1 - O1), E2 = min(T2, n2 - O2), E3 = min(T3, n3 - O3);
        const int4 ba = I.boxes[2 * t], bb = I.boxes[2 * t + 1];
        int B0 = ba.y - ba.x, B1 = ba.w - ba.z, B2 = bb.y - bb.x, B3 = bb.w - bb.z;
        if (B0 <= 0 || B1 <= 0 || B2 <= 0 || B3 <= 0 || !(I.fix_scale > 0.0f)) {
            // an empty box (or an all-zero state): no source
            B0 = B1 = B2 = 1;
            B3 = 0;
        }
        for (int k = threadIdx.x; k < lds_cells; k += blockDim.x) acc4[k] = 0ll;
        __syncthreads();
        if (E0 <= n0 - 3 && E1 <= n1 - 3)
            scan_box4<PUSH, true>(I, acc4, w_in, ba, bb, B0, B1, B2, B3, O0, O1, O2, O3, E0, E1, E2, E3);
        else
            scan_box4<PUSH, false>(I, acc4, w_in, ba, bb, B0, B1, B2, B3, O0, O1, O2, O3, E0, E1, E2, E3);
        __syncthreads();
        bool out_of_range = false;
        const double inv = (double)I.fix_inv;
        for (int k = threadIdx.x; k < cells; k += blockDim.x) {
            int r = k;
            const int e0 = r % T0;
            r /= T0;
            const int e1 = r % T1;
            r /= T1;
            const int e2 = r % T2;
            const int e3 = r / T2;
            if (e0 >= E0 || e1 >= E1 || e2 >= E2 || e3 >= E3) continue;
            const long long v = fix48_value(acc4[((e3 * T2 + e2) * T1 + e1) * P0 + e0]);
            out_of_range |= (unsigned long long)v + (1ull << 46) >= (1ull << 47);
            A.dst[(((size_t)(O3 + e3) * n2 + (O2 + e2)) * n1 + (O1 + e1)) * n0 + (O0 + e0)] = (float)((double)v * inv);
        }
        // one flag write per wavefront that saw a cell out of range (an
        // atomic per thread on one address would serialise the launch)
        if (__any(out_of_range) && (threadIdx.x & 63) == 0) atomicOr(&I.counters[kRangeFlag], 1u);
        __syncthreads();
    }
}

// One line of the mass-matrix solve M y = b, M = tridiag(1/6, 2/3, 1/6), as
// y = b - T^{-1}(D2 b) with T = 6M = tridiag(1, 4, 1) (the 2-D solve's form:
// the FP32 recursions only carry the small correction).  Element k of the
// line is in[k * stride], the result goes to out[k * stride] (z is kept there
// between the sweeps).  A periodic line is solved on the line extended by
// kSolve4Halo wrapped nodes per side with the recursions starting from zero
// (the error decays by 2 - sqrt 3 per node, ~7e-10 at the line); an open line
// is the truncated matrix, exact, with the LU factors of the first rows from
// the edge (d_0 = 4, d_k = 4 - 1/d_{k-1}).
// The sweeps take the line in chunks of kChunk4 nodes whose loads are all
// issued before the chunk's recursion steps (the recursions wait on one FMA
// per node, not on a load); lines longer than the halo (periodic) or the edge
// table (open) wrap and pick their factors without a per-node test.  The
// arithmetic, and so every result bit, is that of the node-by-node sweeps.
constexpr int kChunk4 = 8;
static_assert(kEdge % kChunk4 == 0 && kSolve4Halo % kChunk4 == 0, "whole chunks of edge factors and halo");

// The sweeps' arithmetic is written out (no implicit contraction): the
// forward step z_k = b_{k-1} + b_{k+1} - 2 b_k - m_k z_{k-1} (one FMA), the
// backward step c_k = (z_k - c_{k+1}) m and y_k = b_k - c_k, each rounded.
__device__ inline float tri_z(float acc, float m, float bm, float bp, float b0) {
#pragma clang fp contract(off)
    return fmaf(-m, acc, (bm + bp) - 2.0f * b0);
}

__device__ inline void solve_line4(const float* __restrict__ in, float* __restrict__ out, int n, size_t stride,
                                   bool periodic, const float (&dinv)[kEdge], const float (&mult)[kEdge]) {
#pragma clang fp contract(off)
    constexpr int C = kChunk4;
    auto b = [&](int k) { return in[(size_t)k * stride]; };
    auto o = [&](int k) -> float& { return out[(size_t)k * stride]; };
    if (periodic) {
        constexpr int H = kSolve4Halo;
        float zt[H];
        float acc = 0.0f;
        if (n <= H) {  // a line no longer than the halo: general wraps
            float bm = b(wrap4(-H - 1, n)), b0 = b(wrap4(-H, n));
            for (int k = -H; k < n + H; ++k) {
                const float bp = b(wrap4(k + 1, n));
                acc = tri_z(acc, kMinf, bm, bp, b0);
                if (k >= 0 && k < n) o(k) = acc;
                else if (k >= n) zt[k - n] = acc;
                bm = b0;
                b0 = bp;
            }
        } else {
            // indices within one period of the line: one conditional wrap
            auto w = [&](int k) { return k < 0 ? k + n : (k >= n ? k - n : k); };
            float bm = b(w(-H - 1)), b0 = b(w(-H));
            // warm-up over the wrapped halo before the line
#pragma unroll
            for (int k0 = -H; k0 < 0; k0 += C) {
                float bb[C];
#pragma unroll
                for (int q = 0; q < C; ++q) bb[q] = b(w(k0 + 1 + q));
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    acc = tri_z(acc, kMinf, bm, bb[q], b0);
                    bm = b0;
                    b0 = bb[q];
                }
            }
            int k = 0;
            for (; k + C <= n; k += C) {
                float bb[C];
#pragma unroll
                for (int q = 0; q < C; ++q) bb[q] = b(w(k + 1 + q));
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    acc = tri_z(acc, kMinf, bm, bb[q], b0);
                    o(k + q) = acc;
                    bm = b0;
                    b0 = bb[q];
                }
            }
            for (; k < n; ++k) {
                const float bp = b(w(k + 1));
                acc = tri_z(acc, kMinf, bm, bp, b0);
                o(k) = acc;
                bm = b0;
                b0 = bp;
            }
            // the halo after the line
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += C) {
                float bb[C];
#pragma unroll
                for (int q = 0; q < C; ++q) bb[q] = b(w(n + k0 + 1 + q));
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    acc = tri_z(acc, kMinf, bm, bb[q], b0);
                    zt[k0 + q] = acc;
                    bm = b0;
                    b0 = bb[q];
                }
            }
        }
        float c = 0.0f;
#pragma unroll
        for (int k = H - 1; k >= 0; --k) c = (zt[k] - c) * kMinf;
        int k = n - 1;
        for (; k - C + 1 >= 0; k -= C) {
            float zz[C], bb[C];
#pragma unroll
            for (int q = 0; q < C; ++q) {
                zz[q] = o(k - q);
                bb[q] = b(k - q);
            }
#pragma unroll
            for (int q = 0; q < C; ++q) {
                c = (zz[q] - c) * kMinf;
                o(k - q) = bb[q] - c;
            }
        }
        for (; k >= 0; --k) {
            c = (o(k) - c) * kMinf;
            o(k) = b(k) - c;
        }
        return;
    }
    if (n <= kEdge) {  // an open line within the edge table: node by node
        float acc = 0.0f, bm = 0.0f, b0 = b(0);
        for (int k = 0; k < n; ++k) {
            const float bp = k + 1 < n ? b(k + 1) : 0.0f;
            acc = tri_z(acc, mult[k], bm, bp, b0);
            o(k) = acc;
            bm = b0;
            b0 = bp;
        }
        float c = 0.0f;
        for (int k = n - 1; k >= 0; --k) {
            c = (o(k) - c) * dinv[k];
            o(k) = b(k) - c;
        }
        return;
    }
    float acc = 0.0f, bm = 0.0f, b0 = b(0);
    // the first kEdge nodes with the edge factors (compile-time operands)
#pragma unroll
    for (int k0 = 0; k0 < kEdge; k0 += C) {
        float bb[C];
#pragma unroll
        for (int q = 0; q < C; ++q) bb[q] = b(k0 + 1 + q);  // k0 + 1 + q <= kEdge < n
#pragma unroll
        for (int q = 0; q < C; ++q) {
            acc = tri_z(acc, kLuEdge.m[k0 + q], bm, bb[q], b0);
            o(k0 + q) = acc;
            bm = b0;
            b0 = bb[q];
        }
    }
    int k = kEdge;
    for (; k + C <= n; k += C) {
        float bb[C];
#pragma unroll
        for (int q = 0; q < C; ++q) bb[q] = k + 1 + q < n ? b(k + 1 + q) : 0.0f;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            acc = tri_z(acc, kMinf, bm, bb[q], b0);
            o(k + q) = acc;
            bm = b0;
            b0 = bb[q];
        }
    }
    for (; k < n; ++k) {
        const float bp = k + 1 < n ? b(k + 1) : 0.0f;
        acc = tri_z(acc, kMinf, bm, bp, b0);
        o(k) = acc;
        bm = b0;
        b0 = bp;
    }
    float c = 0.0f;
    k = n - 1;
    for (; k - C + 1 >= kEdge; k -= C) {
        float zz[C], bb[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            zz[q] = o(k - q);
            bb[q] = b(k - q);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            c = (zz[q] - c) * kMinf;
            o(k - q) = bb[q] - c;
        }
    }
    for (; k >= kEdge; --k) {
        c = (o(k) - c) * kMinf;
        o(k) = b(k) - c;
    }
    // the first kEdge nodes with the edge factors
#pragma unroll
    for (int k0 = kEdge - 1; k0 >= 0; k0 -= C) {
        float zz[C], bb[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            zz[q] = o(k0 - q);
            bb[q] = b(k0 - q);
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            c = (zz[q] - c) * kLuEdge.dinv[k0 - q];
            o(k0 - q) = bb[q] - c;
        }
    }
}

// k_solve4: one thread per lattice line along A.axis, from A.src into A.dst.
// Along y, p_x and p_y neighbouring threads take neighbouring x, so every
// access is coalesced; along x a thread walks its own contiguous line.
__global__ __launch_bounds__(kSolve4Threads) void k_solve4(Launch4Args A) {
    const Vp4Inst& I = *A.inst;
    float dinv[kEdge], mult[kEdge];
#pragma unroll
    for (int k = 0; k < kEdge; ++k) {
        dinv[k] = kLuEdge.dinv[k];
        mult[k] = kLuEdge.m[k];
    }
    const int L = blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= A.total) return;
    const int n0 = I.n[0], n1 = I.n[1], n2 = I.n[2];
    size_t start, stride;
    int n;
    if (A.axis == 0) {
        start = (size_t)L * n0;
        stride = 1;
        n = n0;
    } else {
        const int ix = L % n0, rest = L / n0;
        if (A.axis == 1) {  // rest = ipy * n2 + ipx
            start = (size_t)rest * n1 * n0 + ix;
            stride = n0;
            n = n1;
        } else if (A.axis == 2) {  // rest = ipy * n1 + iy
            const int iy = rest % n1, ipy = rest / n1;
            start = (size_t)ipy * n2 * n1 * n0 + (size_t)iy * n0 + ix;
            stride = (size_t)n1 * n0;
            n = n2;
        } else {  // rest = ipx * n1 + iy
            start = (size_t)rest * n0 + ix;
            stride = (size_t)n2 * n1 * n0;
            n = I.n[3];
        }
    }
    solve_line4(A.src + start, A.dst + start, n, stride, A.axis < 2, dinv, mult);
}

// k_solve4_x: the lines along x, which are contiguous: a workgroup copies
// the kSolve4XLines consecutive lines it owns into LDS (coalesced, one padded
// row per line), one thread per line solves it there, and the result goes back
// coalesced.  Lattices with n_x up to kSolve4XMax nodes.
__global__ __launch_bounds__(kSolve4Threads) void k_solve4_x(Launch4Args A) {
    extern __shared__ float lds4x[];
    const Vp4Inst& I = *A.inst;
    float dinv[kEdge], mult[kEdge];
#pragma unroll
    for (int k = 0; k < kEdge; ++k) {
        dinv[k] = kLuEdge.dinv[k];
        mult[k] = kLuEdge.m[k];
    }
    const int nx = I.n[0], pitch = nx + 1;
    const int L0 = blockIdx.x * kSolve4XLines;
    const int lines = min(kSolve4XLines, A.total - L0);
    float* in = lds4x;
    float* out = lds4x + kSolve4XLines * pitch;
    const float* src = A.src + (size_t)L0 * nx;
    // the copies go in batches of kChunk4 elements per thread, every load of
    // a batch issued before its stores (the element's line and position from
    // an exact float quotient: e < 2^14 and nx <= kSolve4XMax)
    const int total = lines * nx, step = (int)blockDim.x;
    const float inv_nx = 1.0f / (float)nx;
    auto slot = [&](int e) {
        int l = (int)(((float)e + 0.5f) * inv_nx);
        return l * pitch + (e - l * nx);
    };
    for (int e0 = threadIdx.x; e0 < total; e0 += kChunk4 * step) {
        float v[kChunk4];
#pragma unroll
        for (int q = 0; q < kChunk4; ++q) {
            const int e = e0 + q * step;
            v[q] = e < total ? src[e] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kChunk4; ++q) {
            const int e = e0 + q * step;
            if (e < total) in[slot(e)] = v[q];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < lines) solve_line4(in + threadIdx.x * pitch, out + threadIdx.x * pitch, nx, 1, true, dinv, mult);
    __syncthreads();
    float* dst = A.dst + (size_t)L0 * nx;
    for (int e0 = threadIdx.x; e0 < total; e0 += kChunk4 * step) {
        float v[kChunk4];
#pragma unroll
        for (int q = 0; q < kChunk4; ++q) {
            const int e = e0 + q * step;
            v[q] = e < total ? out[slot(e)] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kChunk4; ++q) {
            const int e = e0 + q * step;
            if (e < total) dst[e] = v[q];
        }
    }
}

// k_reduce4: FP64 fixed-order sums over a 4-D state (the moments of the 2-D
// reduction, axis by axis).
__global__ __launch_bounds__(kReduceThreads) void k_reduce4(Reduce4Args R) {
    __shared__ double s_part[kReduceThreads / 64][kMoments];
    __shared__ int s_last;
    double acc[kMoments];
#pragma unroll
    for (int k = 0; k < kMoments; ++k) acc[k] = 0.0;
    const long n = (long)R.n[0] * R.n[1] * R.n[2] * R.n[3];
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const double w = (double)R.w[k];
        if (!isfinite(w)) { acc[9] += 1.0; continue; }
        acc[0] += w;
        acc[8] = fmax(acc[8], fabs(w));
        if (R.mode == 2) continue;
        long r = k;
        const int i0 = (int)(r % R.n[0]);
        r /= R.n[0];
        const int i1 = (int)(r % R.n[1]);
        r /= R.n[1];
        const int i2 = (int)(r % R.n[2]);
        const int i3 = (int)(r / R.n[2]);
        const double x = R.lo[0] + i0 * R.h[0], y = R.lo[1] + i1 * R.h[1];
        const double px = R.lo[2] + i2 * R.h[2], py = R.lo[3] + i3 * R.h[3];
        if (w < 0.0) acc[1] += w;
        acc[2] += fabs(w);
        if (w > 0.0) acc[3] += w * log(w);
        acc[4] += w * px;
        acc[5] += w * py;
        const double e = 0.5 * (px * px + R.h[2] * R.h[2] / 6.0) + 0.5 * (py * py + R.h[3] * R.h[3] / 6.0) -
                         R.a * R.sinc2[0] * cos(x) - R.b * R.sinc2[1] * cos(y) -
                         R.c * R.sinc2[0] * R.sinc2[1] * cos(x - y);
        acc[6] += w * e;
    }
#pragma unroll
    for (int k = 0; k < kMoments; ++k)
        for (int o = 32; o > 0; o >>= 1) {
            const double v = __shfl_down(acc[k], o);
            acc[k] = k == 8 ? fmax(acc[k], v) : acc[k] + v;
        }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < kMoments; ++k) s_part[wid][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < kMoments; ++k) {
            double s = 0.0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s = k == 8 ? fmax(s, s_part[q][k]) : s + s_part[q][k];
            R.partials[blockIdx.x * kMoments + k] = s;
        }
        __threadfence();
        s_last = (atomicAdd(R.counter, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (threadIdx.x < kMoments) {
        double s = 0.0;
        for (unsigned q = 0; q < gridDim.x; ++q) {
            const double v = __builtin_nontemporal_load(&R.partials[q * kMoments + threadIdx.x]);
            s = threadIdx.x == 8 ? fmax(s, v) : s + v;
        }
        R.out[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicExch(R.counter, 0u);
    }
}


const void* deposit4_kernel(int push) {
    return push == kPush4Free ? reinterpret_cast<const void*>(&k_deposit4<kPush4Free>)
                              : reinterpret_cast<const void*>(&k_deposit4<kPush4Potential>);
}

hipError_t launch_deposit4(const Launch4Args& a, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    void* args[1] = {const_cast<Launch4Args*>(&a)};
    const void* k = a.push == kPush4Free ? reinterpret_cast<const void*>(&k_deposit4<kPush4Free>)
                                         : reinterpret_cast<const void*>(&k_deposit4<kPush4Potential>);
    if (e0 || e1) return hipExtLaunchKernel(k, dim3(a.total), dim3(kDeposit4Threads), args, lds, s, e0, e1, 0);
    return hipLaunchKernel(k, dim3(a.total), dim3(kDeposit4Threads), args, lds, s);
}

hipError_t launch_solve4(const Launch4Args& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    void* args[1] = {const_cast<Launch4Args*>(&a)};
    if (a.axis == 0 && a.inst_nx <= kSolve4XMax) {
        const dim3 grid((a.total + kSolve4XLines - 1) / kSolve4XLines);
        const size_t lds = 2 * (size_t)kSolve4XLines * (a.inst_nx + 1) * sizeof(float);
        const void* k = reinterpret_cast<const void*>(&k_solve4_x);
        if (e0 || e1) return hipExtLaunchKernel(k, grid, dim3(kSolve4Threads), args, lds, s, e0, e1, 0);
        return hipLaunchKernel(k, grid, dim3(kSolve4Threads), args, lds, s);
    }
    const dim3 grid((a.total + kSolve4Threads - 1) / kSolve4Threads);
    const void* k = reinterpret_cast<const void*>(&k_solve4);
    if (e0 || e1) return hipExtLaunchKernel(k, grid, dim3(kSolve4Threads), args, 0, s, e0, e1, 0);
    return hipLaunchKernel(k, grid, dim3(kSolve4Threads), args, 0, s);
}

hipError_t launch_reduce4(const Reduce4Args& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce4, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace vp
