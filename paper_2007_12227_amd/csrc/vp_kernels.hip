// vp_kernels.hip -- gfx950 kernels of one phase-space-conservation Vlasov step.
//
// Edelen & Webb, Sec. "An Algorithm Based on Phase Space Density Conservation":
// w_fin = Lambda^{-1} Delta^T w_in (eq. 10).  With tents of width h the overlap
// of a tent moved to u (in cells) with the tent of node c is h B3(u - c), B3 the
// centred cubic B-spline (eq. 9), and Lambda = h_x h_p M_x (x) M_p with
// M = tridiag(1/6, 2/3, 1/6) (eq. 8).  k_deposit forms b = Delta^T w / (h_x h_p),
// k_solve forms (M_x^{-1} (x) M_p^{-1}) b.  The state and the
// solves are FP32; the deposit's tap weights and products are FP64 (full rate
// on gfx950), rounded once into exact fixed-point tile sums; the FEL bunching
// sum and the diagnostics are FP64.
#include <mutex>

#include <hip/hip_ext.h>

#include "vp_internal.h"
#include "vp_device.h"

namespace vp {

// Push kinds of the deposit: a phase-dependent kick (free, pendulum, FEL by
// the exact-kick step), the exact rotation, and the FEL by Runge-Kutta.
// kPushMapped: a state-independent push read from the instance's cached map
// (time-invariant for a static Hamiltonian, formed once per plan by k_map).
enum PushKind { kPushPhase = 0, kPushSho = 1, kPushRk4 = 2, kPushMapped = 3 };

// Runge-Kutta stage constants of one FEL step of size h (cell units):
// slope of stage s, k_s = a_s cos psi_s + b_s sin psi_s, and
//   dv = cdv (k1 + 2 k2 + 2 k3 + k4),  du = drift + cdu (k1 + k2 + k3),
//   psi_2 = phi + q, psi_3 = psi_2 + t3 k1, psi_4 = psi_2 + q + t4 k2.
struct RkConsts {
    float a[4], b[4];
    float cdv, cdu, t3, t4;
};

// sin and cos of a Runge-Kutta stage angle t k (t = dz^2/4 or dz^2/2): for
// |x| < 2^-6 by their Taylor series to the x^5 and x^4 terms (the first
// omitted terms are below 3e-14 relative, far under FP32 rounding), with
// every operation written out so all inlined copies round alike; sincosf
// otherwise (a large field or step).
__device__ inline void sincos_stage(float x, float* s, float* c) {
#pragma clang fp contract(off)
    if (fabsf(x) < 0.015625f) {
        const float x2 = x * x;
        *s = x * fmaf(x2, fmaf(x2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
        *c = fmaf(x2, fmaf(x2, 1.0f / 24.0f, -0.5f), 1.0f);
    } else {
        sincosf(x, s, c);
    }
}

// Push one node: its displacement in cells, split into whole cells (ku, kv)
// and fractions (fu, fv) along x and p (the exact rotation, the FEL by
// Runge-Kutta, or a phase-dependent kick from the per-axis tables).
template <int PUSH>
__device__ inline void push_cells(float4 tx, float4 tp, float alpha, float beta, float kd, const RkConsts& rk,
                                  int& ku, float& fu, int& kv, float& fv) {
#pragma clang fp contract(off)  // the same bits in every inlined copy (see bspline_taps)
    if (PUSH == kPushSho) {
        float su, eu, sv, ev;
        two_sum(tx.x, tp.x, su, eu);
        two_sum(tx.z, tp.z, sv, ev);
        split_cell(su, eu + (tx.y + tp.y), ku, fu);
        split_cell(sv, ev + (tx.w + tp.w), kv, fv);
    } else if (PUSH == kPushRk4) {
        // the four stages of the FEL equations (eqs. 13a-c) at this node;
        // cos/sin of each stage phase by rotating the table's e^{i phi}
        const float k1 = fmaf(rk.a[0], tx.y, rk.b[0] * tx.x);
        const float c2 = fmaf(tx.y, tp.w, -(tx.x * tp.z));
        const float s2 = fmaf(tx.x, tp.w, tx.y * tp.z);
        const float k2 = fmaf(rk.a[1], c2, rk.b[1] * s2);
        float sn, cs;
        sincos_stage(rk.t3 * k1, &sn, &cs);
        const float c3 = fmaf(c2, cs, -(s2 * sn)), s3 = fmaf(s2, cs, c2 * sn);
        const float k3 = fmaf(rk.a[2], c3, rk.b[2] * s3);
        const float c2q = fmaf(c2, tp.w, -(s2 * tp.z)), s2q = fmaf(s2, tp.w, c2 * tp.z);
        sincos_stage(rk.t4 * k2, &sn, &cs);
        const float c4 = fmaf(c2q, cs, -(s2q * sn)), s4 = fmaf(s2q, cs, c2q * sn);
        const float k4 = fmaf(rk.a[3], c4, rk.b[3] * s4);
        const float dv = rk.cdv * ((k1 + k4) + 2.0f * (k2 + k3));
        float su, eu;
        two_sum(tp.x, rk.cdu * ((k1 + k2) + k3), su, eu);
        split_cell(su, eu + tp.y, ku, fu);
        split_cell(dv, 0.0f, kv, fv);
    } else {
        // phase phi_i + q_j from the per-axis sine/cosine tables
        const float cph = fmaf(tx.y, tp.w, -(tx.x * tp.z));
        const float sph = fmaf(tx.x, tp.w, tx.y * tp.z);
        const float dv = fmaf(alpha, cph, beta * sph);
        float su, eu;
        two_sum(tp.x, dv * kd, su, eu);
        split_cell(su, eu + tp.y, ku, fu);
        split_cell(dv, 0.0f, kv, fv);
    }
}

// Add the TAPS x TAPS B-spline taps of a node pushed to cell (ku + fu, kv + fv)
// from source row j, unwrapped column ii (weight w already scaled to fixed
// point) into the LDS tile: 4 x 4 cubic taps for tents, 6 x 6 quintic or
// 8 x 8 septic taps for quadratic or cubic basis functions.
template <int TAPS>
__device__ inline void scatter_node(long long* acc, int j, int ii, float w, int ku, float fu, int kv, float fv,
                                    int X0, int Y0, int tw, int th, int ldw) {
#pragma clang fp contract(off)
    // tap (q, r) lands on tile row row0 + q, column col0 + r; a node none of
    // whose taps meets the tile adds nothing (its lane sits the taps out).
    // The test also bounds every access: col0 in [1 - TAPS, tw) and row0 in
    // [1 - TAPS, th) put the taps inside the tile and its border of PAD >=
    // TAPS - 1 cells, whatever the push produced (a non-finite position
    // included).
    constexpr int LO = TAPS / 2 - 1, PAD = TAPS == 4 ? kPad : TAPS == 6 ? kPadQ : kPadC;
    static_assert(PAD >= TAPS - 1, "the tile border must take every tap of a node that meets the tile");
    const int col0 = ii + ku - LO - X0, row0 = j + kv - LO - Y0;
    if ((unsigned)(col0 + TAPS - 1) >= (unsigned)(tw + TAPS - 1) ||
        (unsigned)(row0 + TAPS - 1) >= (unsigned)(th + TAPS - 1))
        return;
    double bx[TAPS], bp[TAPS];
    basis_taps<TAPS>(fu, bx);
    basis_taps<TAPS>(fv, bp);
    long long* base = acc + __umul24(row0 + PAD, ldw) + (col0 + PAD);
    // tap value w * bp * bx: FP64 product, rounded once, exactly, into the
    // fixed-point tile sum, so the deposit adds no product rounding to the
    // state (the FEL instability amplifies it)
#pragma unroll
    for (int q = 0; q < TAPS; ++q) {
        const double wq = (double)w * bp[q];
        unsigned long long* row = (unsigned long long*)(base + q * ldw);
#pragma unroll
        for (int rr = 0; rr < TAPS; ++rr) atomicAdd(row + rr, fix48_word(wq, bx[rr]));
    }
}

template <int PUSH, int TAPS>
__device__ inline void deposit_node(long long* acc, int j, int ii, float w, float4 tx, float4 tp,
                                    float alpha, float beta, float kd, const RkConsts& rk, int X0, int Y0,
                                    int tw, int th, int ldw) {
    int ku, kv;
    float fu, fv;
    push_cells<PUSH>(tx, tp, alpha, beta, kd, rk, ku, fu, kv, fv);
    scatter_node<TAPS>(acc, j, ii, w, ku, fu, kv, fv, X0, Y0, tw, th, ldw);
}

// Spline bases: the taps of two sources of one column in consecutive rows
// j0, j0 + 1 (a work unit's row pair, starting at an even lattice row) merged
// into one (TAPS + 1) x (TAPS + 1) window when their whole cells agree along p
// and differ by at most one along x (their drifts differ by dt h_p / h_x
// cells): 49 atomics for a quadratic pair instead of 72, 81 for a cubic one
// instead of 128.  A window cell's word is the first source's
// tap rounded onto the fixed-point grid by the FMA with the 1.5 2^52
// constant, then the second's added by a second FMA, which rounds that tap
// onto the same integer grid (the first result is an integer of that
// binade): each tap is still rounded once.  Other pairs are scattered source
// by source.  (Measured: 7% off the quadratic deposit, 10% off the cubic one;
// slower for tents, whose loop is bound by instruction issue.)
template <int TAPS>
__device__ __attribute__((always_inline)) inline void scatter_pair(long long* acc, int j0, int j1, int ii, float w0,
                                                                   float w1, int ku0, float fu0,
                                    int kv0, float fv0, int ku1, float fu1, int kv1, float fv1, int X0, int Y0, int tw,
                                    int th, int ldw) {
#pragma clang fp contract(off)
    constexpr int LO = TAPS / 2 - 1, PAD = TAPS == 4 ? kPad : TAPS == 6 ? kPadQ : kPadC;
    static_assert(PAD >= TAPS, "the tile border must take the pair's window");
    const int base = min(ku0, ku1);
    const int d0 = ku0 - base, d1 = ku1 - base;
    if (j1 != j0 + 1 || kv1 != kv0 || (d0 | d1) > 1) {
        scatter_node<TAPS>(acc, j0, ii, w0, ku0, fu0, kv0, fv0, X0, Y0, tw, th, ldw);
        scatter_node<TAPS>(acc, j1, ii, w1, ku1, fu1, kv1, fv1, X0, Y0, tw, th, ldw);
        return;
    }
    // the window, rows row0 .. row0 + TAPS and columns col0 .. col0 + TAPS,
    // meets the tile or is skipped; one that meets it lies in the tile and
    // its border (PAD >= TAPS), whatever the push produced
    const int col0 = ii + base - LO - X0, row0 = j0 + kv0 - LO - Y0;
    if ((unsigned)(col0 + TAPS) >= (unsigned)(tw + TAPS) || (unsigned)(row0 + TAPS) >= (unsigned)(th + TAPS)) return;
    double bx0[TAPS], bp0[TAPS], bx1[TAPS], bp1[TAPS];
    basis_taps<TAPS>(fu0, bx0);
    basis_taps<TAPS>(fv0, bp0);
    basis_taps<TAPS>(fu1, bx1);
    basis_taps<TAPS>(fv1, bp1);
    double wq0[TAPS], wq1[TAPS];
#pragma unroll
    for (int q = 0; q < TAPS; ++q) {
        wq0[q] = (double)w0 * bp0[q];
        wq1[q] = (double)w1 * bp1[q];
    }
    long long* corner = acc + __umul24(row0 + PAD, ldw) + (col0 + PAD);
#pragma clang loop unroll(full)
    for (int c = 0; c <= TAPS; ++c) {
        // each source's x tap at window column c (its taps shifted by its offset)
        const double e0 = d0 ? (c >= 1 ? bx0[c - 1] : 0.0) : (c < TAPS ? bx0[c] : 0.0);
        const double e1 = d1 ? (c >= 1 ? bx1[c - 1] : 0.0) : (c < TAPS ? bx1[c] : 0.0);
        unsigned long long* colp = (unsigned long long*)(corner + c);
        // the last column holds taps only when the two sources' columns differ
        // (2% of the pairs at the benchmark's lattice): skipped when no lane of
        // the wavefront needs it
        if (c < TAPS || (d0 | d1)) {
#pragma clang loop unroll(full)
            for (int d = 0; d <= TAPS; ++d) {
                double v = kFixMagic;
                if (d < TAPS) v = fma(wq0[d], e0, v);
                if (d >= 1) v = fma(wq1[d - 1], e1, v);
                atomicAdd(colp + d * ldw, (unsigned long long)__double_as_longlong(v));
            }
        }
    }
}

// A push cell of the cached map of a state-independent push: whole cells
// packed as two 16-bit integers (ku low, kv high), fractions as a float pair.
__device__ inline void unpack_cells(int32_t k, int& ku, int& kv) {
    ku = (int)(int16_t)(k & 0xffff);
    kv = k >> 16;
}

// The box's sources go to the wavefronts in chunks claimed from an LDS
// counter: a wave that runs ahead takes more chunks, so the waves of a tile
// finish together (a static split leaves them waiting at the barrier for the
// slowest one).  The unit of work is a column of kU consecutive box rows (two
// for the spline bases, unit_rows): unit u = q bw + c covers rows kU q .. kU q
// + kU of box column c.  A chunk is 64
// consecutive units, one per lane, so no lane idles but in the last chunk (and
// past the box's last row); a lane wraps its column and reads its push table
// once for its kU sources, and neighbouring lanes read neighbouring columns of
// the same rows.  COL: 0 open x axis; 1 periodic, box within [-nx, 2 nx) (one
// correction per side); 2 periodic, general wrap.  Kind and wrap mode are
// template parameters, so the loop body is one basic block, free of per-node
// branches.
constexpr int kU = 4;  // sources (rows) per unit
// The spline bases take units of one row pair: a pair's two sets of taps
// leave no registers for a second pair's loads in flight (at four rows the
// quadratic loop spilled 24 bytes, the cubic one more, for no gain).
template <int TAPS>
constexpr int unit_rows() { return TAPS >= 6 ? 2 : kU; }

struct SourceScan {
    long long* acc;
    int* next;  // LDS: the first unclaimed unit
    gfloat* w;
    gfloat4* tab_x;
    gfloat4* tab_p;
    VP_GLOBAL const float2* map_f;  // kPushMapped: fractions (fu, fv) and packed whole cells per node
    VP_GLOBAL const int32_t* map_k;
    int nx, bx0, by0, bw, bh, nunits;
    float inv_nx, scale, alpha, beta, kd;
    double inv_bw;
    int X0, Y0, tw, th, ldw;
    RkConsts rk;
};

template <int PUSH, int COL, int TAPS>
__device__ inline void scan_sources(const SourceScan& S) {
    gfloat* __restrict__ w_g = S.w;
    gfloat4* __restrict__ tab_x = S.tab_x;
    gfloat4* __restrict__ tab_p = S.tab_p;
    settle(w_g);
    settle(tab_x);
    settle(tab_p);
    const int nx = S.nx, bw = S.bw, bh = S.bh, nunits = S.nunits;
    const int lane = (int)(threadIdx.x & 63);
    auto column = [&](int iu) {
        if (COL == 0) return iu;
        if (COL == 1) return iu + (iu < 0 ? nx : 0) - (iu >= nx ? nx : 0);
        return wrap_index(iu, nx, S.inv_nx);
    };
    for (;;) {
        int claim = 0;
        if (lane == 0) claim = atomicAdd(S.next, 64);
        const int u0 = __builtin_amdgcn_readfirstlane(claim);
        if (u0 >= nunits) break;
        // (row quad, column) of the lane's unit: an FP64 quotient, within one
        // unit of the exact one, then corrected; a unit past the box reads
        // the box's first node and weighs zero
        const int u = u0 + lane;
        const bool uvalid = u < nunits;
        int q = (int)((double)u * S.inv_bw);
        int c = u - q * bw;
        q += c < 0 ? -1 : (c >= bw ? 1 : 0);
        c += c < 0 ? bw : (c >= bw ? -bw : 0);
        const int iu = S.bx0 + (uvalid ? c : 0);
        const int i = column(iu);
        constexpr int UR = unit_rows<TAPS>();
        const int r0 = uvalid ? UR * q : 0;
        float4 tx;
        if (PUSH != kPushMapped) tx = tab_x[(unsigned)i];
        int jj[UR];
        float wv[UR];
        float4 tpv[UR];
        float2 mf[UR];
        int32_t mk[UR];
#pragma unroll
        for (int h = 0; h < UR; ++h) {
            const bool valid = uvalid && r0 + h < bh;
            jj[h] = S.by0 + (valid ? r0 + h : 0);
            const size_t node = (size_t)__umul24(jj[h], nx) + i;  // < 2^32: both axes have at most 2^16 nodes
            wv[h] = w_g[node];
            wv[h] = valid ? wv[h] : 0.0f;
            if (PUSH == kPushMapped) {
                mf[h] = S.map_f[node];
                mk[h] = S.map_k[node];
            } else {
                tpv[h] = tab_p[(unsigned)jj[h]];
            }
        }
        // keep the table loads above the skip test (issued with the weights)
        asm volatile("" ::: "memory");
        // a chunk whose weights are all zero (in every lane) adds nothing
        bool live = false;
#pragma unroll
        for (int h = 0; h < UR; ++h) live |= wv[h] != 0.0f;
        if (!__any(live)) continue;
        if constexpr (TAPS >= 6) {
#pragma unroll
            for (int h = 0; h < UR; h += 2) {
                int ku0, kv0, ku1, kv1;
                float fu0, fv0, fu1, fv1;
                if (PUSH == kPushMapped) {
                    unpack_cells(mk[h], ku0, kv0);
                    unpack_cells(mk[h + 1], ku1, kv1);
                    fu0 = mf[h].x;
                    fv0 = mf[h].y;
                    fu1 = mf[h + 1].x;
                    fv1 = mf[h + 1].y;
                } else {
                    push_cells<PUSH>(tx, tpv[h], S.alpha, S.beta, S.kd, S.rk, ku0, fu0, kv0, fv0);
                    push_cells<PUSH>(tx, tpv[h + 1], S.alpha, S.beta, S.kd, S.rk, ku1, fu1, kv1, fv1);
                }
                scatter_pair<TAPS>(S.acc, jj[h], jj[h + 1], iu, wv[h] * S.scale, wv[h + 1] * S.scale, ku0, fu0, kv0,
                                   fv0, ku1, fu1, kv1, fv1, S.X0, S.Y0, S.tw, S.th, S.ldw);
            }
            continue;
        }
#pragma unroll
        for (int h = 0; h < UR; ++h) {
            if (PUSH == kPushMapped) {
                int ku, kv;
                unpack_cells(mk[h], ku, kv);
                scatter_node<TAPS>(S.acc, jj[h], iu, wv[h] * S.scale, ku, mf[h].x, kv, mf[h].y, S.X0, S.Y0, S.tw, S.th,
                                   S.ldw);
            } else {
                deposit_node<PUSH, TAPS>(S.acc, jj[h], iu, wv[h] * S.scale, tx, tpv[h], S.alpha, S.beta, S.kd, S.rk,
                                         S.X0, S.Y0, S.tw, S.th, S.ldw);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_map: the push of every node of a static Hamiltonian, cached for the
// deposit (the node-to-destination map and the fractions that weigh its taps
// are the same every step when H does not depend on the state or the time).
// One thread per node, the same push code as the deposit: the cached cells
// are the bits the deposit would compute.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_map(const VpInst* inst) {
    const VpInst& I = *inst;
    const int nx = I.push.nx, np = I.push.np;
    const long n = (long)nx * np;
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int j = (int)(k / nx), i = (int)(k - (long)j * nx);
    const float4 tx = I.tab_x[i], tp = I.tab_p[j];
    int ku, kv;
    float fu, fv;
    const RkConsts rk{};
    if (I.push.kind == kSho) push_cells<kPushSho>(tx, tp, I.push.alpha, I.push.beta, I.push.kd, rk, ku, fu, kv, fv);
    else push_cells<kPushPhase>(tx, tp, I.push.alpha, I.push.beta, I.push.kd, rk, ku, fu, kv, fv);
    I.map_f[k] = make_float2(fu, fv);
    I.map_k[k] = (int32_t)(((uint32_t)ku & 0xffffu) | ((uint32_t)kv << 16));
}

// The per-tile FP64 bunching partials of an instance summed in one fixed
// order, whichever kernel sums them: thread t < kFieldThreads adds tiles t,
// t + kFieldThreads, ... in turn (kSumBatch tiles' loads in flight at once),
// each wavefront reduces by a shuffle tree, and thread 0 adds the first
// kFieldThreads / 64 wavefronts' sums in turn.  Every thread of the
// workgroup calls it (it holds a barrier); the sums are thread 0's.
__device__ inline void sum_tile_partials(const VpInst& I, double (&s_red)[kPartialsPerTile][kFieldThreads / 64],
                                         double (&sum)[kPartialsPerTile]) {
    constexpr int kSumBatch = 4;
    double acc[kPartialsPerTile] = {0.0, 0.0, 0.0, 0.0};
    const int n = I.k2_tiles;
    if (threadIdx.x < kFieldThreads)
        for (int k0 = threadIdx.x; k0 < n; k0 += kSumBatch * kFieldThreads) {
            double v[kSumBatch][kPartialsPerTile];
#pragma unroll
            for (int q = 0; q < kSumBatch; ++q) {
                const int k = min(k0 + q * kFieldThreads, n - 1);
#pragma unroll
                for (int c = 0; c < kPartialsPerTile; ++c) v[q][c] = I.partials[kPartialsPerTile * k + c];
            }
#pragma unroll
            for (int q = 0; q < kSumBatch; ++q)
                if (k0 + q * kFieldThreads < n)
#pragma unroll
                    for (int c = 0; c < kPartialsPerTile; ++c) acc[c] += v[q][c];
        }
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < kPartialsPerTile; ++c) acc[c] += __shfl_down(acc[c], o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0 && wid < kFieldThreads / 64)
        for (int c = 0; c < kPartialsPerTile; ++c) s_red[c][wid] = acc[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < kPartialsPerTile; ++c) {
            sum[c] = 0.0;
            for (int k = 0; k < kFieldThreads / 64; ++k) sum[c] += s_red[c][k];
        }
}

// The Runge-Kutta step's stage-3 and stage-4 bunchings from their summed
// partials, and the step's new field A + dz/6 (b1 + 2 b2 + 2 b3 + b4)
// (eq. 13c), every operation written out so that each kernel forming them
// rounds alike.
__device__ inline void rk4_stage_fields(const double (&a)[2], const double (&b1)[2], const double (&b2)[2], double n0,
                                        double h, const double (&sum)[kPartialsPerTile], double (&b3)[2],
                                        double (&b4)[2], double (&an)[2]) {
#pragma clang fp contract(off)
    const double inv_n0 = 1.0 / n0;
    for (int c = 0; c < 2; ++c) {
        b3[c] = sum[c] * inv_n0;
        b4[c] = sum[2 + c] * inv_n0;
        an[c] = a[c] + h / 6.0 * (((b1[c] + 2.0 * b2[c]) + 2.0 * b3[c]) + b4[c]);
    }
}

// ---------------------------------------------------------------------------
// k_deposit: push every node of the tile's source box and scatter its weight
// into the LDS image of the destination tile, then write the tile of b once.
// (Integer LDS atomics: gfx950 executes ds_add_f32 some 40x slower than
// ds_add_u32, and integer sums are order independent.)
// LDS holds (tx + 2 PAD) x (ty + 2 PAD) cells: the tile plus a border of PAD
// cells that takes the taps of nodes near the tile's edge which fall outside
// it; they are dropped with it.  TAPS: 4 (tents), 6 (quadratic basis) or 8
// (cubic basis).
// ---------------------------------------------------------------------------
template <int TAPS>
__global__ __launch_bounds__(TAPS == 8 ? kDepositCubicThreads : kDepositMaxThreads) void k_deposit(LaunchArgs A) {
    constexpr int PAD = TAPS == 4 ? kPad : TAPS == 6 ? kPadQ : kPadC;
    extern __shared__ __align__(16) long long acc[];  // 16-byte aligned: read four cells at a time
    __shared__ int s_d, s_box[4], s_next;
    __shared__ float s_ab[2];
    __shared__ RkConsts s_rk;
    __shared__ double s_stage[kPartialsPerTile][kFieldThreads / 64];

    for (int it = blockIdx.x; it < A.total; it += gridDim.x) {
        const int item = tile_of(it, A.total);
        if (threadIdx.x == 0) s_d = find_instance(A.off, A.ninst, item);
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_d);
        const VpInst& I = A.inst[d];
        const int t = item - A.off[d];
        const int tyi = t / I.k1_tiles_x, txi = t - tyi * I.k1_tiles_x;
        const int nx = I.push.nx, np = I.push.np;
        const int X0 = txi * I.k1_tx, X1 = min(X0 + I.k1_tx, nx);
        const int Y0 = tyi * I.k1_ty, Y1 = min(Y0 + I.k1_ty, np);
        const int ldw = I.k1_tx + 2 * PAD, ldh = I.k1_ty + 2 * PAD;
        const int par = (I.parity0 + A.parity) & 1;
        const float* __restrict__ w_in = I.w[par];

        // A launch with mode 1 (one Runge-Kutta FEL instance on tents, no field
        // launch after the stage sums): every workgroup sums the stage-3/4
        // partials itself, in the order the field kernel would (the same
        // bits).  Not compiled into the spline deposits, whose loops it would
        // crowd with spilled scalar registers.
        const bool stage_here = TAPS == 4 && A.mode == 1 && I.push.kind == kFel && I.push.rk4;
        double ssum[kPartialsPerTile] = {0.0, 0.0, 0.0, 0.0};
        if (stage_here) sum_tile_partials(I, s_stage, ssum);

        // a host-planned box: its load is in flight while the tile is cleared
        int4 hb = make_int4(0, 0, 0, 0);
        if (threadIdx.x == 0 && I.boxes) hb = I.boxes[t];
        for (int k = threadIdx.x; k < ldw * ldh; k += blockDim.x) acc[k] = 0ll;
        if (threadIdx.x == 0 && I.boxes) {
            s_ab[0] = I.push.alpha;
            s_ab[1] = I.push.beta;
            s_next = 0;
            s_box[0] = hb.x;
            s_box[1] = hb.y;
            s_box[2] = hb.z;
            s_box[3] = hb.w;
        } else if (threadIdx.x == 0) {
            PushParams P = I.push;
            if (P.kind == kFel && P.rk4) {
                // stage fields A_s and bunchings b_s of the Runge-Kutta step
                // (b1, b2 of the state, b3, b4 from k_fel_stage's partials), FP64
                double* st = I.fel_state;
                const double h = I.fel_dz, sg = (double)I.fel_sigma2;
                double b3[2], b4[2];
                if (stage_here) {
                    const double a0[2] = {st[kA], st[kA + 1]}, b1[2] = {st[kB1], st[kB1 + 1]};
                    const double b2[2] = {st[kBn], st[kBn + 1]};
                    double a_new[2];
                    rk4_stage_fields(a0, b1, b2, st[kN0], h, ssum, b3, b4, a_new);
                    // the instance's first tile keeps them for the field update
                    // after the solve (no workgroup of this launch reads them)
                    if (t == 0)
                        for (int c = 0; c < 2; ++c) {
                            st[kB3 + c] = b3[c];
                            st[kB4 + c] = b4[c];
                            st[kAn + c] = a_new[c];
                        }
                } else {
                    b3[0] = st[kB3];
                    b3[1] = st[kB3 + 1];
                    b4[0] = st[kB4];
                    b4[1] = st[kB4 + 1];
                }
                const double bre[4] = {st[kB1], st[kBn], b3[0], b4[0]};
                const double bim[4] = {st[kB1 + 1], st[kBn + 1], b3[1], b4[1]};
                const double cA[4] = {0.0, 0.5 * h, 0.5 * h, h};  // A_s = A + cA_s b_{s-1}
                double rmax = 0.0;
                for (int k = 0; k < 4; ++k) {
                    const double are = st[kA] + (k ? cA[k] * bre[k - 1] : 0.0);
                    const double aim = st[kA + 1] + (k ? cA[k] * bim[k - 1] : 0.0);
                    // F = -2 Re[(A + i sigma2 b) e^{i psi}] = a cos psi + b sin psi
                    const double re = are - sg * bim[k], im = aim + sg * bre[k];
                    s_rk.a[k] = (float)(-2.0 * re);
                    s_rk.b[k] = (float)(2.0 * im);
                    rmax = fmax(rmax, sqrt(re * re + im * im));
                }
                const double hp = (double)P.hp, hx = (double)P.hx;
                s_rk.cdv = (float)(h / (6.0 * hp));
                s_rk.cdu = (float)(h * h / (6.0 * hx));
                s_rk.t3 = (float)(0.25 * h * h);
                s_rk.t4 = (float)(0.5 * h * h);
                // |dv| <= (h / hp) 2 max_s |A_s + i sigma2 b_s|; |du - drift| <= kd |dv|max
                P.alpha = (float)(2.0 * h / hp * rmax);
                P.beta = 0.0f;
            } else if (P.kind == kFel) {
                // kick field: A at mid-kick plus the space-charge term, A + b dz/2 + i sigma2 b
                const double* st = I.fel_state;
                double are = st[kA] + 0.5 * I.fel_dz * st[kBn] - (double)I.fel_sigma2 * st[kBn + 1];
                double aim = st[kA + 1] + 0.5 * I.fel_dz * st[kBn + 1] + (double)I.fel_sigma2 * st[kBn];
                P.alpha = (float)(I.fel_kick * are);
                P.beta = (float)(-I.fel_kick * aim);
            }
            s_ab[0] = P.alpha;
            s_ab[1] = P.beta;
            s_next = 0;
            source_box(P, X0, X1, Y0, Y1, s_box);
        }
        __syncthreads();

        // the box is the same for every lane: said so, the loop's branches on it
        // are scalar
        const int bx0 = __builtin_amdgcn_readfirstlane(s_box[0]);
        const int bx1 = __builtin_amdgcn_readfirstlane(s_box[1]);
        // spline bases: the box starts at an even row, so the work units' row
        // pairs are the lattice's (2m, 2m + 1) in every tile and their merged
        // sums do not depend on the tiling
        const int by0_box = __builtin_amdgcn_readfirstlane(s_box[2]);
        const int by0 = TAPS >= 6 ? (by0_box & ~1) : by0_box;
        const int bh = __builtin_amdgcn_readfirstlane(s_box[3]) - by0;
        const int bw = max(bx1 - bx0, 1);
        const int nsrc = (bx1 > bx0 && bh > 0) ? bw * bh : 0;
        const float inv_nx = 1.0f / (float)nx;
        const float alpha = s_ab[0], beta = s_ab[1], kd = I.push.kd;
        const int kind = I.push.kind;
        const bool periodic = I.push.x_periodic != 0;

        // Tile sums are exact fixed-point integers: every tap value is rounded
        // to a multiple of 2^-40 of 2^e > max|w0| (the instance's initial
        // weights) and summed with 64-bit integer LDS atomics, so the sum does
        // not depend on the order of the atomics or on the tiling (bitwise
        // reproducible).  The map is area preserving and the weights are
        // carried along it, so a cell collects about max|w|; a cell sum must
        // stay below 2^7 x 2^e (2^47 units, fix48_value): cells beyond 2^6 x 2^e
        // set the instance's range flag.
        const float scale = I.fix_scale, inv_scale = I.fix_inv;  // exact powers of two
        const int nsrc_live = scale > 0.0f ? nsrc : 0;

        // On a periodic axis the column wraps with one correction per side
        // while the box lies within [-nx, 2 nx) (always, unless the lattice is
        // narrower than the box).
        SourceScan S;
        S.acc = acc;
        S.next = &s_next;
        S.w = as_global(w_in);
        S.tab_x = as_global(I.tab_x);
        S.tab_p = as_global(I.tab_p);
        S.nx = nx;
        S.bx0 = bx0;
        S.by0 = by0;
        S.bw = bw;
        S.bh = bh;
        S.nunits = nsrc_live > 0 ? bw * ((bh + unit_rows<TAPS>() - 1) / unit_rows<TAPS>()) : 0;
        S.inv_nx = inv_nx;
        S.inv_bw = 1.0 / (double)bw;
        S.scale = scale;
        S.alpha = alpha;
        S.beta = beta;
        S.kd = kd;
        S.X0 = X0;
        S.Y0 = Y0;
        S.tw = X1 - X0;
        S.th = Y1 - Y0;
        S.ldw = ldw;
        const bool rk4 = kind == kFel && I.push.rk4;
        if (rk4) {
            auto uni = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
            for (int k = 0; k < 4; ++k) {
                S.rk.a[k] = uni(s_rk.a[k]);
                S.rk.b[k] = uni(s_rk.b[k]);
            }
            S.rk.cdv = uni(s_rk.cdv);
            S.rk.cdu = uni(s_rk.cdu);
            S.rk.t3 = uni(s_rk.t3);
            S.rk.t4 = uni(s_rk.t4);
        }
        const bool wrap_near = bx0 >= -nx && bx0 + bw <= 2 * nx;
        const int col = !periodic ? 0 : wrap_near ? 1 : 2;
        S.map_f = (VP_GLOBAL const float2*)I.map_f;
        S.map_k = (VP_GLOBAL const int32_t*)I.map_k;
        if (I.map_f) {
            if (col == 0) scan_sources<kPushMapped, 0, TAPS>(S);
            else if (col == 1) scan_sources<kPushMapped, 1, TAPS>(S);
            else scan_sources<kPushMapped, 2, TAPS>(S);
        } else if (kind == kSho) {
            if (col == 0) scan_sources<kPushSho, 0, TAPS>(S);
            else if (col == 1) scan_sources<kPushSho, 1, TAPS>(S);
            else scan_sources<kPushSho, 2, TAPS>(S);
        } else if (rk4) {
            if (col == 0) scan_sources<kPushRk4, 0, TAPS>(S);
            else if (col == 1) scan_sources<kPushRk4, 1, TAPS>(S);
            else scan_sources<kPushRk4, 2, TAPS>(S);
        } else {
            if (col == 0) scan_sources<kPushPhase, 0, TAPS>(S);
            else if (col == 1) scan_sources<kPushPhase, 1, TAPS>(S);
            else scan_sources<kPushPhase, 2, TAPS>(S);
        }
        __syncthreads();

        const int tw = X1 - X0, th = Y1 - Y0;
        const int T = blockDim.x;
        gfloat_out* __restrict__ b = as_global_out(I.b);
        bool out_of_range = false;
        // A cell goes out as v 2^(e-40) rounded once to FP32 (v, 48 bits, is
        // exact in FP64 and the scale is a power of two).
        const double inv_scale_d = (double)inv_scale;
        auto cell = [&](long long word) {
            const long long v = fix48_value(word);
            out_of_range |= (unsigned long long)v + (1ull << 46) >= (1ull << 47);
            return (float)((double)v * inv_scale_d);
        };
        // Thread t takes items k = t, t + T, ... of the tile, k = rr w + cc:
        // (rr, cc) advance by (T / w, T % w) with one carry.
        if ((I.k1_tx & 3) == 0 && (nx & 3) == 0) {
            // four consecutive cells per item (two 16-byte LDS reads, one
            // 16-byte store): rows of the tile and of b start 16-byte
            // aligned (the pad is even)
            const int tq = tw >> 2;
            const int wdr = T / tq, wdc = T - wdr * tq;
            int rr = (int)threadIdx.x / tq, cq = (int)threadIdx.x - rr * tq;
            while (rr < th) {
                const long long* src = acc + (rr + PAD) * ldw + 4 * cq + PAD;
                const longlong2 a0 = reinterpret_cast<const longlong2*>(src)[0];
                const longlong2 a1 = reinterpret_cast<const longlong2*>(src)[1];
                const float4 o = make_float4(cell(a0.x), cell(a0.y), cell(a1.x), cell(a1.y));
                reinterpret_cast<VP_GLOBAL float4*>(b + (size_t)(Y0 + rr) * nx + X0)[cq] = o;
                cq += wdc;
                rr += wdr;
                const bool carry = cq >= tq;
                cq -= carry ? tq : 0;
                rr += carry ? 1 : 0;
            }
        } else {
            const int wdr = T / tw, wdc = T - wdr * tw;
            int rr = (int)threadIdx.x / tw, cc = (int)threadIdx.x - rr * tw;
            while (rr < th) {
                b[(size_t)(Y0 + rr) * nx + X0 + cc] = cell(acc[(rr + PAD) * ldw + cc + PAD]);
                cc += wdc;
                rr += wdr;
                const bool carry = cc >= tw;
                cc -= carry ? tw : 0;
                rr += carry ? 1 : 0;
            }
        }
        // one flag write per wavefront that saw a cell out of range: an
        // atomic per thread on one address would serialise the whole launch
        if (__any(out_of_range) && (threadIdx.x & 63) == 0) {
            atomicOr(&I.counters[kRangeFlag], 1u);
            atomicOr(A.any_range, 1u);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_solve: w_new = (M_x^{-1} (x) M_p^{-1}) b in one pass, one lattice line per
// lane (line_solve: the LU recursions of T = tridiag(1,4,1),
//   forward  z_k = r_k - m_k z_{k-1},   backward c_k = (z_k - c_{k+1}) / d_k,
// with exact per-node (m_k, 1/d_k) on a line that starts at an open edge).
// The two factors commute, so the p solves go first.  A workgroup (one
// wavefront) owns a kSegX x kSegP output tile inside the kLineX x kLineP
// window around it: kHalo more nodes on every side, wrapped on a periodic
// axis and shifted to end at the edge on an open one.  Where the window is
// cut inside the lattice the recursions start from zero, an error that decays
// by 2 - sqrt 3 per node and is ~7e-10 at the tile.
//  p phase: lane c loads window column c of b straight into registers (each
//    load instruction reads one row's kLineX consecutive nodes: two cache
//    lines), solves it along p and puts the kept rows into LDS.
//  x phase: lane r solves kept row r along x in LDS.
//  out:     the kept columns of the kept rows go out, two rows per store.
// The intermediate never leaves LDS (16.6 KB), and with at most 256 VGPRs
// eight tiles are resident per compute unit: all 2048 tiles of a 2048^2
// lattice at once.  For the FEL the write-out also forms the FP64 bunching
// partials of the new state, per tile (k_fel_field sums them).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSolveThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_solve(LaunchArgs A) {
    static_assert(kSolveThreads == kLineX && kSolveThreads == kSegP && kSegX * 2 == kSolveThreads,
                  "p phase: a window column per lane; x phase: a kept row per lane; out: two rows per store");
    // kept rows at pitch ldx: 16-byte aligned, and the 16-byte accesses of
    // consecutive rows (x phase, lane = row) fall on disjoint banks
    constexpr int ldx = kLineX + 4;
    constexpr int kStageRows = kSegP;  // window rows staged in LDS (the rest in registers)
    static_assert(kStageRows * kLineX <= kSegP * ldx, "the staged rows fit the LDS of the kept rows");
    __shared__ float xs[kSegP * ldx];  // staged rows, then the kept rows p-solved, then x-solved in place
    __shared__ double2 s_eq[kSegP];    // FEL: e^{iq} of the tile's rows
    __shared__ int s_d;

    for (int it = blockIdx.x; it < A.total; it += gridDim.x) {
        const int item = tile_of(it, A.total);
        if (threadIdx.x == 0) s_d = find_instance(A.off, A.ninst, item);
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_d);
        const VpInst& I = A.inst[d];
        const int t = item - A.off[d];
        const int nx = I.push.nx, np = I.push.np;
        const bool periodic = I.push.x_periodic != 0;
        const int tiles_x = (nx + kSegX - 1) / kSegX;
        const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
        const int X0 = txi * kSegX, tw = min(kSegX, nx - X0);
        const int Y0 = tyi * kSegP, th = min(kSegP, np - Y0);
        // windows (x unwrapped on a periodic axis)
        const int wx = periodic ? X0 - kHalo : open_window(X0, nx, kLineX);
        const int nwx = periodic ? kLineX : min(kLineX, nx);
        const int wp = open_window(Y0, np, kLineP), nwp = min(kLineP, np);
        const int kind_p = nwp < kLineP ? 2 : (wp == 0 ? 1 : 0);
        const int lo_p = Y0 - wp;  // the kept rows are window rows lo_p .. lo_p + th
        const int par = (I.parity0 + A.parity) & 1;
        gfloat_out* __restrict__ dst = as_global_out(I.w[par ^ 1]);
        const int lane = threadIdx.x;

        const bool fel = I.push.kind == kFel;
        if (fel && lane < th) s_eq[lane] = I.fel_eq[Y0 + lane];

        // p: lane = window column c (columns past a narrow open lattice are zero)
        {
            // stage the window: rows 0 .. kStageRows go straight into LDS, row k
            // at xs + k kLineX (global_load_lds: one row's kLineX consecutive
            // nodes per instruction, no registers hold the data), the rest into
            // registers through a buffer resource based at the window's first
            // row (the row's byte offset is wave-uniform, the lane's column
            // offset 32 bits); all rows in flight, rows past a short lattice zero
            float v[kLineP];
            {
                const int rows = kind_p == 2 ? nwp : kLineP;
                const int rows_lds = min(rows, kStageRows);
                int gc = wx + lane;
                if (periodic) gc = wrap_index(gc, nx, 1.0f / (float)nx);
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void*)(I.b + (size_t)wp * nx), (short)0, -1, kBufferWord3);
                const int ub = gc * 4;         // < 2^18: a row has at most 2^16 nodes
                const int row_bytes = nx * 4;  // k row_bytes < kLineP 2^18
                if (lane < nwx) {
                    gfloat* p = as_global(I.b) + (size_t)wp * nx + gc;
                    for (int k = 0; k < rows_lds; ++k)
                        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(p + (size_t)k * nx),
                                                         (__attribute__((address_space(3))) void*)(xs + k * kLineX), 4, 0, 0);
                    if (rows == kLineP) {
#pragma unroll
                        for (int k = kStageRows; k < kLineP; ++k)
                            v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, ub, k * row_bytes, 0));
                    } else {
#pragma unroll
                        for (int k = kStageRows; k < kLineP; ++k)
                            v[k] = k < rows ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, ub, k * row_bytes, 0)) : 0.0f;
                    }
                } else {
                    for (int k = 0; k < rows_lds; ++k) xs[k * kLineX + lane] = 0.0f;
#pragma unroll
                    for (int k = kStageRows; k < kLineP; ++k) v[k] = 0.0f;
                }
                for (int k = rows_lds; k < kStageRows; ++k) xs[k * kLineX + lane] = 0.0f;
                __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            }
#pragma unroll
            for (int k = 0; k < kStageRows; ++k) v[k] = xs[k * kLineX + lane];
            // Every lane has its column in registers before any kept row is
            // written over the staging image (the LDS operations of one
            // wavefront take effect in program order).
            float* out = xs + lane;
            if (kind_p == 0) {
                line_solve<kLineP, kHalo, false, false>(v, nwp);
                if (lo_p == kHalo) {
#pragma unroll
                    for (int r = 0; r < kSegP; ++r) out[r * ldx] = v[kHalo + r];
                } else {
                    const int lov = (int)in_vgpr((unsigned)lo_p);
#pragma unroll
                    for (int k = kHalo; k < kLineP; ++k)
                        if ((unsigned)(k - lov) < (unsigned)kSegP) out[(k - lov) * ldx] = v[k];
                }
            } else if (kind_p == 1 && lo_p == 0 && th == kSegP) {
                // a full window at the open edge that keeps its first kSegP
                // rows: the halo's results are dead, so v[kSegP..] frees early
                line_solve<kLineP, 0, true, false>(v, nwp);
#pragma unroll
                for (int r = 0; r < kSegP; ++r) out[r * ldx] = v[r];
            } else {
                // a short lattice (masked) or a window at the edge that keeps
                // other rows: z goes to the staging image (this lane's column
                // of it, b being in registers by now), and the kept rows are
                // written once every z has been read back
                if (kind_p == 2) line_solve_lds<kLineP, kStageRows, true>(v, nwp, xs + lane, kLineX);
                else line_solve_lds<kLineP, kStageRows, false>(v, nwp, xs + lane, kLineX);
#pragma unroll
                for (int k = 0; k < kLineP; ++k)
                    if ((unsigned)(k - lo_p) < (unsigned)th) out[(k - lo_p) * ldx] = v[k];
            }
        }
        __syncthreads();

        // x: lane = kept row r, solved in place (rows past the tile are solved and dropped)
        {
            float v[kLineX];
            float4* row = reinterpret_cast<float4*>(xs + lane * ldx);
#pragma unroll
            for (int q = 0; q < kLineX / 4; ++q) {
                const float4 a = row[q];
                v[4 * q] = a.x;
                v[4 * q + 1] = a.y;
                v[4 * q + 2] = a.z;
                v[4 * q + 3] = a.w;
            }
            int q0 = 0, q1 = kLineX / 4;  // quads written back
            if (periodic) {
                line_solve<kLineX, kHalo, false, false>(v, kLineX);
                q0 = kHalo / 4;
                q1 = (kHalo + kSegX) / 4;
            } else {
                const int kind_x = nwx < kLineX ? 2 : (wx == 0 ? 1 : 0);
                if (kind_x == 2) line_solve<kLineX, 0, true, true>(v, nwx);
                else if (kind_x == 1) line_solve<kLineX, 0, true, false>(v, nwx);
                else line_solve<kLineX, 0, false, false>(v, nwx);
            }
#pragma unroll
            for (int q = 0; q < kLineX / 4; ++q)
                if (q >= q0 && q < q1) row[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        }
        __syncthreads();

        // out: the kept columns of the kept rows; FEL: the bunching sums
        const bool rk4 = fel && I.push.rk4;
        double acc_re = 0.0, acc_im = 0.0, acc1_re = 0.0, acc1_im = 0.0;
        const int lo_x = X0 - wx;  // the kept columns are window columns lo_x .. lo_x + tw
        if ((nx & 3) == 0 && (lo_x & 3) == 0) {
            // lane = column quad q of rows (lane / kQuads) + kRowsPer i: 16-byte
            // LDS reads and stores, kRowsPer rows per store (rows of b and of
            // the tile start 16-byte aligned, and tw is a multiple of four)
            constexpr int kQuads = kSegX / 4, kRowsPer = kSolveThreads / kQuads;
            const int q = lane & (kQuads - 1), r0 = lane / kQuads;
            if (4 * q < tw) {
                const float* in = xs + r0 * ldx + lo_x + 4 * q;
                gfloat_out* o = dst + (size_t)(Y0 + r0) * nx + X0 + 4 * q;
                unsigned qo = in_vgpr(0u);  // running offset of the row (< kSegP rows x nx)
                double cre[4] = {0.0, 0.0, 0.0, 0.0}, cim[4] = {0.0, 0.0, 0.0, 0.0}, c1[4] = {0.0, 0.0, 0.0, 0.0};
                auto row = [&](int i) {
                    const float4 y = *reinterpret_cast<const float4*>(in + i * kRowsPer * ldx);
                    *reinterpret_cast<VP_GLOBAL float4*>(o + qo) = y;
                    qo += (unsigned)(kRowsPer * nx);
                    if (fel) {
                        const double2 e = s_eq[r0 + kRowsPer * i];  // times e^{-i q}
                        const float yy[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            cre[j] += (double)yy[j] * e.x;
                            cim[j] -= (double)yy[j] * e.y;
                            if (rk4) c1[j] += (double)yy[j];
                        }
                    }
                };
                const int rows = (th - r0 + kRowsPer - 1) / kRowsPer;  // this lane's kept rows
                if (rows == kSegP / kRowsPer) {
#pragma unroll
                    for (int i = 0; i < kSegP / kRowsPer; ++i) row(i);
                } else {
                    for (int i = 0; i < rows; ++i) row(i);
                }
                if (fel) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double2 e = I.fel_ex[X0 + 4 * q + j];  // times e^{-i phi}
                        acc_re += cre[j] * e.x + cim[j] * e.y;
                        acc_im += cim[j] * e.x - cre[j] * e.y;
                        acc1_re += c1[j] * e.x;
                        acc1_im -= c1[j] * e.y;
                    }
                }
            }
        } else {
            // lane = kept column c of rows (lane / kSegX) + 2 i, two rows per store
            const int c = lane & (kSegX - 1), r0 = lane / kSegX;
            if (c < tw) {
                const float* in = xs + r0 * ldx + lo_x + c;
                gfloat_out* o = dst + (size_t)(Y0 + r0) * nx + X0 + c;
                unsigned qo = in_vgpr(0u);  // running offset of the row (< kSegP rows x nx)
                double cre = 0.0, cim = 0.0, c1 = 0.0;
                const int rows = (th - r0 + 1) >> 1;  // this lane's kept rows
                if (rows == kSegP / 2) {
#pragma unroll
                    for (int i = 0; i < kSegP / 2; ++i) {
                        const float y = in[2 * i * ldx];
                        o[qo] = y;
                        qo += 2u * (unsigned)nx;
                        if (fel) {
                            const double2 e = s_eq[r0 + 2 * i];  // times e^{-i q}
                            cre += (double)y * e.x;
                            cim -= (double)y * e.y;
                            if (rk4) c1 += (double)y;
                        }
                    }
                } else {
                    for (int i = 0; i < rows; ++i) {
                        const float y = in[2 * i * ldx];
                        o[qo] = y;
                        qo += 2u * (unsigned)nx;
                        if (fel) {
                            const double2 e = s_eq[r0 + 2 * i];
                            cre += (double)y * e.x;
                            cim -= (double)y * e.y;
                            if (rk4) c1 += (double)y;
                        }
                    }
                }
                if (fel) {
                    const double2 e = I.fel_ex[X0 + c];  // times e^{-i phi}
                    acc_re = cre * e.x + cim * e.y;
                    acc_im = cim * e.x - cre * e.y;
                    acc1_re = c1 * e.x;
                    acc1_im = -c1 * e.y;
                }
            }
        }

        if (fel) {
            // FP64 bunching of the new state: this tile's partials, at the
            // half-drift phases and (Runge-Kutta) at the lattice phases
            // (k_fel_field sums the partials)
            for (int o = 32; o > 0; o >>= 1) {
                acc_re += __shfl_down(acc_re, o);
                acc_im += __shfl_down(acc_im, o);
                acc1_re += __shfl_down(acc1_re, o);
                acc1_im += __shfl_down(acc1_im, o);
            }
            if (lane == 0) {
                double* pt = I.partials + kPartialsPerTile * t;
                pt[0] = acc_re;
                pt[1] = acc_im;
                pt[2] = acc1_re;
                pt[3] = acc1_im;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Spline bases: the mass matrix (eq. 8) of B-spline basis functions of degree
// d is M = P / scale, P the symmetric Toeplitz band of the degree-(2d+1)
// spline at the integers, truncated at an open edge: BW = d sub-diagonals,
// P = pentadiag(1, 26, 66, 26, 1) / 120 (quadratic), or
// heptadiag(1, 120, 1191, 2416, 1191, 120, 1) / 5040 (cubic).
// P = L D L^T with L unit lower triangular with BW sub-diagonals (l_m(k): row
// k, column k - m).  On a line that starts at an open edge the factors of the
// first rows are those of the truncated matrix; they reach their interior
// limits (set by the poles of the band's symbol: -0.0431 and -0.4306 for the
// quadratic, down to -0.5353 for the cubic) to FP32 precision within ~10 and
// ~20 rows; band_edge_rows(BW) rows are tabulated at compile time (FP64,
// rounded once), the fewest that reach the limits (every tabulated row of a
// line costs a scalar select per factor).
// The truncation at the far end of a line changes no factor, so the same
// table serves lines that end at an edge.
// ---------------------------------------------------------------------------
constexpr int band_edge_rows(int bw) { return bw == 2 ? 16 : kEdgeQ; }

template <int BW>
struct BandLdl {
    float l[BW + 1][kEdgeQ + 1];  // l[m][k], m = 1 .. BW; row kEdgeQ: the interior limits
    float dinv[kEdgeQ + 1];       // scale / d_k
};

template <int BW>
constexpr BandLdl<BW> band_ldl_table(const double (&c)[BW + 1], double scale) {
    constexpr int K = 128;
    double d[K] = {}, l[K][BW + 1] = {};
    for (int k = 0; k < K; ++k) {
        // l_m(k) for m = BW .. 1 (the sums use the larger offsets, done first)
        for (int m = BW; m >= 1; --m) {
            const int j = k - m;
            if (j < 0) continue;
            double acc = c[m];
            for (int i = (k - BW > 0 ? k - BW : 0); i < j; ++i) acc -= l[k][k - i] * d[i] * l[j][j - i];
            l[k][m] = acc / d[j];
        }
        double dk = c[0];
        for (int m = 1; m <= BW && m <= k; ++m) dk -= l[k][m] * l[k][m] * d[k - m];
        d[k] = dk;
    }
    BandLdl<BW> T{};
    for (int k = 0; k <= kEdgeQ; ++k) {
        const int r = k < band_edge_rows(BW) ? k : K - 1;
        for (int m = 1; m <= BW; ++m) T.l[m][k] = (float)l[r][m];
        T.dinv[k] = (float)(scale / d[r]);
    }
    return T;
}
constexpr double kBandQuad[3] = {66.0, 26.0, 1.0};
constexpr double kBandCubic[4] = {2416.0, 1191.0, 120.0, 1.0};
// namespace-scope constants, so that unrolled code folds every factor into an
// instruction operand
constexpr BandLdl<2> kBandLdl2 = band_ldl_table<2>(kBandQuad, 120.0);
constexpr BandLdl<3> kBandLdl3 = band_ldl_table<3>(kBandCubic, 5040.0);
template <int BW>
__host__ __device__ constexpr const BandLdl<BW>& band_table() {
    if constexpr (BW == 2) return kBandLdl2;
    else return kBandLdl3;
}

// Solve M y = v in place along one whole window line (kLineQ elements) held
// in registers (every index is a constant: the interior factors are
// instruction operands).  edge: the line starts at an open edge (the
// tabulated first rows, chosen by scalar selects); else it starts at a cut
// inside the lattice or on a periodic wrap, where the recursions start from
// zero with the interior factors, an error that decays with the slowest pole.
// The far end needs no flag (see above); a cut there starts the backward
// recursion from zero, with the same decay.  The terms of the older
// neighbours are added first, so each recursion step waits on one fused
// multiply-add of the step before.
template <int BW>
__device__ inline void band_line(float (&v)[kLineQ], bool edge) {
    constexpr const BandLdl<BW>& T = band_table<BW>();
    constexpr int E = band_edge_rows(BW);
    auto lm = [&](int m, int k) { return k < E && edge ? T.l[m][k] : T.l[m][kEdgeQ]; };
    auto dinv = [&](int k) { return k < E && edge ? T.dinv[k] : T.dinv[kEdgeQ]; };
    // forward: z_k = v_k - sum_m l_m(k) z_{k-m};  v_k <- z_k / d_k
    float z[BW + 1] = {};  // z[m]: z_{k-m}
#pragma unroll
    for (int k = 0; k < kLineQ; ++k) {
        float acc = v[k];
#pragma unroll
        for (int m = BW; m >= 1; --m) acc = fmaf(-lm(m, k), z[m], acc);
#pragma unroll
        for (int m = BW; m >= 2; --m) z[m] = z[m - 1];
        z[1] = acc;
        v[k] = acc * dinv(k);
    }
    // backward: y_k = v_k - sum_m l_m(k+m) y_{k+m}
    float y[BW + 1] = {};  // y[m]: y_{k+m}
#pragma unroll
    for (int k = kLineQ - 1; k >= 0; --k) {
        float acc = v[k];
#pragma unroll
        for (int m = BW; m >= 1; --m) acc = fmaf(-lm(m, k + m), y[m], acc);
#pragma unroll
        for (int m = BW; m >= 2; --m) y[m] = y[m - 1];
        y[1] = acc;
        v[k] = acc;
    }
}

// The same solve along a line of n <= kLineQ elements in LDS, v[k * S], for
// lattice axes shorter than the window (taken whole): a loop, the values
// going through registers U at a time.
template <int S, int BW>
__device__ inline void band_line_lds(float* v, int n, bool edge) {
    constexpr const BandLdl<BW>& T = band_table<BW>();
    constexpr int U = 8, E = band_edge_rows(BW);
    static_assert(E % U == 0, "a group of rows is wholly inside or outside the table");
    float z[BW + 1] = {};
    for (int k0 = 0; k0 < n; k0 += U) {
        float r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = k0 + u < n ? v[(k0 + u) * S] : 0.0f;
        const bool tab = edge && k0 < E;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tab ? k0 + u : kEdgeQ;
            float acc = r[u];
#pragma unroll
            for (int m = BW; m >= 1; --m) acc = fmaf(-T.l[m][k], z[m], acc);
#pragma unroll
            for (int m = BW; m >= 2; --m) z[m] = z[m - 1];
            z[1] = acc;
            r[u] = acc * T.dinv[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < n) v[(k0 + u) * S] = r[u];
    }
    float y[BW + 1] = {};
    for (int k1 = n - 1; k1 >= 0; k1 -= U) {
        float r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = k1 - u >= 0 ? v[(k1 - u) * S] : 0.0f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k1 - u;
            float acc = r[u];
#pragma unroll
            for (int m = BW; m >= 1; --m) acc = fmaf(-T.l[m][edge && k + m < E ? k + m : kEdgeQ], y[m], acc);
#pragma unroll
            for (int m = BW; m >= 2; --m) y[m] = y[m - 1];
            y[1] = acc;
            r[u] = acc;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k1 - u >= 0) v[(k1 - u) * S] = r[u];
    }
}

// FEL: a solve tile's FP64 bunching of the new state, the sums over its kept
// nodes of w e^{-i(phi_i + q_j)} (half-drift phases) and of w e^{-i phi_i}
// (lattice phases, the Runge-Kutta step's stage 1); k_fel_field sums the
// tiles.  v: this thread's parts.  Called by every thread.
__device__ inline void spline_tile_partials(double* pt, double (&v)[kPartialsPerTile],
                                          double (&s_red)[kSolveQThreads / 64][kPartialsPerTile]) {
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < kPartialsPerTile; ++c) v[c] += __shfl_down(v[c], o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < kPartialsPerTile; ++c) s_red[wid][c] = v[c];
    __syncthreads();
    if (threadIdx.x < kPartialsPerTile) {
        double a = 0.0;
        for (int k = 0; k < kSolveQThreads / 64; ++k) a += s_red[k][threadIdx.x];
        pt[threadIdx.x] = a;
    }
}

// The kept nodes of a solve tile out of LDS (kept row r at win[r * kPitchQ],
// column c at ox + c), whole rows per store; for the FEL also the tile's
// bunching partials.
__device__ inline void spline_tile_out(const VpInst& I, int t, const float* win, int ox, int X0, int kw, int P0, int kp,
                                     int nx, float* dst, double (&s_red)[kSolveQThreads / 64][kPartialsPerTile]) {
    const int tid = threadIdx.x;
    const bool fel = I.push.kind == kFel;
    double v[kPartialsPerTile] = {0.0, 0.0, 0.0, 0.0};
    if (tid < kw) {
        float* out = dst + (size_t)P0 * nx + X0 + tid;
        const float* in = win + ox + tid;
        if (!fel) {
            for (int r = 0; r < kp; ++r) out[(size_t)r * nx] = in[r * kPitchQ];
        } else {
            double cre = 0.0, cim = 0.0, c1 = 0.0;
            for (int r = 0; r < kp; ++r) {
                const float y = in[r * kPitchQ];
                out[(size_t)r * nx] = y;
                const double2 e = I.fel_eq[P0 + r];  // times e^{-i q}
                cre += (double)y * e.x;
                cim -= (double)y * e.y;
                c1 += (double)y;
            }
            const double2 e = I.fel_ex[X0 + tid];  // times e^{-i phi}
            v[0] = cre * e.x + cim * e.y;
            v[1] = cim * e.x - cre * e.y;
            v[2] = c1 * e.x;
            v[3] = -c1 * e.y;
        }
    }
    if (fel) spline_tile_partials(I.partials + kPartialsPerTile * t, v, s_red);
}

// Window geometry of a solve tile (spline basis of band BW): kept nodes
// [X0, X0 + kw) x [P0, P0 + kp), seg x seg at most; window columns
// [xs, xs + lx) (unwrapped on a periodic axis: always a whole line there, the
// halo on the far side of a narrow last tile only longer) and rows
// [ps, ps + lp), shifted to end at an open edge; an open axis shorter than the
// window is taken whole.
template <int BW>
struct SplineTile {
    static constexpr int kHalo = spline_halo(BW), kSeg = spline_seg(BW);
    int nx, np, X0, kw, P0, kp, lx, xs, lp, ps, ox, op;
    bool periodic;
    __device__ SplineTile(const VpInst& I, int t) {
        nx = I.push.nx;
        np = I.push.np;
        periodic = I.push.x_periodic != 0;
        const int tiles_x = (nx + kSeg - 1) / kSeg;
        const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
        X0 = txi * kSeg;
        kw = min(kSeg, nx - X0);
        P0 = tyi * kSeg;
        kp = min(kSeg, np - P0);
        lx = periodic ? kLineQ : min(nx, kLineQ);
        xs = periodic ? X0 - kHalo : max(0, min(X0 - kHalo, nx - lx));
        lp = min(np, kLineQ);
        ps = max(0, min(P0 - kHalo, np - lp));
        ox = X0 - xs;
        op = P0 - ps;
    }
};

// ---------------------------------------------------------------------------
// k_solve_spline<BW>: w_new = (M_x^{-1} (x) M_p^{-1}) b for spline basis
// functions (BW 2: quadratic, 80 x 80 tiles; 3: cubic, 60 x 60), on lattices
// whose open axes have at least kLineQ nodes (k_solve_spline_narrow takes the
// others).  A workgroup of kLineQ threads owns a tile inside the
// kLineQ x kLineQ window around it (SplineTile).
//  p phase: thread c loads window column c into registers through a buffer
//    resource based at the window's first row (the row's byte offset advances
//    by a register add; every row in flight at once; a wavefront's lanes read
//    64 consecutive nodes of a row per instruction), solves it, and puts the
//    kept rows into LDS (rows outside them go to two trash rows, so the
//    writes need no branches).  (Half the rows staged by direct loads into
//    LDS instead measured 2.7 us slower at 2048^2, quadratic: the column has
//    to reach the registers anyway.)
//  x phase: thread r solves kept row r in registers.
//  out:     the kept columns of the kept rows go out, whole rows per store.
// The LDS holds the kept rows and two trash rows at an odd pitch (42 KB for
// the quadratic: three tiles per compute unit, the 676 tiles of a 2048^2
// lattice in one round), and both passes address it without bank conflicts.
// For the FEL the write-out also forms the tile's bunching partials.
// ---------------------------------------------------------------------------
template <int BW>
__global__ __launch_bounds__(kSolveQThreads) void k_solve_spline(LaunchArgs A) {
    constexpr int kSeg = spline_seg(BW);
    __shared__ float win[(kSeg + 2) * kPitchQ];  // row 1 + r: kept row r; rows 0 and kSeg + 1: trash
    __shared__ double s_red[kSolveQThreads / 64][kPartialsPerTile];
    __shared__ int s_d;
    const int tid = threadIdx.x;
    const int item = tile_of(blockIdx.x, A.total);  // one tile per workgroup (the grid is the tile count)
    if (tid == 0) s_d = find_instance(A.off, A.ninst, item);
    __syncthreads();
    const int d = __builtin_amdgcn_readfirstlane(s_d);
    const VpInst& I = A.inst[d];
    const int t = item - A.off[d];
    const SplineTile<BW> T(I, t);
    const int nx = T.nx;
    float* __restrict__ dst = I.w[((I.parity0 + A.parity) & 1) ^ 1];

    {
        // p phase, thread = window column (lx = lp = kLineQ here)
        const int col = T.periodic ? wrap_index(T.xs + tid, nx, 1.0f / (float)nx) : T.xs + tid;
        float v[kLineQ];
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)(I.b + (size_t)T.ps * nx), (short)0, -1, kBufferWord3);
        // byte offset of the lane's node in row k: col 4 + k nx 4 < 2^25 (both
        // axes have at most 2^16 nodes), advanced row by row
        const int row_bytes = nx * 4;
        int off = col * 4;
#pragma unroll
        for (int k = 0; k < kLineQ; ++k, off += row_bytes)
            v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
        band_line<BW>(v, T.ps == 0);
        // window row k -> LDS row 1 + (k - op).  Interior tiles (op = the
        // halo) and tiles at the first edge (op = 0) write their kept rows at
        // constant offsets; the others clamp the rows outside to the trash rows
        const int op = __builtin_amdgcn_readfirstlane(T.op);
        float* colp = win + kPitchQ + tid;
        if (op == T.kHalo) {
#pragma unroll
            for (int k = 0; k < kSeg; ++k) colp[k * kPitchQ] = v[T.kHalo + k];
        } else if (op == 0) {
#pragma unroll
            for (int k = 0; k < kSeg; ++k) colp[k * kPitchQ] = v[k];
        } else {
#pragma unroll
            for (int k = 0; k < kLineQ; ++k) colp[min(max(k - op, -1), kSeg) * kPitchQ] = v[k];
        }
    }
    __syncthreads();
    if (tid < T.kp) {
        // x phase, thread = kept row
        float* row = win + (tid + 1) * kPitchQ;
        float v[kLineQ];
#pragma unroll
        for (int k = 0; k < kLineQ; ++k) v[k] = row[k];
        band_line<BW>(v, !T.periodic && T.xs == 0);
#pragma unroll
        for (int k = 0; k < kLineQ; ++k) row[k] = v[k];
    }
    __syncthreads();
    spline_tile_out(I, t, win + kPitchQ, T.ox, T.X0, T.kw, T.P0, T.kp, nx, dst, s_red);
}

// ---------------------------------------------------------------------------
// k_solve_spline_narrow<BW>: the same solve for launches with an open axis
// shorter than kLineQ nodes.  The whole window (up to kLineQ x kLineQ) is
// staged in LDS by direct loads and every line is solved there by
// band_line_lds: slower, and only small lattices take it.
// ---------------------------------------------------------------------------
template <int BW>
__global__ __launch_bounds__(kSolveQThreads) void k_solve_spline_narrow(LaunchArgs A) {
    __shared__ float win[kLineQ * kPitchQ];
    __shared__ double s_red[kSolveQThreads / 64][kPartialsPerTile];
    __shared__ int s_d;
    const int tid = threadIdx.x;
    const int item = tile_of(blockIdx.x, A.total);
    if (tid == 0) s_d = find_instance(A.off, A.ninst, item);
    __syncthreads();
    const int d = __builtin_amdgcn_readfirstlane(s_d);
    const VpInst& I = A.inst[d];
    const int t = item - A.off[d];
    const SplineTile<BW> T(I, t);
    const int nx = T.nx;
    float* __restrict__ dst = I.w[((I.parity0 + A.parity) & 1) ^ 1];
    if (tid < T.lx) {
        const int col = T.periodic ? wrap_index(T.xs + tid, nx, 1.0f / (float)nx) : T.xs + tid;
        gfloat* src = as_global(I.b) + (size_t)T.ps * nx + col;
        float* row0 = win + __builtin_amdgcn_readfirstlane(tid & ~63);
        for (int r = 0; r < T.lp; ++r)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + (size_t)r * nx),
                                             (__attribute__((address_space(3))) void*)(row0 + r * kPitchQ), 4, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (tid < T.lx) band_line_lds<kPitchQ, BW>(win + tid, T.lp, T.ps == 0);
    __syncthreads();
    if (tid < T.kp) band_line_lds<1, BW>(win + (T.op + tid) * kPitchQ, T.lx, !T.periodic && T.xs == 0);
    __syncthreads();
    spline_tile_out(I, t, win + T.op * kPitchQ, T.ox, T.X0, T.kw, T.P0, T.kp, nx, dst, s_red);
}

// ---------------------------------------------------------------------------
// k_fel_field: one workgroup per instance of the launch list; for an FEL
// instance it sums the per-tile bunching partials of the preceding kernel in
// the fixed order of sum_tile_partials and advances the field (eq. 13c).  A kernel of its own, because a last-tile-sums scheme
// inside k_solve needs a device-scope release per tile, which on a multi-XCD
// part writes back the L2 and costs more than the solve.
//  mode 0 (after k_solve; partials: the new state's bunching at the half-drift
//    and at the lattice phases).  Exact-kick step: A moves by dz times the
//    bunching of the state that was pushed; Runge-Kutta: A takes the step's
//    new value.  The new bunchings are kept for the next step.
//  mode 1 (after k_fel_stage, Runge-Kutta only; partials: the bunching at the
//    phases of stages 3 and 4): keeps b3, b4 and forms the step's new field
//    A + dz/6 (b1 + 2 b2 + 2 b3 + b4).  A launch of one instance with few
//    enough solve tiles skips it: its deposit sums the same partials itself.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFieldThreads) void k_fel_field(LaunchArgs A) {
    __shared__ double s_red[kPartialsPerTile][kFieldThreads / 64];
    const VpInst& I = A.inst[blockIdx.x];
    if (I.push.kind != kFel || (A.mode == 1 && !I.push.rk4)) return;
    // the field state the update needs, loaded while the partials are summed
    double* st = I.fel_state;
    double n0 = 0.0, a[2] = {0.0, 0.0}, bn[2] = {0.0, 0.0}, b1[2] = {0.0, 0.0}, an[2] = {0.0, 0.0};
    if (threadIdx.x == 0) {
        n0 = st[kN0];
        for (int c = 0; c < 2; ++c) {
            a[c] = st[kA + c];
            bn[c] = st[kBn + c];
            b1[c] = st[kB1 + c];
            an[c] = st[kAn + c];
        }
    }
    double acc[kPartialsPerTile];
    sum_tile_partials(I, s_red, acc);
    if (threadIdx.x == 0) {
        const double inv_n0 = 1.0 / n0, h = I.fel_dz;
        if (A.mode == 1) {
            double b3[2], b4[2], a_new[2];
            rk4_stage_fields(a, b1, bn, n0, h, acc, b3, b4, a_new);
            for (int c = 0; c < 2; ++c) {
                st[kB3 + c] = b3[c];
                st[kB4 + c] = b4[c];
                st[kAn + c] = a_new[c];
            }
            return;
        }
        if (I.push.rk4) {
            st[kA] = an[0];
            st[kA + 1] = an[1];
            st[kB1] = acc[2] * inv_n0;
            st[kB1 + 1] = acc[3] * inv_n0;
        } else {
            st[kA] = a[0] + h * bn[0];
            st[kA + 1] = a[1] + h * bn[1];
        }
        st[kBn] = acc[0] * inv_n0;
        st[kBn + 1] = acc[1] * inv_n0;
        st[kDzB] = h;
    }
}

// sin and cos of x: for |x| < 2^-6 by their Taylor series to the x^9 and x^10
// terms (the first omitted terms are below 2^-70 relative), else sincos.  The
// Runge-Kutta stage angles dz^2/2 k are that small unless dz or the field is large.
__device__ inline void sincos_small(double x, double* s, double* c) {
    if (fabs(x) < 0.015625) {
        const double x2 = x * x;
        *s = x * (1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 + x2 * (1.0 / 362880.0)))));
        *c = 1.0 + x2 * (-0.5 + x2 * (1.0 / 24.0 + x2 * (-1.0 / 720.0 + x2 * (1.0 / 40320.0 + x2 * (-1.0 / 3628800.0)))));
    } else {
        sincos(x, s, c);
    }
}

// ---------------------------------------------------------------------------
// k_fel_stage: the bunching at the phases of the Runge-Kutta step's stages 3
// and 4 (FEL only), FP64, one per-tile partial per solve tile of the
// instance's solve.  A workgroup of four wavefronts per tile: thread t takes
// a column and every kRowStep-th row of it; the sums are reduced in a fixed
// order (shuffle tree per wavefront, then the wavefronts in turn).  With
// k1 = a1 cos phi + b1 sin phi and k2 = a2 cos psi2 + b2 sin psi2 the slopes
// of stages 1 and 2 (fields A1 = A, A2 = A + dz/2 b1), the phases are
// psi3 = phi + q + dz^2/4 k1 and psi4 = phi + 2 q + dz^2/2 k2, q the half
// drift of the node's row.  k1 depends on the column only, so stage 3's sum
// is a column sum of w e^{-i q} turned by e^{-i(phi + dz^2/4 k1)}.
// ---------------------------------------------------------------------------
// One solve tile of SX x SP nodes (the tiles of the instance's solve: tents
// 32 x 64, quadratic basis 80 x 80, cubic 60 x 60); thread t takes column t mod SX and rows
// t / SX + (256 / SX) i (threads past the last whole row group idle).
template <int SX, int SP>
__device__ inline void stage_tile(const VpInst& I, int t, int parity, double (&s_red)[kStageThreads / 64][4]) {
    constexpr int kWaves = kStageThreads / 64, kRowStep = kStageThreads / SX;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nx = I.push.nx, np = I.push.np;
    const int tiles_x = (nx + SX - 1) / SX;
    const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
    const int X0 = txi * SX, tw = min(SX, nx - X0);
    const int Y0 = tyi * SP, th = min(SP, np - Y0);
    const int par = (I.parity0 + parity) & 1;
    const float* __restrict__ w = I.w[par];
    const double* st = I.fel_state;
    const double h = I.fel_dz, sg = (double)I.fel_sigma2;
    // slope coefficients of stages 1 and 2 (as in the deposit, FP64)
    const double b1r = st[kB1], b1i = st[kB1 + 1], b2r = st[kBn], b2i = st[kBn + 1];
    const double a1r = st[kA] - sg * b1i, a1i = st[kA + 1] + sg * b1r;
    const double a2r = st[kA] + 0.5 * h * b1r - sg * b2i, a2i = st[kA + 1] + 0.5 * h * b1i + sg * b2r;
    const double t3 = 0.25 * h * h, t4 = 0.5 * h * h;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // stage 3 (re, im), stage 4 (re, im)
    const int col = tid % SX, r0 = tid / SX;
    if (col < tw && r0 < kRowStep) {
        const int gx = X0 + col;
        const double2 ex = I.fel_ex[gx];
        double cre = 0.0, cim = 0.0;
        // Rows in batches of kStageBatch whose loads are all issued before the
        // first is used (one memory round trip per batch, not per row).  Rows
        // past the tile load its last row and weigh zero: the sums are never
        // -0, so adding +-0 leaves them as the rows of the tile alone make them.
        constexpr int kStageBatch = 8;
        for (int r1 = r0; r1 < th; r1 += kStageBatch * kRowStep) {
            float wr[kStageBatch];
            double2 eqr[kStageBatch];
#pragma unroll
            for (int q = 0; q < kStageBatch; ++q) {
                const int j = Y0 + min(r1 + q * kRowStep, th - 1);
                wr[q] = w[(size_t)j * nx + gx];
                eqr[q] = I.fel_eq[j];
            }
#pragma unroll
            for (int q = 0; q < kStageBatch; ++q) {
                const double wk = r1 + q * kRowStep < th ? (double)wr[q] : 0.0;
                const double2 eq = eqr[q];
                cre += wk * eq.x;
                cim -= wk * eq.y;
                // e^{i psi2} = e^{i phi} e^{i q}
                const double c2 = ex.x * eq.x - ex.y * eq.y, s2 = ex.y * eq.x + ex.x * eq.y;
                const double k2 = -2.0 * (a2r * c2 - a2i * s2);
                double sn, cs;
                sincos_small(t4 * k2, &sn, &cs);
                // e^{i psi4} = e^{i psi2} e^{i q} e^{i t4 k2}
                const double c2q = c2 * eq.x - s2 * eq.y, s2q = s2 * eq.x + c2 * eq.y;
                const double c4 = c2q * cs - s2q * sn, s4 = s2q * cs + c2q * sn;
                acc[2] += wk * c4;
                acc[3] -= wk * s4;
            }
        }
        const double k1 = -2.0 * (a1r * ex.x - a1i * ex.y);
        double sn, cs;
        sincos_small(t3 * k1, &sn, &cs);
        const double c3 = ex.x * cs - ex.y * sn, s3 = ex.y * cs + ex.x * sn;  // e^{i(phi + t3 k1)}
        acc[0] = cre * c3 + cim * s3;
        acc[1] = cim * c3 - cre * s3;
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < 4; ++c) acc[c] += __shfl_down(acc[c], o);
    if (lane == 0)
        for (int c = 0; c < 4; ++c) s_red[wid][c] = acc[c];
    __syncthreads();
    if (tid < 4) {
        double v = 0.0;
        for (int k = 0; k < kWaves; ++k) v += s_red[k][tid];
        I.partials[kPartialsPerTile * t + tid] = v;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kStageThreads) void k_fel_stage(LaunchArgs A) {
    __shared__ double s_red[kStageThreads / 64][4];
    for (int item = blockIdx.x; item < A.total; item += gridDim.x) {
        const int d = __builtin_amdgcn_readfirstlane(find_instance(A.off, A.ninst, item));
        const VpInst& I = A.inst[d];
        if (I.push.kind != kFel || !I.push.rk4) continue;
        if (I.push.wide == kBasisQuadratic) stage_tile<kSegQ, kSegQ>(I, item - A.off[d], A.parity, s_red);
        else if (I.push.wide == kBasisCubic) stage_tile<kSegC, kSegC>(I, item - A.off[d], A.parity, s_red);
        else stage_tile<kSegX, kSegP>(I, item - A.off[d], A.parity, s_red);
    }
}

// ---------------------------------------------------------------------------
// k_reduce: FP64 sums over one state, fixed-order (deterministic) reduction.
//  mode 0 (diagnostics): sum w, sum_{w<0} w, sum |w|, sum_{w>0} w ln w,
//    sum w p, sum w (kinetic + potential), sum w cos x, sum w sin x, max |w|,
//    #nonfinite.
//  mode 1 (FEL bunching): sum w e^{-i (phi_i + q_j)} / N0 and
//    sum w e^{-i phi_i} / N0 -> fel_state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_reduce(ReduceArgs R) {
    __shared__ double s_part[kReduceThreads / 64][kMoments];
    __shared__ int s_last;
    double acc[kMoments];
#pragma unroll
    for (int k = 0; k < kMoments; ++k) acc[k] = 0.0;
    const long n = (long)R.nx * R.np;
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const int j = (int)(k / R.nx), i = (int)(k - (long)j * R.nx);
        const double w = (double)R.w[k];
        if (R.mode == 1) {
            const double2 ex = R.fel_ex[i], eq = R.fel_eq[j];
            // e^{-i(phi+q)} = (cos phi cos q - sin phi sin q) - i (sin phi cos q + cos phi sin q)
            acc[0] += w * (ex.x * eq.x - ex.y * eq.y);
            acc[1] -= w * (ex.y * eq.x + ex.x * eq.y);
            // and at the lattice phases, e^{-i phi} (the Runge-Kutta step's stage 1)
            acc[2] += w * ex.x;
            acc[3] -= w * ex.y;
            continue;
        }
        if (!isfinite(w)) { acc[9] += 1.0; continue; }
        if (R.mode == 2) {  // sum, largest magnitude and non-finite count only
            acc[0] += w;
            acc[8] = fmax(acc[8], fabs(w));
            continue;
        }
        const double x = R.x_lo + (double)i * R.hx, p = R.p_lo + (double)j * R.hp;
        acc[0] += w;
        acc[8] = fmax(acc[8], fabs(w));
        if (w < 0.0) acc[1] += w;
        acc[2] += fabs(w);
        if (w > 0.0) acc[3] += w * log(w);
        acc[4] += w * p;
        double e = 0.5 * (p * p + R.hp * R.hp * R.var_c);
        if (R.kind == kPendulum) e -= R.a * R.cos_fac * cos(x);
        else if (R.kind == kSho) e += 0.5 * (x * x + R.hx * R.hx * R.var_c);
        acc[5] += w * e;
        if (R.kind == kFel) {
            acc[6] += w * cos(x);
            acc[7] -= w * sin(x);
        }
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
        if (R.mode == 1) {
            if (threadIdx.x < 2) R.out[kBn + threadIdx.x] = s * R.inv_n0;
            else if (threadIdx.x < 4) R.out[kB1 + threadIdx.x - 2] = s * R.inv_n0;
            if (threadIdx.x == 0) R.out[kDzB] = R.dz;
        } else {
            R.out[threadIdx.x] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicExch(R.counter, 0u);
    }
}

// ---------------------------------------------------------------------------
// Allocation-free stepping: the scratch array and the kernels that set it up
// for one call of vp_step_noalloc and report back.  Each call writes every
// byte it reads later (tables, descriptor, offsets, FEL state, counters; b is
// written by the deposit before the solve reads it), so nothing of an earlier
// call leaks into a later one; calls that overlap on one device race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

void* noalloc_scratch(hipError_t* err) {
    constexpr int kMaxDevices = 64;
    static void* ptr[kMaxDevices] = {};
    static std::mutex mu;
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        // the array's name is a host-side stand-in: kernels get this address
        void* p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

__global__ void k_noalloc_setup(NoAllocSetup S) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = S.inst.push.nx, np = S.inst.push.np;
    if (k < nx) table_x(S.tables, k, S.tab_x[k], S.fel_ex[k]);
    if (k < np) table_p(S.tables, k, S.tab_p[k], S.fel_eq[k]);
    if (k == 0) {
        *S.inst_out = S.inst;
        S.off_out[0] = 0;
        S.off_out[1] = S.inst.k1_tiles;
        S.off_out[2] = 0;
        S.off_out[3] = S.inst.k2_tiles;
        for (int q = 0; q < kFelStateLen; ++q) S.fel_state[q] = 0.0;
        if (S.fel_A) {
            S.fel_state[kA] = S.fel_A[0];
            S.fel_state[kA + 1] = S.fel_A[1];
        }
        S.fel_state[kN0] = S.n0;
        for (int q = 0; q < 4; ++q) S.counters[q] = 0u;
    }
}

__global__ void k_noalloc_scale(VpInst* inst, const double* m) {
    // 2^(40 - e) with max|w| < 2^e, as vp_set_density sets it
    const double wmax = m[8];
    int e = 0;
    if (wmax > 0.0 && isfinite(wmax)) {
        (void)frexp(wmax, &e);
        e = max(e, kFixBits - 126);
    }
    const bool bad = m[9] > 0.0;
    inst->fix_scale = bad ? 0.0f : ldexpf(1.0f, kFixBits - e);
    inst->fix_inv = ldexpf(1.0f, e - kFixBits);
}

__global__ void k_noalloc_finish(const double* m, const double* fel_state, const uint32_t* counters, double* fel_A,
                                 int32_t* status) {
    if (fel_A) {
        fel_A[0] = fel_state[kA];
        fel_A[1] = fel_state[kA + 1];
    }
    if (status) *status = m[9] > 0.0 ? -6 : (counters[kRangeFlag] ? -7 : 0);  // VP_ENONFINITE, VP_ERANGE, VP_OK
}

hipError_t launch_noalloc_setup(const NoAllocSetup& S, int nx, int np, hipStream_t s) {
    const int n = max(nx, np), threads = 256;
    hipLaunchKernelGGL(k_noalloc_setup, dim3((n + threads - 1) / threads), dim3(threads), 0, s, S);
    return hipGetLastError();
}
hipError_t launch_noalloc_scale(VpInst* inst, const double* moments, hipStream_t s) {
    hipLaunchKernelGGL(k_noalloc_scale, dim3(1), dim3(1), 0, s, inst, moments);
    return hipGetLastError();
}
hipError_t launch_noalloc_finish(const double* moments, const double* fel_state, const uint32_t* counters,
                                 double* fel_A, int32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_noalloc_finish, dim3(1), dim3(1), 0, s, moments, fel_state, counters, fel_A, status);
    return hipGetLastError();
}

// One launch of a per-step kernel.  With events (timing), hipExtLaunchKernel
// records them with the kernel's own dispatch, so their interval is the
// kernel's execution, without the gaps a separate event record adds.
static hipError_t launch_k(const void* fn, int grid, int threads, size_t lds, hipStream_t s, const LaunchArgs& a,
                           hipEvent_t e0, hipEvent_t e1) {
    void* args[1] = {const_cast<LaunchArgs*>(&a)};
    if (e0 || e1) return hipExtLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, s, e0, e1, 0);
    return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, s);
}

hipError_t launch_deposit(const LaunchArgs& a, int grid, size_t lds, int threads, hipStream_t s, int basis,
                          hipEvent_t e0, hipEvent_t e1) {
    return launch_k(deposit_kernel(basis), grid, threads, lds, s, a, e0, e1);
}

hipError_t launch_solve(const LaunchArgs& a, int grid, hipStream_t s, int kind, hipEvent_t e0, hipEvent_t e1) {
    return launch_k(solve_kernel(kind), grid, solve_threads(kind), 0, s, a, e0, e1);
}

hipError_t launch_fel_field(const LaunchArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return launch_k(fel_field_kernel(), a.ninst, kFieldThreads, 0, s, a, e0, e1);
}

hipError_t launch_fel_stage(const LaunchArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return launch_k(fel_stage_kernel(), grid, kStageThreads, 0, s, a, e0, e1);
}

hipError_t launch_map(const VpInst* inst, long nodes, hipStream_t s) {
    hipLaunchKernelGGL(k_map, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s, inst);
    return hipGetLastError();
}


hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

const void* deposit_kernel(int basis) {
    if (basis == kBasisQuadratic) return reinterpret_cast<const void*>(&k_deposit<6>);
    if (basis == kBasisCubic) return reinterpret_cast<const void*>(&k_deposit<8>);
    return reinterpret_cast<const void*>(&k_deposit<4>);
}
const void* solve_kernel(int kind) {
    if (kind == kSolveQuad) return reinterpret_cast<const void*>(&k_solve_spline<2>);
    if (kind == kSolveQuadNarrow) return reinterpret_cast<const void*>(&k_solve_spline_narrow<2>);
    if (kind == kSolveCubic) return reinterpret_cast<const void*>(&k_solve_spline<3>);
    if (kind == kSolveCubicNarrow) return reinterpret_cast<const void*>(&k_solve_spline_narrow<3>);
    return reinterpret_cast<const void*>(&k_solve);
}
const void* fel_field_kernel() { return reinterpret_cast<const void*>(&k_fel_field); }
const void* fel_stage_kernel() { return reinterpret_cast<const void*>(&k_fel_stage); }

}  // namespace vp
