// vp_kernels.hip -- gfx950 kernels of one phase-space-conservation Vlasov step.
//
// Edelen & Webb, Sec. "An Algorithm Based on Phase Space Density Conservation":
// w_fin = Lambda^{-1} Delta^T w_in (eq. 10).  With tents of width h the overlap
// of a tent moved to u (in cells) with the tent of node c is h B3(u - c), B3 the
// centred cubic B-spline (eq. 9), and Lambda = h_x h_p M_x (x) M_p with
// M = tridiag(1/6, 2/3, 1/6) (eq. 8).  k_deposit forms b = Delta^T w / (h_x h_p),
// k_solve forms (M_x^{-1} (x) M_p^{-1}) b.  All state arithmetic is FP32; FP64
// is used only for the FEL bunching sum and the diagnostics.
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

// Integer part and fraction in [0,1) of hi + lo, |lo| small.
__device__ inline void split_cell(float hi, float lo, int& k, float& t) {
    float f = floorf(hi);
    float r = (hi - f) + lo;
    if (r >= 1.0f) {
        r -= 1.0f;
        f += 1.0f;
    } else if (r < 0.0f) {
        r += 1.0f;
        f -= 1.0f;
    }
    k = (int)f;
    t = r;
}

// Round v in [0, 1] to a multiple of 2^-23 ((v + 1) - 1, both steps exact or
// correctly rounded, never contracted).
__device__ inline float grid23(float v) { return __fsub_rn(__fadd_rn(v, 1.0f), 1.0f); }

// Cubic B-spline tap weights B3(t+1), B3(t), B3(1-t), B3(2-t) for t in [0,1).
// They sum to exactly one in FP32 (the partition of unity behind the
// conservation argument of eqs. 11-12): three taps are rounded to multiples
// of 2^-23, so their sum and 1 minus it are exact and give the fourth.
// (Without that rounding, 1 - sum itself rounds, biased: at t = 0 the taps
// sum to 1 - 3e-8 and the state would lose that much mass per axis per step.)
__device__ inline void bspline_taps(float t, float (&b)[4]) {
    const float sixth = 1.0f / 6.0f;
    float s = 1.0f - t;
    float t2 = t * t;
    b[0] = grid23((s * sixth) * (s * s));
    const float t3 = (t * sixth) * t2;
    b[3] = grid23(t3);
    b[2] = grid23(fmaf(0.5f, t + t2, sixth) - 3.0f * t3);
    b[1] = 1.0f - ((b[0] + b[3]) + b[2]);
}

// Round a value of magnitude below 2^51 to the nearest 64-bit integer (two's
// complement bits) exactly: adding 1.5 * 2^52 leaves round-to-nearest(v) in
// the low 52 bits of the sum's encoding, two's complement relative to the
// constant's encoding.
__device__ inline unsigned long long fix64(double v) {
    const double d = v + 6755399441055744.0;  // 1.5 * 2^52
    return (unsigned long long)(__double_as_longlong(d) - 0x4338000000000000ll);
}

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

// LU coefficients at node g from the open edge: tabulated below kEdge, the
// interior constant beyond.  Branch-free: the (clamped) table read is
// unconditional and a select picks the value.
template <bool EDGE>
__device__ inline float lu_m(int g, const float2* edge) {
    if (!EDGE) return kMinf;
    const float t = edge[min(g, kEdge - 1)].x;
    return g < kEdge ? t : kMinf;
}
template <bool EDGE>
__device__ inline float lu_dinv(int g, const float2* edge) {
    if (!EDGE) return kMinf;
    const float t = edge[min(g, kEdge - 1)].y;
    return g < kEdge ? t : kMinf;
}

// Solve M y = b, M = tridiag(1/6, 2/3, 1/6), along one line of n <= kLine
// values v[0..n) (registers; entries past n are zero), written as
//     y = b - T^{-1} (D2 b),   T = 6 M = tridiag(1, 4, 1),  D2 b = b[k-1] - 2 b[k] + b[k+1]
// (T = 6 I + D2, so 6 T^{-1} = I - T^{-1} D2).  The LU recursions of T then only
// carry the correction T^{-1} D2 b, so their FP32 rounding (whose fixed point
// is biased on slowly varying data) acts on a term much smaller than b: the
// mass a line carries is kept to ~1e-10 per step instead of ~1e-8.
// Neighbours outside [0, n) count as zero: exact at an open edge (the
// truncated M), and a cut inside the lattice only disturbs the halo.
// first = index of v[0] from the open edge when below kEdge (EDGE: the exact
// tabulated LU coefficients apply there), interior constants elsewhere.
// The solution replaces v.  Fixed length, fully unrolled, no branches.
template <bool EDGE>
__device__ inline void line_solve(float (&v)[kLine], int n, int first, const float2* edge) {
    float z[kLine];
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < kLine; ++k) {
        const float r = ((k > 0 ? v[k - 1] : 0.0f) + (k + 1 < kLine ? v[k + 1] : 0.0f)) - 2.0f * v[k];
        acc = fmaf(-lu_m<EDGE>(first + k, edge), acc, r);
        acc = k < n ? acc : 0.0f;
        z[k] = acc;
    }
    float c = 0.0f;
#pragma unroll
    for (int k = kLine - 1; k >= 0; --k) {
        c = (z[k] - c) * lu_dinv<EDGE>(first + k, edge);
        v[k] -= c;
    }
}

__device__ inline void line_solve_any(float (&v)[kLine], int n, int first, const float2* edge) {
    if (first >= kEdge) line_solve<false>(v, n, first, edge);
    else line_solve<true>(v, n, first, edge);
}

}  // namespace

// Push one node (source row j, unwrapped column ii, weight w already scaled to
// fixed point) and add its 16 B-spline taps into the LDS tile.
__device__ inline void deposit_node(long long* acc, int j, int ii, float w, float4 tx, float4 tp, int kind,
                                    float alpha, float beta, float kd, int X0, int Y0, int ldw, int cmax,
                                    int rmax) {
    if (w == 0.0f) return;
    int ku, kv;
    float fu, fv;
    if (kind == kSho) {
        float su, eu, sv, ev;
        two_sum(tx.x, tp.x, su, eu);
        two_sum(tx.z, tp.z, sv, ev);
        split_cell(su, eu + (tx.y + tp.y), ku, fu);
        split_cell(sv, ev + (tx.w + tp.w), kv, fv);
    } else {
        // phase phi_i + q_j from the per-axis sine/cosine tables
        const float cph = tx.y * tp.w - tx.x * tp.z;
        const float sph = tx.x * tp.w + tx.y * tp.z;
        const float dv = alpha * cph + beta * sph;
        float su, eu;
        two_sum(tp.x, dv * kd, su, eu);
        split_cell(su, eu + tp.y, ku, fu);
        split_cell(dv, 0.0f, kv, fv);
    }
    float bx[4], bp[4];
    bspline_taps(fu, bx);
    bspline_taps(fv, bp);
    // tap (q, r) lands on row j + kv - 1 + q, column ii + ku - 1 + r
    const int c0 = clampi(ii + ku - 1 - X0 + kPad, 0, cmax);
    const int r0 = clampi(j + kv - 1 - Y0 + kPad, 0, rmax);
    long long* base = acc + r0 * ldw + c0;
    // tap value w * bp * bx formed in FP64 and rounded once, exactly, into
    // the fixed-point tile sum: the deposit adds no FP32 product rounding to
    // the state (the FEL instability amplifies it)
    double bxd[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) bxd[rr] = (double)bx[rr];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double wq = (double)w * (double)bp[q];
        long long* row = base + q * ldw;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) atomicAdd((unsigned long long*)(row + rr), fix64(wq * bxd[rr]));
    }
}

// ---------------------------------------------------------------------------
// k_deposit: push every node of the tile's source box and scatter its weight
// into the LDS image of the destination tile, then write the tile of b once.
// (Integer LDS atomics: gfx950 executes ds_add_f32 some 40x slower than
// ds_add_u32, and integer sums are order independent.)
// LDS holds (tx + 8) x (ty + 8) cells: the tile plus a 4-cell trash border.
// Every tap index is clamped into that border, so no access can leave LDS
// whatever the push does; taps that land outside the tile are dropped there.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kDepositThreads) void k_deposit(LaunchArgs A) {
    extern __shared__ long long acc[];
    __shared__ int s_d, s_box[4];
    __shared__ float s_ab[2];

    for (int item = blockIdx.x; item < A.total; item += gridDim.x) {
        if (threadIdx.x == 0) s_d = find_instance(A.off, A.ninst, item);
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_d);
        const VpInst& I = A.inst[d];
        const int t = item - A.off[d];
        const int tyi = t / I.k1_tiles_x, txi = t - tyi * I.k1_tiles_x;
        const int nx = I.push.nx, np = I.push.np;
        const int X0 = txi * I.k1_tx, X1 = min(X0 + I.k1_tx, nx);
        const int Y0 = tyi * I.k1_ty, Y1 = min(Y0 + I.k1_ty, np);
        const int ldw = I.k1_tx + 2 * kPad, ldh = I.k1_ty + 2 * kPad;
        const int cmax = I.k1_tx + kPad, rmax = I.k1_ty + kPad;
        const int par = (I.parity0 + A.parity) & 1;
        const float* __restrict__ w_in = I.w[par];

        for (int k = threadIdx.x; k < ldw * ldh; k += blockDim.x) acc[k] = 0ll;
        if (threadIdx.x == 0) {
            PushParams P = I.push;
            if (P.kind == kFel) {
                // kick field: A at mid-kick plus the space-charge term, A + b dz/2 + i sigma2 b
                const double* st = I.fel_state;
                double are = st[kA] + 0.5 * I.fel_dz * st[kBn] - (double)I.fel_sigma2 * st[kBn + 1];
                double aim = st[kA + 1] + 0.5 * I.fel_dz * st[kBn + 1] + (double)I.fel_sigma2 * st[kBn];
                P.alpha = (float)(I.fel_kick * are);
                P.beta = (float)(-I.fel_kick * aim);
            }
            s_ab[0] = P.alpha;
            s_ab[1] = P.beta;
            source_box(P, X0, X1, Y0, Y1, s_box);
        }
        __syncthreads();

        const int bx0 = s_box[0], bw = s_box[1] - s_box[0];
        const int by0 = s_box[2], bh = s_box[3] - s_box[2];
        const int nsrc = (bw > 0 && bh > 0) ? bw * bh : 0;
        const float inv_bw = 1.0f / (float)max(bw, 1);
        const float inv_nx = 1.0f / (float)nx;
        const float alpha = s_ab[0], beta = s_ab[1], kd = I.push.kd;
        const int kind = I.push.kind;
        const bool periodic = I.push.x_periodic != 0;

        // Tile sums are exact fixed-point integers: every tap value is rounded
        // to a multiple of 2^-40 of the instance's initial max|w| and summed
        // with 64-bit integer LDS atomics, so the sum does not depend on the
        // order of the atomics (bitwise reproducible).  The map is area
        // preserving, so a cell collects about max|w|; a tap must stay below
        // 2^11 max|w| (the conversion's range) and a sum below 2^23 max|w|.
        const float scale = I.fix_scale, inv_scale = I.fix_inv;  // exact powers of two
        const int nsrc_live = scale > 0.0f ? nsrc : 0;

        // Four sources per thread and iteration, every load issued before any
        // use, so an iteration waits for one memory latency, not a chain.
        constexpr int kU = 4;
        for (int s0 = threadIdx.x; s0 < nsrc_live; s0 += kU * blockDim.x) {
            int jj[kU], iiu[kU];
            float wv[kU];
            float4 txv[kU], tpv[kU];
#pragma unroll
            for (int h = 0; h < kU; ++h) {
                const int s = min(s0 + h * (int)blockDim.x, nsrc_live - 1);
                int r = (int)(((float)s + 0.5f) * inv_bw);
                int c = s - r * bw;
                if (c < 0) { c += bw; --r; }
                if (c >= bw) { c -= bw; ++r; }
                jj[h] = by0 + r;
                iiu[h] = bx0 + c;  // unwrapped source column
                const int i = periodic ? wrap_index(iiu[h], nx, inv_nx) : iiu[h];
                wv[h] = w_in[(size_t)jj[h] * nx + i];
                txv[h] = I.tab_x[i];
                tpv[h] = I.tab_p[jj[h]];
            }
#pragma unroll
            for (int h = 0; h < kU; ++h) {
                if (s0 + h * (int)blockDim.x >= nsrc_live) break;
                deposit_node(acc, jj[h], iiu[h], wv[h] * scale, txv[h], tpv[h], kind, alpha, beta, kd, X0, Y0,
                             ldw, cmax, rmax);
            }
        }
        __syncthreads();

        const int tw = X1 - X0, th = Y1 - Y0;
        float* __restrict__ b = I.b;
        for (int k = threadIdx.x; k < tw * th; k += blockDim.x) {
            int rr = k / tw, cc = k - rr * tw;
            b[(size_t)(Y0 + rr) * nx + X0 + cc] = (float)acc[(rr + kPad) * ldw + cc + kPad] * inv_scale;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// The mass-matrix solve (M_x^{-1} (x) M_p^{-1}) b in two kernels, one lattice
// line segment per lane (line_solve): LU recursions of T = tridiag(1,4,1),
//   forward  z_k = r_k - m_k z_{k-1},   backward c_k = (z_k - c_{k+1}) / d_k,
// with exact per-node (m_k, 1/d_k) near an open edge (so the true edges are
// exact) and the interior constants elsewhere.  A segment carries a 16-node
// halo on each side; where the halo is cut inside the lattice the recursion
// starts from zero, an error that decays by 2 - sqrt 3 per node and is ~7e-10
// at the segment.
//  k_solve_x: b -> the old state buffer (free once the deposit has read it).
//    A wavefront owns 64 rows x kSeg columns; the rows plus halos are staged
//    in LDS (coalesced) and each lane solves one row from registers.
//  k_solve_p: that buffer -> the new state.  A lane owns kSeg rows of one
//    column and streams the column plus halos straight from global memory
//    into registers (coalesced across lanes); no LDS.  For the FEL its
//    epilogue also forms the FP64 bunching of the new state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSolveXThreads) void k_solve_x(LaunchArgs A) {
    __shared__ float lds[kSolveXThreads * (kLine + 1)];
    __shared__ int s_d;
    __shared__ float2 s_edge[kEdge];

    for (int item = blockIdx.x; item < A.total; item += gridDim.x) {
        if (threadIdx.x == 0) s_d = find_instance(A.off, A.ninst, item);
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_d);
        const VpInst& I = A.inst[d];
        const int t = item - A.off[d];
        const int nx = I.push.nx, np = I.push.np;
        const bool periodic = I.push.x_periodic != 0;
        const int tiles_x = (nx + kSeg - 1) / kSeg;
        const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
        const int X0 = txi * kSeg, X1 = min(X0 + kSeg, nx);
        const int Y0 = tyi * kSolveXThreads, Y1 = min(Y0 + kSolveXThreads, np);
        const int rc0 = periodic ? X0 - kHalo : max(0, X0 - kHalo);
        const int rc1 = periodic ? X1 + kHalo : min(nx, X1 + kHalo);
        const int RW = rc1 - rc0, th = Y1 - Y0, tw = X1 - X0;
        const int par = (I.parity0 + A.parity) & 1;
        const float* __restrict__ src = I.b;
        float* __restrict__ dst = I.w[par];  // the state just deposited from
        const float inv_nx = 1.0f / (float)nx;
        constexpr int ldw = kLine + 1;

        if (threadIdx.x < kEdge)
            s_edge[threadIdx.x] = periodic ? make_float2(kMinf, kMinf) : I.coef_x[min((int)threadIdx.x, nx - 1)];
        // stage rows Y0..Y1, columns rc0..rc1: lane = column, loop over rows
        for (int c = threadIdx.x; c < kLine; c += blockDim.x) {
            int gc = rc0 + min(c, RW - 1);
            if (periodic) gc = wrap_index(gc, nx, inv_nx);
            const float* col = src + (size_t)Y0 * nx + gc;
#pragma unroll 16
            for (int r = 0; r < th; ++r) lds[r * ldw + c] = c < RW ? col[(size_t)r * nx] : 0.0f;
        }
        __syncthreads();

        const int first = (!periodic && rc0 < kEdge) ? rc0 : kEdge;
        if ((int)threadIdx.x < th) {
            float v[kLine];
            float* row = lds + threadIdx.x * ldw;
#pragma unroll
            for (int k = 0; k < kLine; ++k) v[k] = row[k];
            line_solve_any(v, RW, first, s_edge);
#pragma unroll
            for (int k = 0; k < kLine; ++k) row[k] = v[k];
        }
        __syncthreads();

        for (int c = threadIdx.x; c < tw; c += blockDim.x) {
            float* col = dst + (size_t)Y0 * nx + X0 + c;
            const int lc = X0 - rc0 + c;
#pragma unroll 16
            for (int r = 0; r < th; ++r) col[(size_t)r * nx] = lds[r * ldw + lc];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSolvePThreads) void k_solve_p(LaunchArgs A) {
    __shared__ int s_d;
    __shared__ int s_last;
    __shared__ float2 s_edge[kEdge];
    __shared__ double s_red[2][kSolvePThreads / 64];

    for (int item = blockIdx.x; item < A.total; item += gridDim.x) {
        if (threadIdx.x == 0) s_d = find_instance(A.off, A.ninst, item);
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_d);
        const VpInst& I = A.inst[d];
        const int t = item - A.off[d];
        const int nx = I.push.nx, np = I.push.np;
        const int tiles_x = (nx + kSolvePThreads - 1) / kSolvePThreads;
        const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
        const int col = txi * kSolvePThreads + threadIdx.x;
        const int Y0 = tyi * kSeg, Y1 = min(Y0 + kSeg, np);
        const int rr0 = max(0, Y0 - kHalo), rr1 = min(np, Y1 + kHalo);
        const int RH = rr1 - rr0;
        const int par = (I.parity0 + A.parity) & 1;
        const float* __restrict__ src = I.w[par];
        float* __restrict__ dst = I.w[par ^ 1];

        if (threadIdx.x < kEdge) s_edge[threadIdx.x] = I.coef_p[min((int)threadIdx.x, np - 1)];
        __syncthreads();

        const bool fel = I.push.kind == kFel;
        double acc_re = 0.0, acc_im = 0.0;
        if (col < nx) {
            float v[kLine];
            const float* c0 = src + (size_t)rr0 * nx + col;
#pragma unroll
            for (int k = 0; k < kLine; ++k) {
                const float x = c0[(size_t)min(k, RH - 1) * nx];
                v[k] = k < RH ? x : 0.0f;
            }
            line_solve_any(v, RH, rr0 < kEdge ? rr0 : kEdge, s_edge);
            float* o = dst + col;
            const int lo = Y0 - rr0;
            double cre = 0.0, cim = 0.0;
#pragma unroll
            for (int k = 0; k < kLine; ++k) {
                if (k >= lo && k < lo + (Y1 - Y0)) {
                    o[(size_t)(rr0 + k) * nx] = v[k];
                    if (fel) {
                        const double2 e = I.fel_eq[rr0 + k];  // times e^{-i q}
                        cre += (double)v[k] * e.x;
                        cim -= (double)v[k] * e.y;
                    }
                }
            }
            if (fel) {
                const double2 e = I.fel_ex[col];  // times e^{-i phi}
                acc_re = cre * e.x + cim * e.y;
                acc_im = cim * e.x - cre * e.y;
            }
        }

        if (fel) {
            // FP64 bunching of the new state: tile partial, then the last tile
            // of the instance sums all partials in tile order.
            for (int o = 32; o > 0; o >>= 1) {
                acc_re += __shfl_down(acc_re, o);
                acc_im += __shfl_down(acc_im, o);
            }
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
            if (lane == 0) { s_red[0][wid] = acc_re; s_red[1][wid] = acc_im; }
            __syncthreads();
            if (threadIdx.x == 0) {
                double re = 0.0, im = 0.0;
                for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { re += s_red[0][k]; im += s_red[1][k]; }
                I.partials[2 * t] = re;
                I.partials[2 * t + 1] = im;
                __threadfence();
                const uint32_t prev = atomicAdd(I.counters, 1u);
                s_last = (prev == (uint32_t)(I.k2_tiles - 1));
            }
            __syncthreads();
            if (s_last) {
                __threadfence();
                double re = 0.0, im = 0.0;
                for (int k = threadIdx.x; k < I.k2_tiles; k += blockDim.x) {
                    re += __builtin_nontemporal_load(&I.partials[2 * k]);
                    im += __builtin_nontemporal_load(&I.partials[2 * k + 1]);
                }
                for (int o = 32; o > 0; o >>= 1) {
                    re += __shfl_down(re, o);
                    im += __shfl_down(im, o);
                }
                __syncthreads();
                if (lane == 0) { s_red[0][wid] = re; s_red[1][wid] = im; }
                __syncthreads();
                if (threadIdx.x == 0) {
                    re = 0.0;
                    im = 0.0;
                    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { re += s_red[0][k]; im += s_red[1][k]; }
                    double* st = I.fel_state;
                    const double inv_n0 = 1.0 / st[kN0];
                    // A advances by the bunching of the state that was pushed (eq. 13c)
                    st[kA] += I.fel_dz * st[kBn];
                    st[kA + 1] += I.fel_dz * st[kBn + 1];
                    st[kBn] = re * inv_n0;
                    st[kBn + 1] = im * inv_n0;
                    st[kDzB] = I.fel_dz;
                    __threadfence();
                    atomicExch(I.counters, 0u);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_reduce: FP64 sums over one state, fixed-order (deterministic) reduction.
//  mode 0 (diagnostics): sum w, sum_{w<0} w, sum |w|, sum_{w>0} w ln w,
//    sum w p, sum w (kinetic + potential), sum w cos x, sum w sin x, max |w|,
//    #nonfinite.
//  mode 1 (FEL bunching): sum w e^{-i (phi_i + q_j)} / N0 -> fel_state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_reduce(ReduceArgs R) {
    __shared__ double s_part[kReduceThreads / 64][kMoments];
    __shared__ int s_last;
    double acc[kMoments];
#pragma unroll
    for (int k = 0; k < kMoments; ++k) acc[k] = 0.0;
    const long n = (long)R.nx * R.np;
    const double cosfac = [&] {
        double y = 0.5 * R.hx;
        double sc = y == 0.0 ? 1.0 : sin(y) / y;
        return sc * sc;
    }();
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const int j = (int)(k / R.nx), i = (int)(k - (long)j * R.nx);
        const double w = (double)R.w[k];
        if (R.mode == 1) {
            const double2 ex = R.fel_ex[i], eq = R.fel_eq[j];
            // e^{-i(phi+q)} = (cos phi cos q - sin phi sin q) - i (sin phi cos q + cos phi sin q)
            acc[0] += w * (ex.x * eq.x - ex.y * eq.y);
            acc[1] -= w * (ex.y * eq.x + ex.x * eq.y);
            continue;
        }
        if (!isfinite(w)) { acc[9] += 1.0; continue; }
        const double x = R.x_lo + (double)i * R.hx, p = R.p_lo + (double)j * R.hp;
        acc[0] += w;
        acc[8] = fmax(acc[8], fabs(w));
        if (w < 0.0) acc[1] += w;
        acc[2] += fabs(w);
        if (w > 0.0) acc[3] += w * log(w);
        acc[4] += w * p;
        double e = 0.5 * (p * p + R.hp * R.hp / 6.0);
        if (R.kind == kPendulum) e -= R.a * cosfac * cos(x);
        else if (R.kind == kSho) e += 0.5 * (x * x + R.hx * R.hx / 6.0);
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

hipError_t launch_deposit(const LaunchArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(k_deposit, dim3(grid), dim3(kDepositThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_solve_x(const LaunchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_x, dim3(grid), dim3(kSolveXThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_solve_p(const LaunchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_p, dim3(grid), dim3(kSolvePThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

const void* deposit_kernel() { return reinterpret_cast<const void*>(&k_deposit); }
const void* solve_x_kernel() { return reinterpret_cast<const void*>(&k_solve_x); }
const void* solve_p_kernel() { return reinterpret_cast<const void*>(&k_solve_p); }

}  // namespace vp
