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

// In-place solve of M y = b, M = tridiag(1/6, 2/3, 1/6), along n elements of L
// (stride apart), written as
//     y = b - T^{-1} (D2 b),   T = 6 M = tridiag(1, 4, 1),  D2 b = b[k-1] - 2 b[k] + b[k+1]
// (T = 6 I + D2, so 6 T^{-1} = I - T^{-1} D2).  The LU recursions of T then only
// carry the correction T^{-1} D2 b, so their FP32 rounding (whose fixed point
// is biased on slowly varying data) acts on a term much smaller than b, and
// the mass the line carries is kept to ~1e-10 per step instead of ~1e-8.
// Neighbours outside [0, n) count as zero: exact at an open edge (the
// truncated M), and a cut inside the lattice only disturbs the halo.
// first = index of L[0] from the open edge if below kEdge (exact tabulated
// edge coefficients), else kEdge (interior constants).  Z (same layout as L)
// holds the forward sweep.  Loads are issued eight elements ahead.
template <bool EDGE>
__device__ inline float lu_m(int g, const float2* edge) { return (EDGE && g < kEdge) ? edge[g].x : kMinf; }
template <bool EDGE>
__device__ inline float lu_dinv(int g, const float2* edge) { return (EDGE && g < kEdge) ? edge[g].y : kMinf; }

template <bool EDGE>
__device__ inline void solve_line_t(float* L, float* Z, int stride, int n, int first, const float2* edge) {
    float prev = 0.0f, cur = L[0], acc = 0.0f;
    int k = 0;
    for (; k + 8 < n; k += 8) {
        float nx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) nx[u] = L[(k + 1 + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float m = lu_m<EDGE>(first + k + u, edge);
            acc = fmaf(-m, acc, (prev + nx[u]) - 2.0f * cur);
            Z[(k + u) * stride] = acc;
            prev = cur;
            cur = nx[u];
        }
    }
    for (; k < n; ++k) {
        const float next = k + 1 < n ? L[(k + 1) * stride] : 0.0f;
        const float m = lu_m<EDGE>(first + k, edge);
        acc = fmaf(-m, acc, (prev + next) - 2.0f * cur);
        Z[k * stride] = acc;
        prev = cur;
        cur = next;
    }
    float c = 0.0f;
    k = n - 1;
    for (; k >= 7; k -= 8) {
        float zv[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            zv[u] = Z[(k - u) * stride];
            bv[u] = L[(k - u) * stride];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float dinv = lu_dinv<EDGE>(first + k - u, edge);
            c = (zv[u] - c) * dinv;
            L[(k - u) * stride] = bv[u] - c;
        }
    }
    for (; k >= 0; --k) {
        const float dinv = lu_dinv<EDGE>(first + k, edge);
        c = (Z[k * stride] - c) * dinv;
        L[k * stride] = L[k * stride] - c;
    }
}

// Lines that start kEdge or more nodes from an open edge (all lines of a
// periodic axis) use only the interior constants: no table reads in the loop.
__device__ inline void solve_line(float* L, float* Z, int stride, int n, int first, const float2* edge) {
    if (first >= kEdge) solve_line_t<false>(L, Z, stride, n, first, edge);
    else solve_line_t<true>(L, Z, stride, n, first, edge);
}

}  // namespace

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

        for (int s = threadIdx.x; s < nsrc_live; s += blockDim.x) {
            int r = (int)(((float)s + 0.5f) * inv_bw);
            int c = s - r * bw;
            if (c < 0) { c += bw; --r; }
            if (c >= bw) { c -= bw; ++r; }
            const int j = by0 + r;
            const int ii = bx0 + c;  // unwrapped source column
            const int i = periodic ? wrap_index(ii, nx, inv_nx) : ii;
            const float w = w_in[(size_t)j * nx + i] * scale;
            if (w == 0.0f) continue;
            const float4 tx = I.tab_x[i];
            const float4 tp = I.tab_p[j];
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
            // tap value w * bp * bx formed in FP64 and rounded once, exactly,
            // into the fixed-point tile sum: the deposit adds no FP32 product
            // rounding to the state (the FEL instability amplifies it)
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
// k_solve: w_out = (M_x^{-1} (x) M_p^{-1}) b on one tile, one line at a time
// (solve_line): the LU recursions of T = tridiag(1,4,1),
//   forward  z_k = r_k - m_k z_{k-1},   backward c_k = (z_k - c_{k+1}) / d_k,
// with exact per-node (m_k, 1/d_k) near an open edge (so the true edges are
// exact) and the interior constants elsewhere.  Where the tile's halo is cut
// inside the lattice the recursion starts from zero; the error decays by
// 2 - sqrt 3 per node and is ~7e-10 after the 16-node halo.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSolveThreads) void k_solve(LaunchArgs A) {
    extern __shared__ float lds[];
    __shared__ int s_d;
    __shared__ double s_red[2][kSolveThreads / 64];
    __shared__ int s_last;
    __shared__ float2 s_edge_x[kEdge], s_edge_p[kEdge];

    for (int item = blockIdx.x; item < A.total; item += gridDim.x) {
        if (threadIdx.x == 0) s_d = find_instance(A.off, A.ninst, item);
        __syncthreads();
        const int d = __builtin_amdgcn_readfirstlane(s_d);
        const VpInst& I = A.inst[d];
        const int t = item - A.off[d];
        const int nx = I.push.nx, np = I.push.np;
        const bool periodic = I.push.x_periodic != 0;
        const int tyi = t / I.k2_tiles_x, txi = t - tyi * I.k2_tiles_x;
        const int X0 = txi * I.k2_tx, X1 = min(X0 + I.k2_tx, nx);
        const int Y0 = tyi * I.k2_ty, Y1 = min(Y0 + I.k2_ty, np);
        const int rc0 = periodic ? X0 - kHalo : max(0, X0 - kHalo);
        const int rc1 = periodic ? X1 + kHalo : min(nx, X1 + kHalo);
        const int rr0 = max(0, Y0 - kHalo), rr1 = min(np, Y1 + kHalo);
        const int RW = rc1 - rc0, RH = rr1 - rr0;
        const int ldw = solve_ldw(I.k2_tx);
        const int zoff = ldw * (I.k2_ty + 2 * kHalo);  // second buffer: the forward sweeps
        const int par = (I.parity0 + A.parity) & 1;
        float* __restrict__ w_out = I.w[par ^ 1];
        const float* __restrict__ b = I.b;
        const float inv_nx = 1.0f / (float)nx;
        const float inv_rw = 1.0f / (float)RW;

        // LU coefficients differ from the interior constant only within
        // kEdge nodes of an open axis' first node; stage those in LDS.
        if (threadIdx.x < kEdge) {
            s_edge_p[threadIdx.x] = I.coef_p[min((int)threadIdx.x, np - 1)];
            s_edge_x[threadIdx.x] = periodic ? make_float2(kMinf, kMinf) : I.coef_x[min((int)threadIdx.x, nx - 1)];
        }
        for (int k = threadIdx.x; k < RW * RH; k += blockDim.x) {
            int r = (int)(((float)k + 0.5f) * inv_rw);
            int c = k - r * RW;
            if (c < 0) { c += RW; --r; }
            if (c >= RW) { c -= RW; ++r; }
            int gc = rc0 + c;
            if (periodic) gc = wrap_index(gc, nx, inv_nx);
            lds[r * ldw + c] = b[(size_t)(rr0 + r) * nx + gc];
        }
        __syncthreads();

        // x lines: one thread per row of the region
        for (int r = threadIdx.x; r < RH; r += blockDim.x) {
            float* L = lds + r * ldw;
            // a periodic axis, or a region starting kEdge or more nodes from
            // the open edge, only sees the interior constants
            const bool edge = !periodic && rc0 < kEdge;
            solve_line(L, L + zoff, 1, RW, edge ? rc0 : kEdge, s_edge_x);
        }
        __syncthreads();

        // p lines: one thread per output column
        const int tw = X1 - X0;
        const bool fel = I.push.kind == kFel;
        double acc_re = 0.0, acc_im = 0.0;
        for (int c = threadIdx.x; c < tw; c += blockDim.x) {
            const int lc = X0 - rc0 + c;
            solve_line(lds + lc, lds + zoff + lc, ldw, RH, rr0 < kEdge ? rr0 : kEdge, s_edge_p);
            double cre = 0.0, cim = 0.0;
            for (int gr = Y0; gr < Y1; ++gr) {
                const float out = lds[(gr - rr0) * ldw + lc];
                w_out[(size_t)gr * nx + X0 + c] = out;
                if (fel) {
                    const double2 e = I.fel_eq[gr];
                    cre += (double)out * e.x;
                    cim -= (double)out * e.y;
                }
            }
            if (fel) {
                const double2 e = I.fel_ex[X0 + c];  // times e^{-i phi}
                acc_re += cre * e.x + cim * e.y;
                acc_im += cim * e.x - cre * e.y;
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
                    re = 0.0; im = 0.0;
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

hipError_t launch_solve(const LaunchArgs& a, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(k_solve, dim3(grid), dim3(kSolveThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

const void* deposit_kernel() { return reinterpret_cast<const void*>(&k_deposit); }
const void* solve_kernel() { return reinterpret_cast<const void*>(&k_solve); }

}  // namespace vp
