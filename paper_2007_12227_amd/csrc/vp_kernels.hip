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

// Cubic B-spline tap weights B3(t+1), B3(t), B3(1-t), B3(2-t) for t in [0,1).
// The second tap is 1 minus the others, so the four sum to one to rounding
// (the partition of unity behind the conservation argument of eqs. 11-12).
__device__ inline void bspline_taps(float t, float (&b)[4]) {
    const float sixth = 1.0f / 6.0f;
    float s = 1.0f - t;
    float t2 = t * t;
    b[0] = (s * sixth) * (s * s);
    b[3] = (t * sixth) * t2;
    b[2] = fmaf(0.5f, t + t2, sixth) - 3.0f * b[3];
    b[1] = 1.0f - ((b[0] + b[3]) + b[2]);
}

// Round a float of magnitude below 2^62 to a 64-bit integer (two's complement
// bits): v = hi * 2^32 + lo with hi = floor(v / 2^32) and 0 <= lo < 2^32; both
// parts are exact in FP32 whenever |v| >= 2^32, and for smaller |v| the low
// part rounds to a multiple of at most 2^8, i.e. 2^-49 of the tile maximum.
__device__ inline unsigned long long fix64(float v) {
    const float hf = floorf(v * 2.3283064365386963e-10f);  // 2^-32
    const int hi = (int)hf;
    const float lo = fminf(fmaf(hf, -4294967296.0f, v), 4294967040.0f);
    const unsigned lo_u = (unsigned)lo;
    return ((unsigned long long)(unsigned)hi << 32) + (unsigned long long)lo_u;
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
    __shared__ float s_max[kDepositThreads / 64];

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
                P.alpha = (float)((double)I.fel_kick * are);
                P.beta = (float)(-(double)I.fel_kick * aim);
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
        // to a multiple of 2^-57 * max|w| over the source box and accumulated
        // with 64-bit integer LDS atomics, so the sum does not depend on the
        // order of the atomics (bitwise reproducible).  The map is area
        // preserving, so a cell collects about max|w|; 6 spare bits cover 64x.
        float wmax = 0.0f;
        for (int s = threadIdx.x; s < nsrc; s += blockDim.x) {
            int r = (int)(((float)s + 0.5f) * inv_bw);
            int c = s - r * bw;
            if (c < 0) { c += bw; --r; }
            if (c >= bw) { c -= bw; ++r; }
            const int ii = bx0 + c;
            const int i = periodic ? wrap_index(ii, nx, inv_nx) : ii;
            wmax = fmaxf(wmax, fabsf(w_in[(size_t)(by0 + r) * nx + i]));
        }
        for (int o = 32; o > 0; o >>= 1) wmax = fmaxf(wmax, __shfl_xor(wmax, o));
        if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = wmax;
        __syncthreads();
        wmax = s_max[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) wmax = fmaxf(wmax, s_max[k]);
        // scale = 2^(57 - e) with max|w| < 2^e
        const int e = wmax > 0.0f ? max(ilogbf(wmax) + 1, kFixBits - 127) : 0;
        const float scale = ldexpf(1.0f, kFixBits - e), inv_scale = ldexpf(1.0f, e - kFixBits);
        const int nsrc_live = wmax > 0.0f ? nsrc : 0;

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
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float wq = w * bp[q];
                long long* row = base + q * ldw;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) atomicAdd((unsigned long long*)(row + rr), fix64(wq * bx[rr]));
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
// k_solve: w_out = (M_x^{-1} (x) M_p^{-1}) b on one tile.  Each line is solved
// with the LU recursions of T = tridiag(1,4,1) = 6 M:
//   forward  z_k = b_k - m_k z_{k-1},   backward y_k = (z_k - y_{k+1}) / d_k,
// with exact per-node (m_k, 1/d_k) on an open axis (so the true edges are
// exact) and the interior constants on a periodic one.  Where the tile's halo
// is cut inside the lattice the recursion starts from zero; the error decays
// by 2 - sqrt 3 per node and is ~7e-10 after the 16-node halo.  The factor 6
// per axis is applied once at the end as scale_hi + scale_lo, chosen so that
// the FP32 coefficients give a DC gain of exactly one.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSolveThreads) void k_solve(LaunchArgs A) {
    extern __shared__ float lds[];
    __shared__ int s_d;
    __shared__ double s_red[2][kSolveThreads / 64];
    __shared__ int s_last;

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
        const int par = (I.parity0 + A.parity) & 1;
        float* __restrict__ w_out = I.w[par ^ 1];
        const float* __restrict__ b = I.b;
        const float inv_nx = 1.0f / (float)nx;
        const float inv_rw = 1.0f / (float)RW;

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
            float z = 0.0f;
            if (periodic) {
                for (int c = 0; c < RW; ++c) { z = fmaf(-kMinf, z, L[c]); L[c] = z; }
                float y = 0.0f;
                for (int c = RW - 1; c >= 0; --c) { y = (L[c] - y) * kMinf; L[c] = y; }
            } else {
                const float2* cf = I.coef_x + rc0;
                for (int c = 0; c < RW; ++c) { z = fmaf(-cf[c].x, z, L[c]); L[c] = z; }
                float y = 0.0f;
                for (int c = RW - 1; c >= 0; --c) { y = (L[c] - y) * cf[c].y; L[c] = y; }
            }
        }
        __syncthreads();

        // p lines: one thread per output column
        const int tw = X1 - X0;
        const bool fel = I.push.kind == kFel;
        double acc_re = 0.0, acc_im = 0.0;
        for (int c = threadIdx.x; c < tw; c += blockDim.x) {
            const int lc = X0 - rc0 + c;
            const float2* cf = I.coef_p + rr0;
            float z = 0.0f;
            for (int r = 0; r < RH; ++r) {
                z = fmaf(-cf[r].x, z, lds[r * ldw + lc]);
                lds[r * ldw + lc] = z;
            }
            float y = 0.0f;
            double cre = 0.0, cim = 0.0;
            for (int r = RH - 1; r >= 0; --r) {
                y = (lds[r * ldw + lc] - y) * cf[r].y;
                const int gr = rr0 + r;
                if (gr >= Y0 && gr < Y1) {
                    const float out = fmaf(y, I.scale_hi, y * I.scale_lo);
                    w_out[(size_t)gr * nx + X0 + c] = out;
                    if (fel) {
                        const double2 e = I.fel_eq[gr];
                        cre += (double)out * e.x;
                        cim -= (double)out * e.y;
                    }
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
//    sum w p, sum w (kinetic + potential), sum w cos x, sum w sin x, #nonfinite.
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
        for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_down(acc[k], o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < kMoments; ++k) s_part[wid][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < kMoments; ++k) {
            double s = 0.0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += s_part[q][k];
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
        for (unsigned q = 0; q < gridDim.x; ++q)
            s += __builtin_nontemporal_load(&R.partials[q * kMoments + threadIdx.x]);
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
