/*
 * vp_oracle.c -- plain FP64 CPU oracle of one phase-space-conservation Vlasov step.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the GPU smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code with the
 * GPU library (paper_2007_12227_amd/csrc) and the GPU library never calls it.
 *
 * What one step computes (Edelen & Webb, "A Vlasov Algorithm Derived from Phase
 * Space Conservation"):
 *   f(x,p) = sum_j w_j Lambda(x-x_j) Lambda(p-p_j)          (Sec. Algorithm, eq. 4)
 *   every lattice node is pushed one step by a particle pusher (Sec. Background,
 *   eq. vlasov_flow, and eqs. 6-7), and the pushed tents are projected back on
 *   the fixed lattice:
 *   sum_j Lambda_{jj'} w_j^fin = sum_k Delta_{kj'} w_k^in   (eqs. 7-9)
 *   w^fin = Lambda^{-1} Delta^T w^in                         (eq. 10)
 * With the tent basis of width h, the overlap of two tents whose centres are
 * s*h apart is h*B3(s), B3 the centred cubic B-spline.  Hence
 *   Delta_{kj'}  = h_x h_p B3((X_k-x_j')/h_x) B3((P_k-p_j')/h_p)
 *   Lambda_{jj'} = h_x h_p M_x (x) M_p,   M = tridiag(1/6, 2/3, 1/6)
 * (cyclic on a periodic axis).  The h_x h_p factors cancel, so the step is the
 * B3 scatter of every pushed node followed by one tridiagonal solve per
 * lattice line along each axis.  Lambda^{-1} = M_x^{-1} (x) M_p^{-1} exactly,
 * so this is the paper's dense update to rounding.
 *
 * Readings where the paper is silent, ambiguous or garbled:
 *  - force sign: Hamilton's equations x' = p, p' = -V'(x)  (eq. 2 is garbled);
 *  - pendulum V(x) = -a cos x; the symplectic integrator is drift-kick-drift;
 *  - the harmonic oscillator is advanced by the exact rotation of
 *    H = (p^2+x^2)/2 through the angle omega*dt (Sec. Harmonic Oscillators);
 *  - FEL (Sec. FEL simulations, eqs. 13a-c): drift-kick-drift with the kick
 *    sub-flow integrated exactly (phase frozen, so <e^{-i Phi}> is constant and
 *    A grows linearly through the kick); the average <.> is N0^{-1} sum w e^{-i psi}
 *    over the nodes at their half-drift phases, N0 = sum w at the start.  The
 *    paper's own integrator, fourth-order Runge-Kutta, is the alternative
 *    (orc_push_rk4): there <.> is taken at each stage's phases;
 *  - periodic axis: n nodes on [lo,hi); open axis: n nodes including both ends,
 *    full tents at the edge nodes, taps that fall outside are lost
 *    (Sec. Numerical Examples: open momentum boundaries lose density).
 *
 * Parallelism: the push and the line solves are independent per node / per
 * line (OpenMP); the scatter runs serially in source order, so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FREE 0
#define ORC_SHO_EXACT 1
#define ORC_PENDULUM 2
#define ORC_FEL 3

typedef struct {
    double lo, hi;
    int32_t n;
    int32_t periodic;
} orc_axis;

#define ORC_DKD 0 /* FEL integrator: drift, exact kick, drift */
#define ORC_RK4 1 /* FEL integrator: classical fourth-order Runge-Kutta (Sec. FEL simulations) */

typedef struct {
    int32_t kind;
    int32_t integrator; /* FEL only: ORC_DKD or ORC_RK4 */
    double a;          /* pendulum amplitude, V = -a cos x */
    double omega;      /* rotation angle per unit time */
    double fel_delta;  /* detuning, eq. 13a */
    double fel_sigma2; /* space-charge coefficient, eq. 13b */
} orc_ham;

typedef struct {
    double sum_w, mass, neg_mass, l1, entropy, mean_p, energy;
    double A_re, A_im, bunch_re, bunch_im, fel_invariant;
    int64_t step;
} orc_moments;

static double spacing(const orc_axis* a) { return (a->hi - a->lo) / (a->periodic ? a->n : a->n - 1); }
static double node_at(const orc_axis* a, long i) { return a->lo + (double)i * spacing(a); }

/* Map a lattice index onto the axis: wrap on a periodic axis, -1 if outside an open one. */
static long axis_index(const orc_axis* a, long i) {
    if (a->periodic) {
        long m = i % a->n;
        return m < 0 ? m + a->n : m;
    }
    return (i < 0 || i >= a->n) ? -1 : i;
}

/* Overlap integral of two unit-height tents of half-width h, centres s*h apart, over h. */
double orc_b3(double s) {
    s = fabs(s);
    if (s < 1.0) return 2.0 / 3.0 - s * s + 0.5 * s * s * s;
    if (s < 2.0) {
        double t = 2.0 - s;
        return t * t * t / 6.0;
    }
    return 0.0;
}

/* ---- push (Sec. Background: any particle pusher approximates the flow) ---- */

/* Displacement of one phase-space point over one step.  At = FEL kick field
 * (A + b dz/2 + i sigma2 b), ignored by the other kinds. */
static void push_point(const orc_ham* h, double dt, double x, double p, const double At[2],
                       double* dx, double* dp) {
    switch (h->kind) {
    case ORC_FREE:
        *dx = p * dt;
        *dp = 0.0;
        break;
    case ORC_SHO_EXACT: {
        double th = h->omega * dt, c = cos(th), s = sin(th);
        double X = x * c + p * s, P = -x * s + p * c;
        *dx = X - x;
        *dp = P - p;
        break;
    }
    case ORC_PENDULUM: {
        /* drift dt/2, kick dt with force -V'(x) = -a sin x, drift dt/2 */
        double xh = x + 0.5 * dt * p;
        double pn = p - h->a * sin(xh) * dt;
        double xn = xh + 0.5 * dt * pn;
        *dx = xn - x;
        *dp = pn - p;
        break;
    }
    case ORC_FEL: {
        /* drift dz/2 (dpsi/dz = delta + eta), exact kick dz, drift dz/2 */
        double ph = x + 0.5 * dt * (h->fel_delta + p);
        double pn = p - 2.0 * dt * (At[0] * cos(ph) - At[1] * sin(ph));
        double xn = ph + 0.5 * dt * (h->fel_delta + pn);
        *dx = xn - x;
        *dp = pn - p;
        break;
    }
    default:
        *dx = *dp = 0.0;
    }
}

/* Displacement of every lattice node in cell units (du = dx/h_x, dv = dp/h_p). */
void orc_push(const orc_axis* ax, const orc_axis* ap, const orc_ham* h, double dt,
              const double* At, double* du, double* dv) {
    const double hx = spacing(ax), hp = spacing(ap);
    const double zero[2] = {0.0, 0.0};
    if (!At) At = zero;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < ap->n; ++j) {
        double p = node_at(ap, j);
        for (long i = 0; i < ax->n; ++i) {
            double dx, dp;
            push_point(h, dt, node_at(ax, i), p, At, &dx, &dp);
            du[j * ax->n + i] = dx / hx;
            dv[j * ax->n + i] = dp / hp;
        }
    }
}

/* ---- projection right-hand side b = Delta^T w (eq. 9) ---- */

void orc_deposit(const orc_axis* ax, const orc_axis* ap, const double* du, const double* dv,
                 const double* w, double* b) {
    const long nx = ax->n, np = ap->n;
    memset(b, 0, sizeof(double) * nx * np);
    for (long j = 0; j < np; ++j) {
        for (long i = 0; i < nx; ++i) {
            const long k = j * nx + i;
            const double u = (double)i + du[k], v = (double)j + dv[k];
            const long i0 = (long)floor(u), j0 = (long)floor(v);
            for (long row = j0 - 1; row <= j0 + 2; ++row) {
                long jr = axis_index(ap, row);
                if (jr < 0) continue;
                const double wp = w[k] * orc_b3(v - (double)row);
                for (long col = i0 - 1; col <= i0 + 2; ++col) {
                    long ic = axis_index(ax, col);
                    if (ic < 0) continue;
                    b[jr * nx + ic] += wp * orc_b3(u - (double)col);
                }
            }
        }
    }
}

/* ---- Lambda^{-1}: one tridiagonal solve per lattice line (eq. 8) ---- */

/* Thomas elimination of tridiag(1/6, diag[i], 1/6) y = r on n points, in place in r. */
static void thomas(long n, const double* diag, double* r, long stride, double* cp) {
    const double off = 1.0 / 6.0;
    double m = diag[0];
    cp[0] = off / m;
    r[0] /= m;
    for (long i = 1; i < n; ++i) {
        m = diag[i] - off * cp[i - 1];
        cp[i] = off / m;
        r[i * stride] = (r[i * stride] - off * r[(i - 1) * stride]) / m;
    }
    for (long i = n - 2; i >= 0; --i) r[i * stride] -= cp[i] * r[(i + 1) * stride];
}

/* Solve M y = r along one line of n points (stride apart), M cyclic if periodic.
 * The cyclic case uses the Sherman-Morrison formula: M = T + u v^T with T
 * tridiagonal, u = (g, 0.., 1/6), v = (1, 0.., (1/6)/g), g = -2/3. */
static void solve_line(long n, int periodic, double* r, long stride, double* work) {
    double* diag = work;
    double* cp = work + n;
    double* z = work + 2 * n;
    for (long i = 0; i < n; ++i) diag[i] = 2.0 / 3.0;
    if (!periodic) {
        thomas(n, diag, r, stride, cp);
        return;
    }
    const double off = 1.0 / 6.0, g = -2.0 / 3.0;
    diag[0] -= g;
    diag[n - 1] -= off * off / g;
    thomas(n, diag, r, stride, cp);
    for (long i = 0; i < n; ++i) z[i] = 0.0;
    z[0] = g;
    z[n - 1] = off;
    thomas(n, diag, z, 1, cp);
    const double vy = r[0] + (off / g) * r[(n - 1) * stride];
    const double vz = z[0] + (off / g) * z[n - 1];
    const double f = vy / (1.0 + vz);
    for (long i = 0; i < n; ++i) r[i * stride] -= f * z[i];
}

/* w <- (M_x^{-1} (x) M_p^{-1}) w, in place. */
void orc_solve(const orc_axis* ax, const orc_axis* ap, double* w) {
    const long nx = ax->n, np = ap->n;
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * 3 * (nx > np ? nx : np));
#pragma omp for schedule(static)
        for (long j = 0; j < np; ++j) solve_line(nx, ax->periodic, w + j * nx, 1, work);
#pragma omp for schedule(static)
        for (long i = 0; i < nx; ++i) solve_line(np, ap->periodic, w + i, nx, work);
        free(work);
    }
}

/* ---- FEL field coupling (eqs. 13b-c) ---- */

/* b = N0^{-1} sum_k w_k exp(-i psi_k), psi at the half-drift position psi + (delta+eta) dz/2. */
void orc_bunching(const orc_axis* ax, const orc_axis* ap, const orc_ham* h, double dz,
                  const double* w, double N0, double* b) {
    double re = 0.0, im = 0.0;
    for (long j = 0; j < ap->n; ++j) {
        const double eta = node_at(ap, j);
        for (long i = 0; i < ax->n; ++i) {
            const double ph = node_at(ax, i) + 0.5 * dz * (h->fel_delta + eta);
            const double wk = w[j * ax->n + i];
            re += wk * cos(ph);
            im -= wk * sin(ph);
        }
    }
    b[0] = re / N0;
    b[1] = im / N0;
}

/* ---- FEL by the classical Runge-Kutta method (Sec. FEL simulations) ----
 *
 * The lattice nodes are the particles of eqs. 13a-c: psi_k' = delta + eta_k,
 * eta_k' = F(psi_k, A, b) = -2 Re[(A + i sigma2 b) e^{i psi_k}], A' = b with
 * b = N0^{-1} sum_k w_k e^{-i psi_k} over the current phases.  One step of
 * size h takes the four stages of the method; each needs the bunching of its
 * own stage phases, a sum over all nodes.  Stage s (s = 1..4) evaluates the
 * slopes at psi_s = psi + c_s h k_{s-1}^psi, eta_s = eta + c_s h k_{s-1}^eta,
 * A_s = A + c_s h b_{s-1}, with c = (0, 1/2, 1/2, 1); the update weighs the
 * stages 1, 2, 2, 1 over 6.  The weights w stay fixed through the step: they
 * are the particles' charges, moved only by the projection that follows. */

static double fel_force(const orc_ham* h, double ph, const double A[2], const double b[2]) {
    /* -2 Re[(A + i sigma2 b) e^{i ph}] */
    const double re = A[0] - h->fel_sigma2 * b[1], im = A[1] + h->fel_sigma2 * b[0];
    return -2.0 * (re * cos(ph) - im * sin(ph));
}

static void add_bunch(double wk, double ph, double* acc) {
    acc[0] += wk * cos(ph);
    acc[1] -= wk * sin(ph);
}

/* Displacements (cells) of every node over one RK4 step, and the new field. */
void orc_push_rk4(const orc_axis* ax, const orc_axis* ap, const orc_ham* h, double dz, const double* w,
                  double N0, const double* A, double* du, double* dv, double* A_new) {
    const long nx = ax->n, np = ap->n;
    const double hx = spacing(ax), hp = spacing(ap), d = h->fel_delta;
    double b[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    double As[4][2];
    /* stage 1 and 2 phases need no bunching: psi, and psi + (h/2)(delta + eta) */
    for (long j = 0; j < np; ++j) {
        const double eta = node_at(ap, j);
        for (long i = 0; i < nx; ++i) {
            const double psi = node_at(ax, i), wk = w[j * nx + i];
            add_bunch(wk, psi, b[0]);
            add_bunch(wk, psi + 0.5 * dz * (d + eta), b[1]);
        }
    }
    for (int c = 0; c < 2; ++c) b[0][c] /= N0, b[1][c] /= N0;
    for (int c = 0; c < 2; ++c) {
        As[0][c] = A[c];
        As[1][c] = A[c] + 0.5 * dz * b[0][c];
        As[2][c] = A[c] + 0.5 * dz * b[1][c];
    }
    /* stages 3 and 4: their phases need the slopes of stages 1 and 2 */
    for (long j = 0; j < np; ++j) {
        const double eta = node_at(ap, j);
        for (long i = 0; i < nx; ++i) {
            const double psi = node_at(ax, i), wk = w[j * nx + i];
            const double k1e = fel_force(h, psi, As[0], b[0]);
            const double psi2 = psi + 0.5 * dz * (d + eta), eta2 = eta + 0.5 * dz * k1e;
            const double k2e = fel_force(h, psi2, As[1], b[1]);
            const double psi3 = psi + 0.5 * dz * (d + eta2);
            const double eta3 = eta + 0.5 * dz * k2e;
            const double psi4 = psi + dz * (d + eta3);
            add_bunch(wk, psi3, b[2]);
            add_bunch(wk, psi4, b[3]);
        }
    }
    for (int c = 0; c < 2; ++c) {
        b[2][c] /= N0, b[3][c] /= N0;
        As[3][c] = A[c] + dz * b[2][c];
    }
    /* the step itself */
#pragma omp parallel for schedule(static)
    for (long j = 0; j < np; ++j) {
        const double eta = node_at(ap, j);
        for (long i = 0; i < nx; ++i) {
            const double psi = node_at(ax, i);
            const double k1p = d + eta, k1e = fel_force(h, psi, As[0], b[0]);
            const double psi2 = psi + 0.5 * dz * k1p, eta2 = eta + 0.5 * dz * k1e;
            const double k2p = d + eta2, k2e = fel_force(h, psi2, As[1], b[1]);
            const double psi3 = psi + 0.5 * dz * k2p, eta3 = eta + 0.5 * dz * k2e;
            const double k3p = d + eta3, k3e = fel_force(h, psi3, As[2], b[2]);
            const double psi4 = psi + dz * k3p, eta4 = eta + dz * k3e;
            const double k4p = d + eta4, k4e = fel_force(h, psi4, As[3], b[3]);
            du[j * nx + i] = dz / 6.0 * (k1p + 2.0 * k2p + 2.0 * k3p + k4p) / hx;
            dv[j * nx + i] = dz / 6.0 * (k1e + 2.0 * k2e + 2.0 * k3e + k4e) / hp;
        }
    }
    for (int c = 0; c < 2; ++c) A_new[c] = A[c] + dz / 6.0 * (b[0][c] + 2.0 * b[1][c] + 2.0 * b[2][c] + b[3][c]);
}

/* ---- diagnostics (Sec. Numerical Examples: phase-space volume and entropy) ---- */

static double sinc(double y) { return y == 0.0 ? 1.0 : sin(y) / y; }

void orc_moments_of(const orc_axis* ax, const orc_axis* ap, const orc_ham* h, const double* w,
                    const double* A, double N0, int64_t step, orc_moments* m) {
    const double hx = spacing(ax), hp = spacing(ap), cell = hx * hp;
    double s = 0, neg = 0, l1 = 0, ent = 0, sp = 0, en = 0, bre = 0, bim = 0;
    /* exact tent integrals: int p^2 Lambda_j dp = h (p_j^2 + h^2/6),
       int cos x Lambda_i dx = h sinc^2(h/2) cos x_i */
    const double cosfac = sinc(0.5 * hx) * sinc(0.5 * hx);
    for (long j = 0; j < ap->n; ++j) {
        const double p = node_at(ap, j);
        const double kin = 0.5 * (p * p + hp * hp / 6.0);
        for (long i = 0; i < ax->n; ++i) {
            const double x = node_at(ax, i), wk = w[j * ax->n + i];
            s += wk;
            l1 += fabs(wk);
            if (wk < 0) neg -= wk;
            if (wk > 0) ent -= wk * log(wk);
            sp += wk * p;
            double pot = 0.0;
            if (h->kind == ORC_PENDULUM) pot = -h->a * cosfac * cos(x);
            else if (h->kind == ORC_SHO_EXACT) pot = 0.5 * (x * x + hx * hx / 6.0);
            en += wk * (kin + pot);
            bre += wk * cos(x);
            bim -= wk * sin(x);
        }
    }
    memset(m, 0, sizeof(*m));
    m->sum_w = s;
    m->mass = cell * s;
    m->neg_mass = cell * neg;
    m->l1 = cell * l1;
    m->entropy = cell * ent;
    m->mean_p = s != 0.0 ? sp / s : 0.0;
    m->energy = cell * en;
    m->step = step;
    if (h->kind == ORC_FEL) {
        m->A_re = A ? A[0] : 0.0;
        m->A_im = A ? A[1] : 0.0;
        m->bunch_re = bre / N0;
        m->bunch_im = bim / N0;
        m->fel_invariant = m->A_re * m->A_re + m->A_im * m->A_im + sp / N0;
    }
}

/* ---- one full step and a run of steps (eq. 10) ---- */

/* Advance w (and the FEL field A) by nsteps steps of size dt.  N0 is the FEL
 * normalisation (sum of w at z = 0).  If round_fp32, the state is rounded to
 * float after every step: the best any FP32-state implementation can reach.
 * If series != NULL it receives the moments after every step. */
int orc_run(const orc_axis* ax, const orc_axis* ap, const orc_ham* h, double dt, int64_t nsteps,
            double* w, double* A, double N0, int32_t round_fp32, orc_moments* series) {
    if (!ax || !ap || !h || !w || ax->n < 4 || ap->n < 4) return -1;
    if (h->kind == ORC_FEL && (!A || !(N0 != 0.0))) return -1;
    const long n = (long)ax->n * ap->n;
    double* du = (double*)malloc(sizeof(double) * n);
    double* dv = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    if (!du || !dv || !b) {
        free(du); free(dv); free(b);
        return -2;
    }
    int static_map = h->kind != ORC_FEL;
    if (static_map) orc_push(ax, ap, h, dt, NULL, du, dv);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (!static_map && h->integrator == ORC_RK4) {
            double An[2];
            orc_push_rk4(ax, ap, h, dt, w, N0, A, du, dv, An);
            A[0] = An[0];
            A[1] = An[1];
        } else if (!static_map) {
            double bn[2];
            orc_bunching(ax, ap, h, dt, w, N0, bn);
            /* kick field: A grows linearly through the kick, so the kick sees
               its mid-kick value; the space-charge term adds i sigma2 b */
            double At[2] = {A[0] + 0.5 * dt * bn[0] - h->fel_sigma2 * bn[1],
                            A[1] + 0.5 * dt * bn[1] + h->fel_sigma2 * bn[0]};
            orc_push(ax, ap, h, dt, At, du, dv);
            A[0] += dt * bn[0];
            A[1] += dt * bn[1];
        }
        orc_deposit(ax, ap, du, dv, w, b);
        orc_solve(ax, ap, b);
        if (round_fp32)
            for (long k = 0; k < n; ++k) w[k] = (double)(float)b[k];
        else
            memcpy(w, b, sizeof(double) * n);
        if (series) orc_moments_of(ax, ap, h, w, A, N0, s + 1, &series[s]);
    }
    free(du);
    free(dv);
    free(b);
    return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
