/*
 * vp.h -- C interface of libvp, the MI355X (gfx950) phase-space-conservation
 * Vlasov solver of Edelen & Webb, "A Vlasov Algorithm Derived from Phase Space
 * Conservation".
 *
 * The method (Sec. "An Algorithm Based on Phase Space Density Conservation"):
 * the density is a sum of tent functions on a fixed 2-D lattice,
 * f(x,p) = sum_j w_j Lambda(x-x_j) Lambda(p-p_j) (eq. 4).  One time step pushes
 * every lattice node with a particle pusher (Sec. "The Vlasov Equation as Flows
 * on Phase Space", eq. vlasov_flow), and projects the moved tents back onto the
 * lattice: w_fin = Lambda^{-1} Delta^T w_in (eqs. 7-10), where Lambda is the
 * tent mass matrix (eq. 8) and Delta the overlap of moved and fixed tents
 * (eq. 9).  Coordinates are periodic and momenta open (Sec. "Numerical
 * Examples"); weight pushed past an open edge is lost.
 *
 * The tents can be replaced by quadratic or cubic B-spline basis functions,
 * the smoother local basis the paper's discussion proposes (vp_set_basis):
 * the overlaps of eq. 9 become B-spline weights of degree 5 or 7 on 6 x 6 or
 * 8 x 8 nodes and the mass matrix of eq. 8 the band
 * (1/120)[1, 26, 66, 26, 1] or (1/5040)[1, 120, 1191, 2416, 1191, 120, 1]
 * per axis.
 *
 * Conventions for every call:
 *  - return 0 on success, a negative VP_E* code on failure; no call throws;
 *    vp_last_error() gives a thread-local message for the last failure;
 *  - arrays are [n_p][n_x] with x fastest, FP32;
 *  - device memory (the workspace, device pointers passed in) belongs to the
 *    caller and must outlive the grid; the library frees nothing it did not
 *    allocate and copies host arrays before returning;
 *  - calls on one grid are not thread-safe; work is ordered on the grid's HIP
 *    stream; vp_step and vp_batch_step return without waiting, vp_moments,
 *    vp_get_density and vp_set_density wait for the stream.
 */
#ifndef VP_H
#define VP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VP_OK 0
#define VP_EINVAL (-1)       /* invalid argument */
#define VP_ENOMEM (-2)       /* workspace missing or too small */
#define VP_ESTATE (-3)       /* call out of order (step before density/Hamiltonian) */
#define VP_EHIP (-4)         /* a HIP runtime call failed */
#define VP_EUNSUPPORTED (-5) /* valid for the method but not built here */
#define VP_ENONFINITE (-6)   /* the state holds NaN or Inf */
#define VP_ERANGE (-7)       /* a deposit cell sum left the fixed-point range */

/* Hamiltonian kinds (Sec. "Numerical Examples") */
#define VP_H_FREE 0       /* free streaming x' = p */
#define VP_H_SHO_EXACT 1  /* H = (p^2+x^2)/2 advanced by its exact rotation (Sec. Harmonic Oscillators) */
#define VP_H_PENDULUM 2   /* H = p^2/2 - a cos x, drift-kick-drift leapfrog (Sec. Harmonic Oscillators) */
#define VP_H_FEL 3        /* 1-D FEL, eqs. 13a-c, self-consistent field A (Sec. FEL simulations) */

/* Basis functions of the expansion (vp_set_basis) */
#define VP_BASIS_TENT 0      /* tents, eq. 4 (the default) */
#define VP_BASIS_QUADRATIC 1 /* centred quadratic B-splines of width 3h on every node */
#define VP_BASIS_CUBIC 2     /* centred cubic B-splines of width 4h on every node */

/* FEL integrators */
#define VP_FEL_DKD 0 /* drift dz/2, exact kick dz, drift dz/2 (one bunching per step) */
#define VP_FEL_RK4 1 /* classical fourth-order Runge-Kutta, the paper's integrator (four bunchings per step) */

typedef struct vp_grid vp_grid;
typedef struct vp_batch vp_batch;

/* One lattice axis.  periodic != 0: n nodes on [lo, hi), spacing (hi-lo)/n.
 * periodic == 0: n nodes on [lo, hi] including both ends, spacing (hi-lo)/(n-1).
 * n >= 4.  The momentum axis (p) must be open. */
typedef struct {
    double lo, hi;
    int32_t n;
    int32_t periodic;
} vp_axis;

/* Grid creation.  workspace: caller-owned device memory of at least
 * vp_workspace_bytes(&x, &p) bytes, 256-byte aligned.  stream: a hipStream_t
 * (NULL = the default stream) on which all work of this grid is ordered. */
typedef struct {
    vp_axis x, p;
    void* workspace;
    size_t workspace_bytes;
    void* stream;
} vp_grid_desc;

/* The Hamiltonian and its pusher.
 *  FREE:      dx = p dt.
 *  SHO_EXACT: rotation of (x, p) by omega*dt; needs an open x axis.
 *  PENDULUM:  V(x) = -a cos x; drift dt/2, kick -a sin(x) dt, drift dt/2.
 *  FEL:       x = phase psi, p = energy eta, dt = dz; dpsi/dz = fel_delta + eta,
 *             deta/dz = -2 Re[(A + i fel_sigma2 <e^{-i psi}>) e^{i psi}],
 *             dA/dz = <e^{-i psi}> with <g> = N0^{-1} sum_j w_j g(psi_j) and N0 the
 *             sum of the weights when the density was set.  Drift dz/2, kick dz
 *             with the phases frozen (integrated exactly: A grows linearly
 *             through the kick), drift dz/2.  A_re, A_im give the field at the
 *             current step; vp_moments reports it as the run advances.
 *             With integrator VP_FEL_RK4 the nodes, as particles of charge w,
 *             and A are advanced by the classical Runge-Kutta method instead,
 *             each stage taking <.> over its own stage phases. */
typedef struct {
    int32_t kind;
    int32_t integrator; /* FEL only: VP_FEL_DKD or VP_FEL_RK4; 0 otherwise */
    double a;
    double omega;
    double fel_delta;
    double fel_sigma2;
    double A_re, A_im;
} vp_hamiltonian;

/* Diagnostics (Sec. "Numerical Examples": phase-space volume and entropy),
 * accumulated in FP64.  Integrals of f are exact sums (either basis):
 *  sum_w    = sum_j w_j
 *  mass     = h_x h_p sum_j w_j                      (integral of f)
 *  neg_mass = -h_x h_p sum_{w_j<0} w_j
 *  l1       = h_x h_p sum_j |w_j|
 *  entropy  = -h_x h_p sum_{w_j>0} w_j ln w_j
 *  mean_p   = sum_j w_j p_j / sum_j w_j
 *  energy   = integral of H f; exact integrals of p^2, x^2 and cos x over the
 *             basis functions (for the B-spline of degree d, tents d = 1:
 *             h^2 (d+1)/12 and sinc^(d+1)(h/2))
 *  FEL: A, bunching <e^{-i psi}> at the lattice phases, and
 *       fel_invariant = |A|^2 + N0^{-1} sum_j w_j eta_j (conserved by the step)
 *  nonfinite = number of NaN/Inf weights (the call then returns VP_ENONFINITE).
 *  The call returns VP_ERANGE (after filling *out) if, since the density was
 *  set, a deposit cell sum exceeded 2^6 x 2^e, max|w0| < 2^e: the deposit
 *  sums cells as fixed point at 2^(e-40), exact up to 2^7 x 2^e.  The
 *  transported weights of a conservative step stay near max|w0|. */
typedef struct {
    double sum_w, mass, neg_mass, l1, entropy, mean_p, energy;
    double A_re, A_im, bunch_re, bunch_im, fel_invariant;
    int64_t step;
    int64_t nonfinite;
} vp_moments_t;

/* Launch shape of the deposit kernel: destination tile (in lattice nodes) and
 * threads per workgroup (a multiple of 64, at most 1024; 768 with the cubic
 * basis).  Zero fields keep
 * the current value.  (The solve works on fixed tiles of 32 x 64 nodes, or
 * of 80 x 80 (quadratic basis) or 60 x 60 (cubic) nodes.) */
typedef struct {
    int32_t k1_tx, k1_ty;
    int32_t k1_threads;
} vp_tiles;

/* Bytes of device workspace a grid of this shape needs (0 if the axes are
 * invalid): three FP32 arrays of n_p*n_x weights (the state, ping-pong, and
 * the projection's right-hand side Delta^T w of eq. 10), the cached push map
 * (12 bytes per node, see vp_set_map_cache), per-axis push tables and small
 * per-tile buffers. */
size_t vp_workspace_bytes(const vp_axis* x, const vp_axis* p);

/* Create a grid: the fixed lattice of nodes z_j of the expansion (eq. 4) with
 * a periodic coordinate and an open momentum axis (Sec. "Numerical Examples":
 * coordinates periodic, momenta open).  desc->workspace is caller-owned device
 * memory (see vp_grid_desc); *out receives the handle.  Fails with VP_EINVAL
 * for invalid axes, VP_ENOMEM for a missing or small workspace,
 * VP_EUNSUPPORTED for a periodic p axis, VP_EHIP if the runtime fails. */
int vp_create_grid(const vp_grid_desc* desc, vp_grid** out);

/* Destroy a grid (NULL is allowed).  Waits for the grid's stream; the
 * workspace stays the caller's.  VP_ESTATE while the grid belongs to a batch. */
int vp_destroy_grid(vp_grid* g);

/* Set the Hamiltonian whose flow moves the nodes (Sec. "The Vlasov Equation as
 * Flows on Phase Space": any particle pusher; the examples of Sec. "Harmonic
 * Oscillators" and the FEL of eqs. 13a-c; kinds and pushers as listed at
 * vp_hamiltonian).  For the FEL, A_re and A_im set the current field.
 * VP_EINVAL for an unknown kind or integrator or a non-finite parameter,
 * VP_EUNSUPPORTED for the exact rotation on a periodic x axis. */
int vp_set_hamiltonian(vp_grid* g, const vp_hamiltonian* h);

/* Set the weights w_j of the expansion f = sum_j w_j Lambda_j (eq. 4): n_p*n_x
 * floats, [n_p][n_x], x fastest; a device pointer if on_device, else host
 * memory (copied before the call returns).  Records N0 = sum w (FP64, the FEL
 * normalisation of eq. 13c) and max|w| (the deposit's fixed-point exponent
 * e, max|w0| < 2^e), clears the range flag and resets the step counter.
 * VP_ENONFINITE if a weight is NaN or infinite (the grid then holds no
 * density). */
int vp_set_density(vp_grid* g, const float* w, int32_t on_device);

/* Exponent e of the deposit's fixed-point cell sums (the tile sums of
 * Delta^T w, eq. 9): taps are rounded to the grid 2^(e-40) and summed exactly
 * while a cell stays below 2^(e+7) in magnitude; beyond 2^(e+6) the range flag
 * is set.  vp_set_density picks the smallest e with max|w0| < 2^e; a caller
 * that expects the weights to grow can raise it (each unit halves the
 * resolution).  Takes effect from the next step; vp_set_density resets it.
 * VP_EINVAL for e outside [-86, 127], VP_ESTATE before a density is set or
 * while the grid belongs to a batch. */
int vp_set_fixed_point(vp_grid* g, int32_t e);

/* Choose the basis functions (VP_BASIS_TENT, VP_BASIS_QUADRATIC or
 * VP_BASIS_CUBIC; VP_EINVAL otherwise).  The weights are read as coefficients of the chosen basis from
 * the next step on; the density already set is kept as it is.  Every
 * Hamiltonian and integrator works with either basis.  A deposit tile whose
 * local memory no longer fits with the wider border of the quadratic basis
 * is replaced by the default shape.  VP_ESTATE while the grid belongs to a batch; a batch
 * takes grids of one basis (VP_EUNSUPPORTED otherwise). */
int vp_set_basis(vp_grid* g, int32_t basis);

/* The scalars that, with the weights, make up a run's state: a run stopped
 * after any step resumes bitwise on another grid of the same axes, basis and
 * Hamiltonian from vp_get_density + vp_get_run_state, then vp_set_density +
 * vp_set_run_state (checkpoint / restart).
 *  fix_exponent: the deposit's fixed-point exponent (vp_set_fixed_point);
 *  step:         the step counter;
 *  n0:           N0 of eq. 13c, the weight sum when the run started;
 *  bunch_dz:     the FEL step size the bunchings in fel[] belong to (NaN: none);
 *  fel:          the FEL field A and the current and stage bunchings (opaque). */
typedef struct {
    int32_t fix_exponent;
    int32_t reserved;
    int64_t step;
    double n0;
    double bunch_dz;
    double fel[16];
} vp_run_state;

/* Read the run state (waits for the stream).  VP_ESTATE before a density. */
int vp_get_run_state(vp_grid* g, vp_run_state* out);
/* Restore a run state after vp_set_density (which it overrides: N0, the
 * exponent, the step counter, the FEL field and bunchings).  VP_EINVAL for an
 * exponent out of range or non-finite values, VP_ESTATE before a density. */
int vp_set_run_state(vp_grid* g, const vp_run_state* s);

/* Copy the current weights w_j (eq. 4) out: n_p*n_x floats into w (device
 * memory if on_device, else host); waits for the stream.  VP_ESTATE before a
 * density is set; VP_ERANGE (after copying) if a deposit cell sum has left
 * the fixed-point range since the density was set: the weights are then not
 * valid. */
int vp_get_density(vp_grid* g, float* w, int32_t on_device);

/* Advance nsteps steps of size dt (dz for the FEL) on the grid's stream.  One
 * step is the update w_fin = Lambda^{-1} Delta^T w_in of eq. 10: every node
 * pushed by the Hamiltonian's integrator (eqs. 6-7), its basis function
 * projected back onto the lattice (eqs. 8-9), the mass-matrix system solved.
 * Returns once the work is enqueued.  VP_ESTATE if no density or Hamiltonian
 * has been set, or for the FEL if the initial weights sum to zero (N0
 * normalises the bunching, eq. 13c); VP_ERANGE, without stepping, once a
 * completed earlier step has set the range flag (see vp_set_fixed_point;
 * a step still in flight reports on a later call or in vp_moments /
 * vp_get_density); VP_EINVAL for a negative count, a non-finite dt, or a dt
 * whose drift or pendulum kick moves a node by more than 2^20 cells per step
 * (the cell arithmetic is 32-bit). */
int vp_step(vp_grid* g, double dt, int64_t nsteps);

/* Diagnostics of the current state (the list at vp_moments_t); waits for the
 * stream.  Returns VP_ENONFINITE or VP_ERANGE after filling *out when the
 * state holds NaN/Inf or the range flag is set. */
int vp_moments(vp_grid* g, vp_moments_t* out);

/* Deposit launch shape.  vp_set_tiles validates it (VP_EINVAL if the tile's
 * local memory would exceed the device limit or the thread count is not a
 * multiple of 64 in [64, 1024], [64, 768] with the cubic basis).  A new grid
 * starts from a shape chosen by its lattice size; vp_autotune picks one by
 * timing. */
int vp_set_tiles(vp_grid* g, const vp_tiles* t);
int vp_get_tiles(const vp_grid* g, vp_tiles* t);

/* For a Hamiltonian that depends neither on the state nor on the time (free,
 * rotation, pendulum) the push of every node, and so the node-to-destination
 * map and the fractions that weigh the overlaps of eq. 9, is the same every
 * step.  With the cache on it is formed once per plan into the workspace (12
 * bytes per node) and the deposit reads it instead of pushing; results are
 * bitwise the same either way.  Off by default: the deposit is bound by its
 * LDS atomics, not by the push, and the map adds 12 bytes of reads per node.
 * The FEL always pushes. */
int vp_set_map_cache(vp_grid* g, int32_t on);

/* Launch mode of vp_step: use_graph != 0 replays the per-step kernels from a
 * HIP graph of several steps; 0 launches each kernel directly ("plain"). */
int vp_set_launch(vp_grid* g, int32_t use_graph);

/* Measurement helper: nsteps steps exactly as vp_step with direct launches,
 * with HIP events recorded on the grid's stream around every kernel.
 * us[0] and us[1] receive the mean duration in microseconds of the deposit
 * kernel (for the Runge-Kutta FEL including the stage sums before it) and of
 * the solve (for the FEL including the field update that follows it).  Waits
 * for the stream. */
int vp_step_timed(vp_grid* g, double dt, int64_t nsteps, double us[2]);

/* Time candidate tile shapes on this grid for step size dt and keep the
 * fastest.  The state is restored afterwards.  best_us receives the time per
 * step of the chosen shape.  Choices are cached per shape class (kind, axis
 * lengths and largest displacement in half-octave buckets); with best_us ==
 * NULL a cached choice is applied without timing. */
int vp_autotune(vp_grid* g, double dt, double* best_us);

/* Batched execution: n grids (each with its density and Hamiltonian set)
 * advance together, one launch of each per-step kernel covering every tile of
 * every grid.  dt[i] is grid i's step size.  All grids must use the same
 * stream (VP_EINVAL otherwise); the batch uses it.  The grids must outlive the
 * batch and must not be stepped on their own while it exists (VP_ESTATE).
 * The deposit launch takes one workgroup size (the one most of the tiles were
 * planned with) and the LDS of the largest tile for every tile, so grids of
 * mixed deposit shapes run their small tiles at the occupancy of the largest:
 * give them one shape (vp_set_tiles) or let vp_batch_autotune choose one. */
int vp_batch_create(vp_grid* const* grids, int32_t n, const double* dt, vp_batch** out);
/* Time candidate launch configurations on the batch itself and keep the
 * fastest: every grid with its own deposit tile shape, or every grid with one
 * shape (64x32x256 .. 128x128x1024, cut to its lattice), each with one
 * deposit workgroup per tile or a persistent deposit (as many workgroups as
 * the device holds at once, looping over the tiles).  The grids' states are
 * restored.  best_us receives the time per batch step of the choice.  The
 * choice is cached per composition class (the multiset of kind, basis and
 * half-octave axis lengths); best_us == NULL applies a cached choice without
 * timing (VP_ESTATE if there is none). */
int vp_batch_autotune(vp_batch* b, double* best_us);
/* The batch's current launch: deposit workgroups per launch (0: one per
 * tile), threads per deposit workgroup, deposit tiles in the launch list. */
int vp_batch_config(const vp_batch* b, int32_t* deposit_grid, int32_t* deposit_threads, int32_t* tiles);
/* nsteps steps of eq. 10 for every grid of the batch, enqueued on its stream.
 * VP_ERANGE, without stepping, once a completed earlier batch step has set the
 * range flag of any of its grids (vp_moments of each grid names which). */
int vp_batch_step(vp_batch* b, int64_t nsteps);
/* Measurement helper: nsteps batch steps exactly as vp_batch_step with direct
 * launches (the batch's launch configuration), with HIP events attached to the
 * dispatches; us[0] and us[1] receive the mean duration in microseconds of
 * the batch's deposit launch and of its solve launch, as vp_step_timed.
 * Waits for the stream.  VP_EINVAL for nsteps < 1, VP_ERANGE as vp_batch_step. */
int vp_batch_step_timed(vp_batch* b, int64_t nsteps, double us[2]);
/* Release the batch (the grids stay; they can be stepped alone again). */
int vp_batch_destroy(vp_batch* b);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops and harnesses that forbid hipMalloc): the steps of vp_step on one
 * lattice given by its axes, with no grid, no workspace and no allocation of
 * any kind.  Its scratch (the right-hand side b, push tables, FEL state,
 * per-tile partials, counters, the descriptor) lives in a static device
 * array of the library (20 MiB, held on every device the library runs on
 * until the process ends): lattices of at most 2^22 nodes (VP_ENOMEM beyond).
 * Every call on a device shares that array: calls that overlap on one device
 * (other streams, other threads) race, and must be ordered by the caller.
 *  x, p, h, basis, dt, nsteps: as for vp_create_grid, vp_set_hamiltonian,
 *      vp_set_basis and vp_step (deposit tiles: the default shape);
 *  w_in:   device, n_p*n_x floats, the weights at the start (not written);
 *  w_out:  device, n_p*n_x floats, the weights after nsteps steps (may equal
 *          w_in: the step then runs in place);
 *  fel_n0: FEL only, N0 of eq. 13c (the sum of the weights when the run
 *          started; the caller keeps it across calls), nonzero;
 *  fel_A:  FEL only, device double[2], the field (re, im): read at the start,
 *          written with the field after the steps;
 *  status: optional device int32, written when the steps are done: VP_OK,
 *          VP_ENONFINITE (w_in holds NaN/Inf: nothing is deposited, w_out
 *          ends zero) or VP_ERANGE (a deposit cell left the fixed-point range
 *          set from max|w_in|, see vp_set_fixed_point);
 *  stream: hipStream_t (NULL = default) on which everything is enqueued; the
 *          call returns without waiting.
 * Argument errors return VP_EINVAL / VP_EUNSUPPORTED / VP_ESTATE as the
 * grid calls do, before anything is enqueued. */
int vp_step_noalloc(const vp_axis* x, const vp_axis* p, const vp_hamiltonian* h, int32_t basis, double dt,
                    int64_t nsteps, const float* w_in, float* w_out, double fel_n0, double* fel_A,
                    int32_t* status, void* stream);

/* ---- Four-dimensional phase space (x, y, p_x, p_y) ----
 * The method carried to 2D2V (Sec. "An Algorithm Based on Phase Space Density
 * Conservation": only Lambda and Delta change with the dimension): tents on
 * every axis, f = sum_j w_j prod_d Lambda(z_d - z_{j,d}); the overlaps of
 * eq. 9 are products of four B3 factors (a 4^4 = 256-tap deposit) and the mass
 * matrix of eq. 8 the Kronecker product of four tridiagonal ones (a line
 * solve per axis).  x and y are periodic, the momenta open (as in 2-D).
 * Weights are [n_py][n_px][n_y][n_x] floats, x fastest.  Conventions as
 * above (status codes, caller-owned workspace and stream, vp_last_error). */
typedef struct vp4_grid vp4_grid;

/* axes: x, y (periodic), p_x, p_y (open); 4 <= n <= 4096 per axis, at most
 * 2^28 nodes.  workspace: at least vp4_workspace_bytes(axes), 256-byte aligned. */
typedef struct {
    vp_axis axes[4];
    void* workspace;
    size_t workspace_bytes;
    void* stream;
} vp4_grid_desc;

/* kind VP_H_FREE: x' = p_x, y' = p_y.  kind VP_H_PENDULUM: H = |p|^2/2 + V with
 * V = -a cos x - b cos y - c cos(x - y) (c = 0: two uncoupled pendulums),
 * drift dt/2, kick dt with -grad V at the half-drift point, drift dt/2. */
typedef struct {
    int32_t kind;
    double a, b, c;
} vp4_hamiltonian;

/* FP64 sums as for vp_moments_t (cell = h_x h_y h_px h_py): energy integrates
 * H over the tent expansion (h^2/6 for p^2, sinc^2(h/2) per cos factor). */
typedef struct {
    double sum_w, mass, neg_mass, l1, entropy, mean_px, mean_py, energy;
    int64_t step;
    int64_t nonfinite;
} vp4_moments_t;

/* Bytes of device workspace for these axes (0 if invalid): three FP32 state
 * arrays, push tables, per-tile source boxes and reduction buffers. */
size_t vp4_workspace_bytes(const vp_axis axes[4]);
/* Create / destroy a 2D2V grid on the caller's workspace and stream (eq. 4's
 * lattice in four dimensions).  VP_EINVAL for invalid axes, VP_EUNSUPPORTED
 * unless x, y are periodic and the momenta open, VP_ENOMEM for a small workspace. */
int vp4_create_grid(const vp4_grid_desc* desc, vp4_grid** out);
int vp4_destroy_grid(vp4_grid* g);
/* The Hamiltonian and its pusher (see vp4_hamiltonian); VP_EINVAL otherwise. */
int vp4_set_hamiltonian(vp4_grid* g, const vp4_hamiltonian* h);
/* Deposit tile (nodes along x, y, p_x, p_y; at least 4 or the whole axis;
 * 8 bytes of LDS per node of the tile with its x rows padded by 3 nodes, plus
 * 64 bytes).  VP_EINVAL if that exceeds the device's LDS.  Results do not
 * depend on it. */
int vp4_set_tiles(vp4_grid* g, const int32_t tile[4]);
/* The current deposit tile (nodes along x, y, p_x, p_y). */
int vp4_get_tiles(const vp4_grid* g, int32_t tile[4]);
/* Set / copy out the weights of eq. 4 (device pointer if on_device, else host).
 * Set: VP_ENONFINITE for a NaN/Inf weight; records max|w| (the deposit's
 * fixed-point exponent).  Get: waits; VP_ERANGE (after copying) if a deposit
 * cell left the fixed-point range. */
int vp4_set_density(vp4_grid* g, const float* w, int32_t on_device);
int vp4_get_density(vp4_grid* g, float* w, int32_t on_device);
/* nsteps steps of eq. 10 in 2D2V on the grid's stream: push, 256-tap
 * deposit, the four line solves.  VP_ESTATE before density and Hamiltonian;
 * VP_EINVAL for a negative count, a non-finite dt, or a dt whose drift or kick
 * moves a node by more than 2^20 cells per step. */
int vp4_step(vp4_grid* g, double dt, int64_t nsteps);
/* As vp4_step, with the mean microseconds of the deposit (us[0]) and of the
 * four solves (us[1]) per step, from events recorded with the kernels. */
int vp4_step_timed(vp4_grid* g, double dt, int64_t nsteps, double us[2]);
/* Pick the deposit tile by timing: up to twelve candidate tiles (16x16x8x8
 * and smaller or flatter ones, cut to the lattice and to the device's LDS),
 * each over a few steps of size dt from the current state, which is restored
 * (with the range flag).  The fastest is kept (a candidate must beat the
 * incumbent by 2%) and best_us receives its time per step; results do not
 * depend on the choice.  The choice is cached per shape class (push kind,
 * half-octave axis lengths); best_us == NULL applies a cached choice without
 * timing (VP_ESTATE if there is none).  VP_ESTATE before density and
 * Hamiltonian. */
int vp4_autotune(vp4_grid* g, double dt, double* best_us);
/* Diagnostics (vp4_moments_t); waits.  VP_ENONFINITE / VP_ERANGE after filling *out. */
int vp4_moments(vp4_grid* g, vp4_moments_t* out);

/* Status text and the calling thread's last error message. */
const char* vp_status_string(int status);
const char* vp_last_error(void);

/* Host-side planning helper (no GPU needed): the source box a deposit tile
 * scans.  Destination tile rows [by0,by1) and columns [bx0,bx1) of a grid with
 * axes x, p and basis functions `basis` under Hamiltonian h, step dt and
 * (FEL) kick field kick_re + i kick_im.  box[4] receives [x0, x1, y0, y1):
 * unwrapped source columns and source rows.  Every node whose pushed position
 * deposits into the tile lies in the box. */
int vp_plan_source_box(const vp_axis* x, const vp_axis* p, const vp_hamiltonian* h, int32_t basis,
                       double dt, double kick_re, double kick_im, int32_t bx0, int32_t bx1,
                       int32_t by0, int32_t by1, int32_t box[4]);

/* Host-side planning helper of the 2D2V deposit (no GPU needed): the source
 * box of the destination tile [tile_lo[d], tile_hi[d]) on every axis d (x, y,
 * p_x, p_y) under Hamiltonian h and step dt.  box[2d], box[2d+1] receive the
 * source range [lo, hi) along axis d: on x and y lo is in [0, n) and the range
 * holds at most n columns, taken modulo n; an empty range has lo = hi.  Every
 * node whose moved tent (first tap at floor of its pushed cell position, less
 * one) deposits into the tile lies in the box (the tent reach of the
 * algorithm section's overlap, eq. 9, per axis).  VP_EINVAL for invalid axes,
 * a tile outside them, an unknown kind or non-finite parameters. */
int vp4_plan_source_box(const vp_axis axes[4], const vp4_hamiltonian* h, double dt, const int32_t tile_lo[4],
                        const int32_t tile_hi[4], int32_t box[8]);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
