/*
 * erpp.h -- C ABI of the MI355X (gfx950) ERPP particle/fluid momentum-coupling
 * step.
 *
 * Method: Gualtieri, Picano, Sardina & Casciola, "Exact regularized point
 * particle method for multi-phase flows in the two-way coupling regime",
 * arXiv:1405.6969.  One coupling step n of every box does, in order:
 *
 *   1. bin      -- sort the particles whose drag is being injected by grid cell
 *                  (locality structure for the scatter; not in the paper);
 *   2. evaluate -- for each particle read the history ring at level n-M
 *                  (position and drag delayed by eps_R = M dt, Sec. 2.3,
 *                  eq. velo_reg_eq) and form the normalised Gaussian amplitude;
 *                  read level n-1-M for the closed-form self-disturbance of
 *                  App. E (eq. disturbance_velo);
 *   3. scatter  -- forcing on the grid, -(1/rho_f) sum_p D_p(t-eps_R)
 *                  g[x - x_p(t-eps_R), eps_R] (Sec. 2.4,
 *                  eq. ns_regularized_filtered), g cut at |x - x_p| <= 3 sigma_R
 *                  (Sec. 3.2) and normalised per particle on the lattice;
 *   4. gather   -- carrier velocity at each particle by trilinear interpolation
 *                  (plus an optional analytic mean shear S (y - Ly/2) e_x);
 *   5. update   -- Stokes drag D = m_p (u~ - v)/tau_p with u~ the carrier minus
 *                  the self-disturbance (Sec. 2.5, eqs. force_stokes_drag and
 *                  particle_motion), stored in ring slot n mod (M+1) with x^n,
 *                  then explicit Euler x^{n+1} = x^n + dt v^n,
 *                  v^{n+1} = v^n + dt D/m_p, periodic wrap.
 *
 * Readings of the paper used throughout: sigma_R is given directly; the delay
 * is eps_R = M dt; the self-disturbance width is sigma_s^2 = sigma_R^2 + 2 nu dt
 * (App. E: sigma^2 = 2 nu (eps_R + dt)); its -dt/rho_f prefactor (App. E,
 * eqs. forcing_step and pseudo_velo_num) is kept; levels before t = 0 carry no
 * drag (f = 0 for n < M, no self term for n <= M).
 *
 * Conventions
 *   - Every pointer in erpp_box is DEVICE memory owned by the caller; the
 *     library never frees or reallocates it.  The plan owns only its scratch.
 *   - Layouts: grid fields [3][Nz][Ny][Nx] (x fastest), nodes at x_i = i L/N;
 *     particle arrays [3][np] (structure of arrays); rings [M+1][3][np].
 *   - Precision ERPP_F64_PLAIN: u, f, ring_d are double; every stage in FP64.
 *     Precision ERPP_F32_FAST: u, f, ring_d are float; kernel evaluation and
 *     grid accumulation in FP32, cell indices, positions, velocities and the
 *     drag in FP64.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on it; errors from earlier asynchronous work surface at a
 *     later call or at erpp_plan_destroy.
 *   - No C++ exception crosses this ABI.  Every call validates its arguments
 *     before it launches anything; on error nothing is launched and
 *     erpp_last_error() describes the problem (thread-local string).
 */
#ifndef ERPP_H
#define ERPP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ERPP_OK = 0,
    ERPP_EINVAL = -1,       /* NULL pointer, np < 0, M < 1, dt <= 0, bad index ... */
    ERPP_ENOMEM = -2,       /* device allocation of plan scratch failed           */
    ERPP_EHIP = -3,         /* a HIP runtime call failed                          */
    ERPP_EGEOM = -4,        /* grid too small for the stencil (N < 2 R_c + 2),
                               L <= 0, sigma <= 0 or cutoff <= 0, or a sphere of
                               radius cutoff*sigma that can miss every node
                               (cutoff*sigma < half the cell diagonal)            */
    ERPP_EUNSUPPORTED = -5  /* outside the library's limits (a dimension > 2048 in
                               x/y or > 1024 in z, more than 2^31-1 particles or
                               nodes per box)                                     */
} erpp_status;

typedef enum {
    ERPP_F64_PLAIN = 0,     /* plain FP64 path (global FP64 atomics, no binning)  */
    ERPP_F32_FAST = 1       /* binned, LDS-tiled FP32 scatter, FP64 integration   */
} erpp_precision;

/* One periodic box.  All pointers: device memory, caller-owned. */
typedef struct {
    int32_t n[3];           /* grid nodes Nx, Ny, Nz                               */
    double  L[3];           /* box lengths                                         */
    int64_t np;             /* particles (0 allowed)                               */
    double *x;              /* [3][np] positions in/out: x^n -> x^{n+1}, in [0,L)  */
    double *v;              /* [3][np] velocities in/out: v^n -> v^{n+1}           */
    double *ring_x;         /* [M+1][3][np] history of positions                   */
    void   *ring_d;         /* [M+1][3][np] history of drags (float or double)     */
    const float *tau;       /* [np] Stokes times tau_p                             */
    const void  *u;         /* [3][Nz][Ny][Nx] carrier velocity (float or double)  */
    void   *f;              /* [3][Nz][Ny][Nx] forcing output, acceleration
                               (float or double); fully overwritten by a scatter   */
    double  m_p;            /* particle mass                                       */
    double  rho_f;          /* fluid density                                       */
    double  nu;             /* kinematic viscosity (self-disturbance width)        */
    double  sigma;          /* regularisation width sigma_R                        */
    double  cutoff;         /* stencil radius in units of sigma_R (3)              */
    double  shear;          /* mean shear S, U_x = S (y - Ly/2); 0 = none.  A
                               particle crossing y = 0 / Ly gets v_x -/+= S Ly     */
} erpp_box;

typedef enum {
    ERPP_EULER = 0,         /* explicit Euler (Sec. 2.5): D^n = m_p (u~ - v^n)/tau_p,
                               v^{n+1} = v^n + dt D^n/m_p + dt g_b,
                               x^{n+1} = x^n + dt v^n                              */
    ERPP_EXPONENTIAL = 1,   /* the linear drag ODE solved exactly over the step with
                               u~ frozen: w = u~ + tau_p g_b,
                               v^{n+1} = w + (v^n - w) e^{-dt/tau_p},
                               x^{n+1} = x^n + dt w + tau_p (v^n - w)(1 - e^{-dt/tau_p});
                               drag handed to the fluid: the step average
                               m_p (v^{n+1} - v^n)/dt - m_p g_b.  Stable for any
                               dt/tau_p                                            */
    ERPP_HEUN = 2           /* two-stage Runge-Kutta (Heun) with the App. E self term
                               removed at each stage (Sec. 2.5): a_1 from u~(x^n),
                               v* = v^n + dt a_1, a_2 from u~(x*) at
                               x* = x^n + dt v^n, v^{n+1} = v^n + dt (a_1 + a_2)/2,
                               x^{n+1} = x^n + dt (v^n + v*)/2; the fluid receives
                               the mean of the two stage drags.  Boxes without
                               mean shear only                                     */
} erpp_integrator;

typedef struct erpp_plan erpp_plan;   /* opaque: copies of the boxes, scratch,
                                         tile shape, captured graph            */

/* Create a plan for `nbox` boxes (copied; the pointers inside must stay valid
 * for the plan's lifetime).  M >= 1 is the delay in steps (eps_R = M dt),
 * self_correction 1 removes the self-disturbance (App. E), 0 keeps it.
 * Allocates the plan's scratch on the current device.  Returns ERPP_EINVAL,
 * ERPP_EGEOM, ERPP_EUNSUPPORTED or ERPP_ENOMEM without creating anything. */
erpp_status erpp_plan_create(erpp_plan **plan, const erpp_box *boxes, int32_t nbox,
                             int32_t M, double dt, erpp_precision precision,
                             int32_t self_correction, void *stream);

/* Scatter decomposition of an ERPP_F32_FAST plan: one workgroup owns a pencil,
 * all Nx nodes of tile[1] x tile[2] grid rows (y, z).  tile[0] is the number of
 * threads per scatter workgroup, 512 or 1024 (0 selects 512); tile[1] in
 * [1, 64], tile[2] in [1, 8].  Per box the pencil is clipped so that a stencil
 * never wraps onto it twice.  The LDS copy of the pencil (12 bytes per node,
 * rows unwrapped by the stencil width) plus the window's record table must fit
 * 150 KiB for every box of the plan; otherwise ERPP_EINVAL and the plan keeps
 * its shape.  Invalidates a captured graph. */
erpp_status erpp_plan_set_tile(erpp_plan *plan, const int32_t tile[3]);
erpp_status erpp_plan_get_tile(const erpp_plan *plan, int32_t tile[3]);

/* Work item of the ERPP_F32_FAST scatter: one lane deposits `rows` consecutive
 * stencil rows (dy, one dz) of one particle, so a wavefront pass covers 64
 * particles and 64 rows times `rows`: fewer rows per item, more particles per
 * wavefront for the same rows.  rows in [2, 4] (default 3), else ERPP_EINVAL.
 * The forcing does not depend on it (exact integer sums).  Invalidates a
 * captured graph.  Accepted and ignored on ERPP_F64_PLAIN plans. */
erpp_status erpp_plan_set_rows_per_item(erpp_plan *plan, int32_t rows);
erpp_status erpp_plan_get_rows_per_item(const erpp_plan *plan, int32_t *rows);

/* Body acceleration of the particles of box `ibox`, (m_p - m_f) g / m_p
 * (Sec. 2.5, eq. particle_motion: gravity acts on the particle minus its
 * displaced fluid mass).  It enters the velocity update only,
 * v^{n+1} = v^n + dt D^n/m_p + dt g_b; the fluid receives the hydrodynamic drag
 * D alone.  Default 0.  Applies to later steps, also to captured graphs (the
 * value lives in the plan's device copy of the box).  Synchronises the device.
 * ERPP_EINVAL for a bad plan or index or a non-finite component. */
erpp_status erpp_plan_set_body_force(erpp_plan *plan, int32_t ibox, const double g[3]);

/* Faxen correction of the drag of box `ibox` (eq. force_particle, first line):
 * D = m_p (u~ + (a_p^2/6) lap u~ - v)/tau_p with a_p the particle radius
 * (0, the default, turns it off).  lap u~ = the trilinear interpolation of the
 * 7-point nodal Laplacian of the carrier minus the Laplacian of the closed-form
 * self-disturbance (the projected Gaussian's second derivatives).  The added
 * mass is set by erpp_plan_set_added_mass, the Basset history force by
 * erpp_plan_set_basset.  Synchronises the device and invalidates captured graphs.
 * ERPP_EINVAL for a bad plan, index or radius. */
erpp_status erpp_plan_set_faxen(erpp_plan *plan, int32_t ibox, double a_p);

/* Added-mass terms of box `ibox` (eq. force_particle, second line) for
 * particles of radius a (0, the default, turns them off): displaced mass
 * m_f = rho_f (4/3) pi a^3, and with u~ the carrier without the particle's own
 * disturbance (its value, Laplacian and gradient at the particle each minus
 * the closed form of the last injection's disturbance), the explicit Euler step
 *   (m_p + m_f/2) (v^{n+1} - v^n)/dt = S + m_f Du~/Dt + (m_f/2) dq/dt + m_p g_b,
 *   S = m_p (u~ + (a_p^2/6) lap u~ - v^n)/tau_p   (a_p: erpp_plan_set_faxen),
 *   q = u~ + (a^2/10) lap u~,
 *   dq/dt = (q^n - q^{n-1})/dt along the particle path, likewise du~/dt,
 *   Du~/Dt = du~/dt + (u~ - v^n) . grad u~   (grad u~: trilinear interpolation
 *            of the central-difference nodal gradient minus the closed form's),
 * and the fluid receives the hydrodynamic force D = m_p (v^{n+1} - v^n)/dt -
 * m_p g_b.  The path derivatives are zero on the first step after this call.
 * hist: device, [6][np] FP64, caller-owned and left allocated while the terms
 * are on: u~ and q of the last step, written by every update (its contents on
 * entry are not read).  Explicit Euler only, boxes without mean shear only.
 * Synchronises the device and invalidates captured graphs.  ERPP_EINVAL for a
 * bad plan, index, radius or a NULL hist; ERPP_EUNSUPPORTED for another
 * integrator or a sheared box. */
erpp_status erpp_plan_set_added_mass(erpp_plan *plan, int32_t ibox, double a, double *hist);

/* Basset history force of box `ibox` (eq. force_particle, third line) for
 * particles of radius a (0, the default, turns it off).  The coupled field
 * already carries the vorticity the particle produced before the current step,
 * so the memory integral covers the last step only (Sec. 2.5, closing
 * paragraph); with the bracket w = u~ + (a^2/6) lap u~ - v changing at the
 * rate (w^n - w^{n-1})/dt over that step,
 *   B^n = 6 pi mu a^2 int_{t-dt}^{t} [pi nu (t - s)]^{-1/2} ds (w^n - w^{n-1})/dt
 *       = 12 pi mu a^2 (w^n - w^{n-1}) / sqrt(pi nu dt),
 * mu = rho_f nu of the box, u~ and lap u~ as for the Faxen and added-mass
 * terms (self-disturbance of the last injection removed).  Explicit Euler:
 *   (m_p + m_f/2) (v^{n+1} - v^n)/dt = S + [added-mass terms] + B^n + m_p g_b
 * (m_f = 0 without added mass), and the fluid receives the hydrodynamic force
 * D = S + [added-mass terms] + B^n = m_p (v^{n+1} - v^n)/dt - m_p g_b.
 * B = 0 on the first step after this call (no previous w).  hist: device,
 * [3][np] FP64, caller-owned and left allocated while the term is on: w of the
 * last step, written by every update (its contents on entry are not read).
 * Explicit Euler only, boxes without mean shear only.  Synchronises the device
 * and invalidates captured graphs.  ERPP_EINVAL for a bad plan, index, radius,
 * nu or a NULL hist; ERPP_EUNSUPPORTED for another integrator or a sheared box. */
erpp_status erpp_plan_set_basset(erpp_plan *plan, int32_t ibox, double a, double *hist);

/* Particle integrator of every box (default ERPP_EULER).  The self-disturbance
 * removed from u~ is the same App. E closed form for all three (the fluid
 * receives one forcing step of the handed-over drag in each; Heun removes it at
 * each stage's position).  Applies to later steps; invalidates captured graphs.
 * Synchronises the device.  ERPP_EINVAL for a bad plan or kind;
 * ERPP_EUNSUPPORTED for Heun while a box has a mean shear, or for another
 * integrator than Euler while a box has the added-mass or Basset terms on. */
erpp_status erpp_plan_set_integrator(erpp_plan *plan, erpp_integrator kind);

/* Autotuner (ERPP_F32_FAST): times every candidate pencil shape on the plan's own
 * boxes (a fixed table plus the balanced heights of the tallest box: its y extent
 * split into the fewest equal pencils that fit the LDS, and into one more) with
 * the scatter of step n, the step following the last one run (the
 * ring, positions and velocities are only read) and keeps the fastest; then, at
 * that pencil, the rows per work item (erpp_plan_set_rows_per_item).
 * Afterwards the step counter is n again and every box's f holds the forcing of
 * step n, which the next erpp_step(n) writes again.  With cache_path != NULL the
 * choice is read from / appended to that text file, keyed by the geometry; a
 * hit skips the timing.  Synchronises `stream`.  ERPP_EINVAL when fewer than M
 * steps have run and the cache has no entry (the scatter of step n reads ring
 * level n - M).  On ERPP_F64_PLAIN plans it is a no-op. */
erpp_status erpp_plan_tune(erpp_plan *plan, const char *cache_path, void *stream);

/* Number of bins of box `ibox` for erpp_bin: its grid cells, Nx * Ny * Nz. */
erpp_status erpp_plan_bins(const erpp_plan *plan, int32_t ibox, int32_t *nbin);

/* Bin `pos` ([3][np] device FP64 positions of box ibox, e.g. x^n or a ring
 * level) by grid cell (stage 1).  The binning is a locality structure of this
 * library, not a step of the paper; its cell rule follows the grid the forcing
 * lives on (nodes at i dx, dx = L/N): key[p] = (k Ny + j) Nx + i is the cell of
 * the wrapped position (i = min(floor(x/dx), N-1), per dimension);
 * bin_start[0..ncell] is the exclusive scan of the cell counts and perm lists
 * the particles grouped by cell in ascending key order (order inside a cell
 * unspecified).  key, perm, bin_start: device, caller-owned, sizes np, np,
 * ncell+1. */
erpp_status erpp_bin(erpp_plan *plan, int32_t ibox, const double *pos, int32_t *key,
                     int32_t *perm, int32_t *bin_start, void *stream);

/* erpp_bin for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * binning of np positions of one box of n[0] x n[1] x n[2] cells and lengths L
 * (host arrays), with no plan.  It allocates nothing: its scratch (cell
 * histogram, ranks, scan partials) is a static device array of the library,
 * one copy per GPU (about 16.8 MB, held until the process ends), found on the
 * first call on each device, which must be the current device.  Limits:
 * n[0] n[1] n[2] <= 2^21 cells and np <= 2^21 particles, else ERPP_EINVAL with
 * nothing launched.  pos, key, perm, bin_start: device, caller-owned, sizes
 * [3][np], np, np, ncell + 1, with the layout and results of erpp_bin.  Every
 * call on a GPU uses that GPU's one scratch array: calls that overlap on one GPU
 * (other streams, other host threads) race and must be ordered by the caller.
 * Asynchronous on `stream` (a stream of the current device). */
erpp_status erpp_bin_static(const int32_t n[3], const double L[3], int64_t np, const double *pos,
                            int32_t *key, int32_t *perm, int32_t *bin_start, void *stream);

/* Stages 1-3 for every box: write f for step `step` from ring level step-M
 * (f = 0 when step < M).  f is the regularised forcing of Sec. 2.4 (eq.
 * ns_regularized_filtered): each particle's drag of M steps earlier (Sec. 2.3,
 * the delay eps_R = M dt), spread as -D/(rho_f) times the Gaussian of width
 * sigma_R cut at 3 sigma (Sec. 3.2), normalised per particle over the nodes it
 * covers so that rho_f dV sum(f) = -sum(D).  f: [3][Nz][Ny][Nx] FP32 (fast) or
 * FP64 (plain) device array of each box, overwritten.  The ring is only read.
 * Errors: ERPP_EINVAL for a NULL plan or step < 0; ERPP_EHIP on a launch
 * failure. */
erpp_status erpp_scatter(erpp_plan *plan, int64_t step, void *stream);

/* Stage 4 for every box: the carrier at the particle (Sec. 2.5, the fluid
 * velocity in the drag of eq. force_stokes_drag), u_p = trilinear(u, x) +
 * S (y - Ly/2) e_x at the current positions x, FP64, [3][np] per box, boxes
 * concatenated in plan order (device, caller-owned).  Errors: ERPP_EINVAL for a
 * NULL plan or u_p (with particles); ERPP_EHIP on a launch failure. */
erpp_status erpp_gather(erpp_plan *plan, double *u_p, void *stream);

/* Stages 1-5 for every box: one coupling step n = step.  The forcing of
 * erpp_scatter, then per particle the drag of Sec. 2.5 (eq. force_stokes_drag,
 * with the particle's own disturbance, App. E eq. disturbance_velo from the
 * injection of level n-1-M, removed from the carrier), the ring write of (x^n,
 * D^n) at slot n mod (M+1), and the step of eq. particle_motion (explicit Euler
 * unless erpp_plan_set_integrator chose otherwise), with periodic wrap.  x, v,
 * the ring and f of every box are updated in place.  Errors: ERPP_EINVAL for a
 * NULL plan or step < 0; ERPP_EHIP on a launch failure. */
erpp_status erpp_step(erpp_plan *plan, int64_t step, void *stream);

/* Steps step0 .. step0+nsteps-1.  use_graph = 1 captures the step once in a
 * HIP graph (step index kept in device memory) and replays it. */
erpp_status erpp_run(erpp_plan *plan, int64_t step0, int64_t nsteps, int32_t use_graph,
                     void *stream);

/* Measurement: run steps step0 .. step0+nsteps-1 (nsteps >= 1) stage by stage
 * without a graph, with a HIP event recorded on `stream` after every stage, and
 * return in ms[k] the average duration (milliseconds) of stage k:
 *   ERPP_F32_FAST:  0 tile histogram, 1 scan, 2 evaluate, 3 tiled scatter,
 *                   4 gather + self term + update;
 *   ERPP_F64_PLAIN: 0 zero the forcing, 1 (nothing), 2 evaluate,
 *                   3 atomic scatter, 4 gather + self term + update.
 * The steps are real steps (particles advance).  Synchronises `stream`. */
erpp_status erpp_stage_times(erpp_plan *plan, int64_t step0, int64_t nsteps, double ms[5],
                             void *stream);

/* Release the plan's scratch and graph.  NULL-safe.  Synchronises the device. */
void erpp_plan_destroy(erpp_plan *plan);

/* ---------------------------------------------------------------------------
 * Fluid step: the periodic unsteady-Stokes equation of the disturbance
 * (Sec. 2.3, eq. velo_reg_eq) advanced over dt by the splitting of App. E:
 *
 *   forcing step    (eq. forcing_step)    u~ = u + dt f
 *   diffusion step  (eq. diffusion_step)  u* = u~ convolved with g(., dt):
 *                                         Fourier mode k times exp(-nu |k|^2 dt)
 *   projection step                       lap(phi) = -div(u*), u = u* + grad(phi)
 *
 * done pseudo-spectrally with hipFFT on the grid of a box (nodes x_i = i L/N,
 * k = 2 pi m / L).  The mean mode is kept, so rho_f * sum(u) dV grows by
 * exactly rho_f * dt * sum(f) dV: the total impulse of Sec. 3.1.  Nyquist
 * index of an even N: the projection's derivatives (div, grad) take that
 * wavenumber component as zero (the grid derivative of (-1)^j vanishes at
 * every node); the diffusion keeps the full |k|^2.  With f the
 * forcing of erpp_scatter/erpp_step this closes the two-way coupling loop for
 * boxes without mean shear (shear needs a deforming-frame transform, not
 * provided).
 * --------------------------------------------------------------------------- */
typedef struct erpp_fluid erpp_fluid;   /* opaque: FFT plans, spectral buffer */

/* Create a fluid stepper for an Nx x Ny x Nz grid of box lengths L, kinematic
 * viscosity nu >= 0 and step dt > 0.  precision ERPP_F32_FAST: u and f float,
 * FP32 transforms; ERPP_F64_PLAIN: double, FP64 transforms.  Allocates the
 * spectral buffer (3 Nz Ny (Nx/2+1) complex) and the FFT plans on the current
 * device; `stream` is the stream of later calls (may be changed per call).
 * ERPP_EINVAL for a NULL out pointer, bad nu/dt/precision; ERPP_EGEOM for
 * N < 1 or L <= 0; ERPP_EUNSUPPORTED beyond 4096 nodes per dimension or
 * 3 N^3 > 2^31-1 values; ERPP_ENOMEM / ERPP_EHIP when allocation or an FFT plan
 * fails. */
erpp_status erpp_fluid_create(erpp_fluid **fluid, const int32_t n[3], const double L[3],
                              double nu, double dt, erpp_precision precision, void *stream);

/* One step in place: u <- P exp(nu dt lap) (u + dt f).  u, f: device
 * [3][Nz][Ny][Nx] of the stepper's precision, caller-owned, not aliased; f is
 * only read.  Asynchronous on `stream`. */
erpp_status erpp_fluid_step(erpp_fluid *fluid, void *u, const void *f, void *stream);

/* Release the FFT plans and the spectral buffer.  NULL-safe.  Synchronises the
 * device. */
void erpp_fluid_destroy(erpp_fluid *fluid);

/* Two-way coupled steps step0 .. step0+nsteps-1: each step runs stages 1-5 of
 * every box (erpp_step), then fluids[b] advances box b's carrier in place with
 * that step's forcing, u_b <- P exp(nu dt lap)(u_b + dt f_b), so the next step
 * gathers the disturbed fluid.  The plan's `u` pointers are written here (the
 * coupling stages themselves only read them).  fluids[b] must match box b: same
 * grid and lengths, the plan's precision and dt, the box's nu (the
 * self-disturbance removed by the update is what this fluid step makes of one
 * forcing step, App. E), and shear = 0; otherwise ERPP_EINVAL and nothing runs.
 * use_graph = 1 captures one coupled step in a HIP graph (recaptured when the
 * fluids change) and replays it. */
erpp_status erpp_run_coupled(erpp_plan *plan, erpp_fluid *const *fluids, int64_t step0,
                             int64_t nsteps, int32_t use_graph, void *stream);

const char *erpp_status_string(erpp_status status);
const char *erpp_last_error(void);   /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* ERPP_H */
