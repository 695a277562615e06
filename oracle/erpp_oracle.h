/*
 * erpp_oracle.h -- plain FP64 CPU reference of the ERPP particle/fluid coupling
 * step (Gualtieri, Picano, Sardina & Casciola, "Exact regularized point particle
 * method for multi-phase flows in the two-way coupling regime", arXiv:1405.6969).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker the GPU path is
 * compared against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the product path never links or calls it.
 *
 * It shares no code, header or constant with the HIP library: all types below
 * are its own.
 *
 * Layouts (all arrays caller-owned, host memory):
 *   grid fields  [3][Nz][Ny][Nx]  (x fastest), nodes at x_i = i*dx, dx = L/N
 *   particles    [3][np]          structure of arrays
 *   ring         [M+1][3][np]     slot l mod (M+1) holds level l
 */
#ifndef ERPP_ORACLE_H
#define ERPP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n[3];        /* nodes per dimension */
    double  L[3];        /* box lengths */
    int64_t np;          /* particles */
    double  m_p;         /* particle mass */
    double  rho_f;       /* fluid density */
    double  nu;          /* kinematic viscosity */
    double  sigma;       /* regularisation width sigma_R */
    double  cutoff;      /* stencil radius in units of sigma (3) */
    double  shear;       /* mean shear rate S; U_x = S (y - Ly/2); 0 = none */
    int32_t M;           /* delay eps_R = M dt, in steps (>= 1) */
    double  dt;          /* time step */
    int32_t self_correction; /* 1: remove the closed-form self disturbance */
    double  g[3];        /* body acceleration of the particles, (m_p - m_f) g / m_p */
    int32_t integrator;  /* 0 explicit Euler, 1 exact linear drag over the step,
                            2 Heun (two stages, self term removed at each) */
    double  a_p;         /* particle radius of the Faxen term (a_p^2/6) lap u~; 0 = off */
    double  a_am;        /* particle radius of the added-mass terms (displaced mass
                            m_f = rho_f 4/3 pi a_am^3, Faxen part a_am^2/10); 0 = off */
    double  a_b;         /* particle radius of the Basset term (coefficient 6 pi mu a_b^2,
                            Faxen part a_b^2/6); 0 = off */
} oracle_params;

/* Cell key of each position and a stable counting sort by key.
 * key[p] = (k*Ny + j)*Nx + i, cell_start[Nc+1], perm[np]. */
void oracle_bin(const oracle_params *P, const double *x, int32_t *key,
                int32_t *cell_start, int32_t *perm);

/* Delayed Gaussian forcing from positions X and drags D (one ring level).
 * Writes f (acceleration) on the node window [lo, lo+wn) (periodic), layout
 * [3][wn_z][wn_y][wn_x]; the window may be the whole grid.  f is overwritten. */
void oracle_deposit(const oracle_params *P, const double *X, const double *D,
                    const int32_t lo[3], const int32_t wn[3], double *f);

/* Per-particle normalisation Z = dV * sum over the stencil of the raw weight. */
void oracle_normalisation(const oracle_params *P, const double *X, double *Z);

/* Closed-form self-induced disturbance at x from the injection made one step
 * earlier at (Xp, Dp): App. E, with width sigma_s^2 = sigma^2 + 2 nu dt. */
void oracle_self_disturbance(const oracle_params *P, const double *x,
                             const double *Xp, const double *Dp, double *vs);

/* Laplacian of the closed-form self-disturbance at x (same arguments as
 * oracle_self_disturbance): the Faxen term's self part. */
void oracle_self_laplacian(const oracle_params *P, const double *x,
                           const double *Xp, const double *Dp, double *ls);

/* Gradient of the closed-form self-disturbance at x (same arguments as
 * oracle_self_disturbance): gs[(3 c + j) np + p] = d v_c / d x_j. */
void oracle_self_gradient(const oracle_params *P, const double *x,
                          const double *Xp, const double *Dp, double *gs);

/* Trilinear interpolation at x of the central-difference nodal gradient of u,
 * plus the mean shear's d U_x / d y = S: gu[(3 c + j) np + p] = d u_c / d x_j. */
void oracle_grid_gradient(const oracle_params *P, const double *u, const double *x,
                          double *gu);

/* Trilinear interpolation at x of the 7-point nodal Laplacian of u. */
void oracle_grid_laplacian(const oracle_params *P, const double *u, const double *x,
                           double *lu);

/* Trilinear interpolation of the carrier u at x plus the mean shear. */
void oracle_gather(const oracle_params *P, const double *u, const double *x,
                   double *up);

/* One coupling step n: forcing f (on the window, NULL to skip), drag D^n into
 * ring slot n mod (M+1), and x^n, v^n -> x^{n+1}, v^{n+1} in place.
 * dout (optional, [3][np]) receives D^n.  With a_am > 0, am_hist ([6][np]:
 * u~ and u~ + (a_am^2/10) lap u~ of the previous step) and *am_valid (0 before
 * the first step with added mass) carry the added-mass history; with a_b > 0,
 * bs_hist ([3][np]: u~ + (a_b^2/6) lap u~ - v of the previous step) and
 * *bs_valid the Basset history; otherwise they may be NULL. */
void oracle_step(const oracle_params *P, int64_t n, const double *u,
                 double *x, double *v, const float *tau, double *ring_x,
                 double *ring_d, const int32_t lo[3], const int32_t wn[3],
                 double *f, double *dout, double *am_hist, int32_t *am_valid,
                 double *bs_hist, int32_t *bs_valid);

#ifdef __cplusplus
}
#endif
#endif
