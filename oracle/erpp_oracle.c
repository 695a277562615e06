/*
 * erpp_oracle.c -- plain FP64 CPU reference ("oracle") of one ERPP
 * particle/fluid momentum-coupling step, arXiv:1405.6969.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.
 *
 * Written for readability, not speed: every stage is the paper's definition in
 * straight loops, in double precision, summed in particle-index order.  Built
 * with -ffp-contract=off so that each floating-point operation is rounded as
 * written.
 *
 * What is computed (paper passages in brackets):
 *   - forcing on the fluid: minus the drag of each particle, delayed by
 *     eps_R = M dt, spread with the diffusion kernel of width sigma_R around the
 *     delayed position [Sec. 2.4, eq. ns_regularized_filtered; Sec. 2.3,
 *     eq. velo_reg_eq; the kernel g is eq. fundamental_fourier / App. A];
 *     the kernel is cut at 3 sigma_R [Sec. 3.2, the 3 sigma_R inner cut-off]
 *     and renormalised per particle so that the forcing carries exactly the
 *     delayed drag (momentum balance, Sec. 1);
 *   - the self-induced disturbance of the previous step's injection, removed
 *     from the fluid velocity seen by the particle [Sec. 2.5 and App. E,
 *     eq. disturbance_velo];
 *   - the Stokes drag D = m_p (u~ - v) / tau_p and explicit Euler motion
 *     [Sec. 2.5, eqs. particle_motion and force_stokes_drag; Sec. 3.2,
 *     eq. Drag_one_way with tau_p];
 *   - optionally the other lines of the general force [Sec. 2.5,
 *     eq. force_particle]: the Faxen terms, the added mass and the Basset
 *     term, whose memory integral covers the last step only (Sec. 2.5, closing
 *     paragraph), each with the self-disturbance removed.
 *
 * Readings where the paper leaves a choice (they are the same on the GPU):
 *   - sigma_R is given directly (a multiple of the grid spacing) and the delay
 *     is eps_R = M dt; the self-disturbance width is sigma_s^2 = sigma_R^2 +
 *     2 nu dt, i.e. 2 nu (eps_R + dt) of App. E;
 *   - the prefactor -dt/rho_f of the forcing and pseudo-velocity steps of
 *     App. E is carried into the closed form of eq. disturbance_velo;
 *   - the forcing at step n uses ring level n-M, the self-disturbance at step n
 *     uses level n-1-M; missing levels (n < M, n <= M) contribute nothing
 *     (Sec. 2: negative delayed times are harmless, the history starts at 0);
 *   - stencil = nodes within the sphere |x_c - X| <= 3 sigma_R (inclusive);
 *   - nodes at x_i = i L/N; interpolation of the carrier is trilinear;
 *   - positions advance with the old velocity (explicit Euler);
 *   - with a mean shear U_x = S (y - Ly/2) the grid holds the fluctuation; a
 *     particle crossing the y boundary has its x velocity shifted by -/+ S Ly.
 */
#include "erpp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double ORACLE_PI = 3.14159265358979323846;

/* x mapped into [0, L) */
static double wrap_coord(double x, double L)
{
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y = 0.0;
    return y;
}

static int64_t imod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* cell index b and fractional offset phi of a coordinate (nodes at i*dx) */
static void cell_of(double x, double L, int32_t N, int32_t *b, double *phi)
{
    double dx = L / (double)N;
    double xh = wrap_coord(x, L);
    double s = xh / dx;
    double fb = floor(s);
    int32_t i = (int32_t)fb;
    if (i > N - 1) i = N - 1;
    if (i < 0) i = 0;
    *b = i;
    *phi = s - (double)i;
}

static int32_t stencil_radius(const oracle_params *P, int d)
{
    double dx = P->L[d] / (double)P->n[d];
    return (int32_t)ceil(P->cutoff * P->sigma / dx);
}

/* ------------------------------------------------------------------ bin --- */

void oracle_bin(const oracle_params *P, const double *x, int32_t *key,
                int32_t *cell_start, int32_t *perm)
{
    const int64_t np = P->np;
    const int64_t nc = (int64_t)P->n[0] * P->n[1] * P->n[2];
    int64_t p, c;
    for (p = 0; p < np; ++p) {
        int32_t b[3];
        double phi;
        int d;
        for (d = 0; d < 3; ++d) cell_of(x[d * np + p], P->L[d], P->n[d], &b[d], &phi);
        key[p] = (int32_t)(((int64_t)b[2] * P->n[1] + b[1]) * P->n[0] + b[0]);
    }
    for (c = 0; c <= nc; ++c) cell_start[c] = 0;
    for (p = 0; p < np; ++p) cell_start[key[p] + 1] += 1;
    for (c = 0; c < nc; ++c) cell_start[c + 1] += cell_start[c];
    {
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
        for (c = 0; c < nc; ++c) fill[c] = cell_start[c];
        for (p = 0; p < np; ++p) perm[fill[key[p]]++] = (int32_t)p;
        free(fill);
    }
}

/* -------------------------------------------------------------- deposit --- */

/* Offsets d = (m - phi) dx of the stencil nodes b+m, m in [-R, R+1], per dim. */
typedef struct {
    int32_t b[3];
    double phi[3];
    int32_t R[3];
    double dx[3];
} stencil_t;

static void stencil_of(const oracle_params *P, const double *X, int64_t p,
                       stencil_t *s)
{
    int d;
    for (d = 0; d < 3; ++d) {
        cell_of(X[d * P->np + p], P->L[d], P->n[d], &s->b[d], &s->phi[d]);
        s->R[d] = stencil_radius(P, d);
        s->dx[d] = P->L[d] / (double)P->n[d];
    }
}

/* Sum of the raw Gaussian exp(-r^2 / 2 sigma^2) over the nodes within the
 * cut-off sphere, times the cell volume. */
static double normalisation(const oracle_params *P, const stencil_t *s)
{
    const double rc = P->cutoff * P->sigma;
    const double R2 = rc * rc;
    const double two_s2 = 2.0 * P->sigma * P->sigma;
    const double dV = s->dx[0] * s->dx[1] * s->dx[2];
    double Z = 0.0;
    int mx, my, mz;
    for (mz = -s->R[2]; mz <= s->R[2] + 1; ++mz) {
        double dz = ((double)mz - s->phi[2]) * s->dx[2];
        for (my = -s->R[1]; my <= s->R[1] + 1; ++my) {
            double dy = ((double)my - s->phi[1]) * s->dx[1];
            for (mx = -s->R[0]; mx <= s->R[0] + 1; ++mx) {
                double ddx = ((double)mx - s->phi[0]) * s->dx[0];
                double r2 = ddx * ddx + dy * dy + dz * dz;
                if (r2 <= R2) Z += exp(-r2 / two_s2);
            }
        }
    }
    return Z * dV;
}

void oracle_normalisation(const oracle_params *P, const double *X, double *Z)
{
    int64_t p;
    for (p = 0; p < P->np; ++p) {
        stencil_t s;
        stencil_of(P, X, p, &s);
        Z[p] = normalisation(P, &s);
    }
}

void oracle_deposit(const oracle_params *P, const double *X, const double *D,
                    const int32_t lo[3], const int32_t wn[3], double *f)
{
    const int64_t np = P->np;
    const int64_t wsz = (int64_t)wn[0] * wn[1] * wn[2];
    const double rc = P->cutoff * P->sigma;
    const double R2 = rc * rc;
    const double two_s2 = 2.0 * P->sigma * P->sigma;
    int64_t p;
    memset(f, 0, sizeof(double) * (size_t)(3 * wsz));
    for (p = 0; p < np; ++p) {
        stencil_t s;
        int d, mx, my, mz, touches = 1;
        double Z, a[3];
        stencil_of(P, X, p, &s);
        /* a particle whose stencil box misses the window contributes nothing */
        for (d = 0; d < 3; ++d) {
            int64_t first = imod((int64_t)s.b[d] - s.R[d] - lo[d], P->n[d]);
            int64_t ext = 2 * (int64_t)s.R[d] + 2;
            if (wn[d] < P->n[d] && first >= wn[d] && first + ext <= P->n[d]) touches = 0;
        }
        if (!touches) continue;
        Z = normalisation(P, &s);
        for (d = 0; d < 3; ++d) a[d] = -D[d * np + p] / P->rho_f;
        for (mz = -s.R[2]; mz <= s.R[2] + 1; ++mz) {
            double dz = ((double)mz - s.phi[2]) * s.dx[2];
            int64_t kz = imod((int64_t)s.b[2] + mz - lo[2], P->n[2]);
            if (kz >= wn[2]) continue;
            for (my = -s.R[1]; my <= s.R[1] + 1; ++my) {
                double dy = ((double)my - s.phi[1]) * s.dx[1];
                int64_t jy = imod((int64_t)s.b[1] + my - lo[1], P->n[1]);
                if (jy >= wn[1]) continue;
                for (mx = -s.R[0]; mx <= s.R[0] + 1; ++mx) {
                    double ddx = ((double)mx - s.phi[0]) * s.dx[0];
                    int64_t ix = imod((int64_t)s.b[0] + mx - lo[0], P->n[0]);
                    double r2 = ddx * ddx + dy * dy + dz * dz;
                    double w;
                    int64_t node;
                    if (ix >= wn[0] || r2 > R2) continue;
                    w = exp(-r2 / two_s2) / Z;
                    node = (kz * wn[1] + jy) * wn[0] + ix;
                    f[0 * wsz + node] += a[0] * w;
                    f[1 * wsz + node] += a[1] * w;
                    f[2 * wsz + node] += a[2] * w;
                }
            }
        }
    }
}

/* ------------------------------------------------------ self-disturbance --- */

/* Closed form of App. E (eq. disturbance_velo) with the -dt/rho_f prefactor of
 * eqs. forcing_step and pseudo_velo_num:
 *
 *   v = -(dt/rho_f) (2 pi s^2)^(-3/2) { [e^{-eta^2} - F] D
 *                                       - (D.rh) [e^{-eta^2} - 3F] rh },
 *   F = f(eta) / (2 eta^3),  f(eta) = (sqrt(pi)/2) erf(eta) - eta e^{-eta^2},
 *   eta = |r| / (sqrt(2) s),  s^2 = sigma_R^2 + 2 nu dt,  r = x - X' (min image).
 *
 * For eta < 0.3 both brackets are summed from their Maclaurin series (the
 * closed form loses all digits to cancellation as eta -> 0):
 *   F              = sum_{j>=0} (-1)^j eta^{2j} / (j! (2j+3))
 *   e^{-eta^2} - 3F = sum_{j>=1} (-1)^j 2j eta^{2j} / (j! (2j+3))
 * and the second term is written (D.r) r [bracket / r^2], finite at r = 0. */
static void self_disturbance_one(const oracle_params *P, const double r[3],
                                 const double Dp[3], double vs[3])
{
    const double s2 = P->sigma * P->sigma + 2.0 * P->nu * P->dt;
    const double pref = -(P->dt / P->rho_f) * pow(2.0 * ORACLE_PI * s2, -1.5);
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double eta2 = rr / (2.0 * s2);
    const double eta = sqrt(eta2);
    const double e = exp(-eta2);
    const double Dr = Dp[0] * r[0] + Dp[1] * r[1] + Dp[2] * r[2];
    double F, Hr; /* Hr = (e^{-eta^2} - 3F) / r^2 */
    int c;
    if (eta < 0.3) {
        double t = 1.0;  /* (-1)^j eta^{2j} / j!          */
        double q = -1.0; /* (-1)^j eta^{2(j-1)} / j!, j>=1 */
        int j;
        F = 0.0;
        Hr = 0.0;
        for (j = 0; j <= 8; ++j) {
            F += t / (2.0 * j + 3.0);
            t *= -eta2 / (double)(j + 1);
        }
        for (j = 1; j <= 8; ++j) {
            Hr += (2.0 * j) * q / (2.0 * j + 3.0);
            q *= -eta2 / (double)(j + 1);
        }
        Hr /= 2.0 * s2; /* eta^2 / r^2 = 1 / (2 s^2) */
    } else {
        double fe = 0.5 * sqrt(ORACLE_PI) * erf(eta) - eta * e;
        F = fe / (2.0 * eta * eta2);
        Hr = (e - 3.0 * F) / rr;
    }
    for (c = 0; c < 3; ++c) vs[c] = pref * ((e - F) * Dp[c] - Dr * r[c] * Hr);
}

void oracle_self_disturbance(const oracle_params *P, const double *x,
                             const double *Xp, const double *Dp, double *vs)
{
    const int64_t np = P->np;
    int64_t p;
    for (p = 0; p < np; ++p) {
        double r[3], D[3], out[3];
        int d;
        for (d = 0; d < 3; ++d) {
            double rd = x[d * np + p] - Xp[d * np + p];
            rd -= P->L[d] * nearbyint(rd / P->L[d]);
            r[d] = rd;
            D[d] = Dp[d * np + p];
        }
        self_disturbance_one(P, r, D, out);
        for (d = 0; d < 3; ++d) vs[d * np + p] = out[d];
    }
}

/* --------------------------------------------------------------- gather --- */

/* Laplacian of the App. E disturbance.  That disturbance is the projection
 * of the regularised impulse -(dt/rho_f) D g(r; s), s = sigma_s^2 (forcing,
 * heat semigroup, projection), and the Laplacian commutes with the
 * projection, so lap v = -(dt/rho_f) [D lap g - grad (D . grad g)]; with the
 * Gaussian's derivatives  lap g = g (r^2/s^2 - 3/s) and
 * d_i d_j g = g (r_i r_j / s^2 - delta_ij / s):
 *   lap v_c = -(dt/rho_f) g [D_c (r^2/s^2 - 2/s) - r_c (D.r)/s^2]. */
static void self_laplacian_one(const oracle_params *P, const double r[3],
                               const double Dp[3], double ls[3])
{
    const double s = P->sigma * P->sigma + 2.0 * P->nu * P->dt;
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double g = pow(2.0 * ORACLE_PI * s, -1.5) * exp(-rr / (2.0 * s));
    const double Dr = Dp[0] * r[0] + Dp[1] * r[1] + Dp[2] * r[2];
    int c;
    for (c = 0; c < 3; ++c)
        ls[c] = -(P->dt / P->rho_f) * g * (Dp[c] * (rr / (s * s) - 2.0 / s) - r[c] * Dr / (s * s));
}

void oracle_self_laplacian(const oracle_params *P, const double *x,
                           const double *Xp, const double *Dp, double *ls)
{
    const int64_t np = P->np;
    int64_t p;
    for (p = 0; p < np; ++p) {
        double r[3], D[3], out[3];
        int d;
        for (d = 0; d < 3; ++d) {
            double rd = x[d * np + p] - Xp[d * np + p];
            rd -= P->L[d] * nearbyint(rd / P->L[d]);
            r[d] = rd;
            D[d] = Dp[d * np + p];
        }
        self_laplacian_one(P, r, D, out);
        for (d = 0; d < 3; ++d) ls[d * np + p] = out[d];
    }
}

/* Gradient of the App. E disturbance.  With v_c = pref [A D_c - (D.r) r_c H],
 * A = e^{-eta^2} - F and H = (e^{-eta^2} - 3F) / r^2 (both functions of r^2
 * through eta^2 = r^2 / (2 s), s = sigma_s^2), the derivatives
 *   dF/d(eta^2) = (e^{-eta^2} - 3F) / (2 eta^2)   (from f'(eta) = 2 eta^2 e^{-eta^2})
 *   dA/d(r^2)   = -(e^{-eta^2}/s + H) / 2
 *   dH/d(r^2)   = -K / 2,  K = (e^{-eta^2}/s + 5H) / r^2
 * give
 *   d_j v_c = pref [ -(e/s + H) r_j D_c - H D_j r_c - H (D.r) delta_cj + K (D.r) r_c r_j ].
 * K is finite at r = 0; for eta < 0.3 it is summed from its Maclaurin series
 *   K = (1 / (2 s^2)) sum_{m>=1} (-1)^m 2m eta^{2(m-1)} / (m! (2m + 5)).
 * (The trace vanishes: the disturbance is solenoidal.) */
static void self_gradient_one(const oracle_params *P, const double r[3],
                              const double Dp[3], double gs[9])
{
    const double s2 = P->sigma * P->sigma + 2.0 * P->nu * P->dt;
    const double pref = -(P->dt / P->rho_f) * pow(2.0 * ORACLE_PI * s2, -1.5);
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double eta2 = rr / (2.0 * s2);
    const double eta = sqrt(eta2);
    const double e = exp(-eta2);
    const double Dr = Dp[0] * r[0] + Dp[1] * r[1] + Dp[2] * r[2];
    double H, K;
    int c, j;
    if (eta < 0.3) {
        double q = -1.0; /* (-1)^m eta^{2(m-1)} / m!, m >= 1 */
        int m;
        H = 0.0;
        K = 0.0;
        for (m = 1; m <= 8; ++m) {
            H += (2.0 * m) * q / (2.0 * m + 3.0);
            K += (2.0 * m) * q / (2.0 * m + 5.0);
            q *= -eta2 / (double)(m + 1);
        }
        H /= 2.0 * s2;
        K /= 2.0 * s2 * s2;
    } else {
        const double fe = 0.5 * sqrt(ORACLE_PI) * erf(eta) - eta * e;
        const double F = fe / (2.0 * eta * eta2);
        H = (e - 3.0 * F) / rr;
        K = (e / s2 + 5.0 * H) / rr;
    }
    for (c = 0; c < 3; ++c)
        for (j = 0; j < 3; ++j) {
            double t = -(e / s2 + H) * r[j] * Dp[c] - H * Dp[j] * r[c] + K * Dr * r[c] * r[j];
            if (c == j) t -= H * Dr;
            gs[3 * c + j] = pref * t;
        }
}

void oracle_self_gradient(const oracle_params *P, const double *x,
                          const double *Xp, const double *Dp, double *gs)
{
    const int64_t np = P->np;
    int64_t p;
    for (p = 0; p < np; ++p) {
        double r[3], D[3], out[9];
        int d;
        for (d = 0; d < 3; ++d) {
            double rd = x[d * np + p] - Xp[d * np + p];
            rd -= P->L[d] * nearbyint(rd / P->L[d]);
            r[d] = rd;
            D[d] = Dp[d * np + p];
        }
        self_gradient_one(P, r, D, out);
        for (d = 0; d < 9; ++d) gs[d * np + p] = out[d];
    }
}

/* Central difference d u_c / d x_j at node (i, j, k), periodic. */
static double node_derivative(const oracle_params *P, const double *u, int c, int dir,
                              int64_t i, int64_t j, int64_t k)
{
    const int64_t Nx = P->n[0], Ny = P->n[1], Nz = P->n[2];
    const double *uc = u + (int64_t)c * Nx * Ny * Nz;
    const double h = P->L[dir] / P->n[dir];
    const int64_t di = dir == 0, dj = dir == 1, dk = dir == 2;
#define U_AT(a, b, d) uc[(imod(d, Nz) * Ny + imod(b, Ny)) * Nx + imod(a, Nx)]
    const double up = U_AT(i + di, j + dj, k + dk), um = U_AT(i - di, j - dj, k - dk);
#undef U_AT
    return (up - um) / (2.0 * h);
}

void oracle_grid_gradient(const oracle_params *P, const double *u, const double *x,
                          double *gu)
{
    const int64_t np = P->np;
    int64_t p;
    for (p = 0; p < np; ++p) {
        int32_t b[3];
        double phi[3], w[3][2], acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        int d, a, bb, cc, c, j;
        for (d = 0; d < 3; ++d) {
            cell_of(x[d * np + p], P->L[d], P->n[d], &b[d], &phi[d]);
            w[d][0] = 1.0 - phi[d];
            w[d][1] = phi[d];
        }
        for (cc = 0; cc < 2; ++cc)
            for (bb = 0; bb < 2; ++bb)
                for (a = 0; a < 2; ++a) {
                    double wt = w[0][a] * w[1][bb] * w[2][cc];
                    for (c = 0; c < 3; ++c)
                        for (j = 0; j < 3; ++j)
                            acc[3 * c + j] += wt * node_derivative(P, u, c, j, (int64_t)b[0] + a,
                                                                   (int64_t)b[1] + bb,
                                                                   (int64_t)b[2] + cc);
                }
        acc[1] += P->shear; /* d U_x / d y of the mean shear */
        for (d = 0; d < 9; ++d) gu[d * np + p] = acc[d];
    }
}

/* 7-point Laplacian of component c at node (i, j, k), periodic. */
static double node_laplacian(const oracle_params *P, const double *u, int c, int64_t i,
                             int64_t j, int64_t k)
{
    const int64_t Nx = P->n[0], Ny = P->n[1], Nz = P->n[2];
    const double *uc = u + (int64_t)c * Nx * Ny * Nz;
    const double h0 = P->L[0] / Nx, h1 = P->L[1] / Ny, h2 = P->L[2] / Nz;
#define U_AT(a, b, d) uc[(imod(d, Nz) * Ny + imod(b, Ny)) * Nx + imod(a, Nx)]
    const double u0 = U_AT(i, j, k);
    const double lx = (U_AT(i + 1, j, k) - 2.0 * u0 + U_AT(i - 1, j, k)) / (h0 * h0);
    const double ly = (U_AT(i, j + 1, k) - 2.0 * u0 + U_AT(i, j - 1, k)) / (h1 * h1);
    const double lz = (U_AT(i, j, k + 1) - 2.0 * u0 + U_AT(i, j, k - 1)) / (h2 * h2);
#undef U_AT
    return lx + ly + lz;
}

void oracle_grid_laplacian(const oracle_params *P, const double *u, const double *x,
                           double *lu)
{
    const int64_t np = P->np;
    int64_t p;
    for (p = 0; p < np; ++p) {
        int32_t b[3];
        double phi[3], w[3][2], acc[3] = {0.0, 0.0, 0.0};
        int d, a, bb, cc, c;
        for (d = 0; d < 3; ++d) {
            cell_of(x[d * np + p], P->L[d], P->n[d], &b[d], &phi[d]);
            w[d][0] = 1.0 - phi[d];
            w[d][1] = phi[d];
        }
        for (cc = 0; cc < 2; ++cc)
            for (bb = 0; bb < 2; ++bb)
                for (a = 0; a < 2; ++a) {
                    double wt = w[0][a] * w[1][bb] * w[2][cc];
                    for (c = 0; c < 3; ++c)
                        acc[c] += wt * node_laplacian(P, u, c, (int64_t)b[0] + a,
                                                      (int64_t)b[1] + bb, (int64_t)b[2] + cc);
                }
        for (c = 0; c < 3; ++c) lu[c * np + p] = acc[c];
    }
}

void oracle_gather(const oracle_params *P, const double *u, const double *x,
                   double *up)
{
    const int64_t np = P->np;
    const int64_t Nx = P->n[0], Ny = P->n[1], Nz = P->n[2];
    const int64_t ng = Nx * Ny * Nz;
    int64_t p;
    for (p = 0; p < np; ++p) {
        int32_t b[3];
        double phi[3], w[3][2], acc[3] = {0.0, 0.0, 0.0};
        int64_t idx[3][2];
        int d, a, bb, cc, c;
        for (d = 0; d < 3; ++d) {
            cell_of(x[d * np + p], P->L[d], P->n[d], &b[d], &phi[d]);
            w[d][0] = 1.0 - phi[d];
            w[d][1] = phi[d];
            idx[d][0] = b[d];
            idx[d][1] = imod((int64_t)b[d] + 1, P->n[d]);
        }
        for (cc = 0; cc < 2; ++cc)
            for (bb = 0; bb < 2; ++bb)
                for (a = 0; a < 2; ++a) {
                    double wt = w[0][a] * w[1][bb] * w[2][cc];
                    int64_t node = (idx[2][cc] * Ny + idx[1][bb]) * Nx + idx[0][a];
                    for (c = 0; c < 3; ++c) acc[c] += wt * u[c * ng + node];
                }
        if (P->shear != 0.0) {
            double yh = wrap_coord(x[np + p], P->L[1]);
            acc[0] += P->shear * (yh - 0.5 * P->L[1]);
        }
        for (c = 0; c < 3; ++c) up[c * np + p] = acc[c];
    }
}

/* ----------------------------------------------------------------- step --- */

void oracle_step(const oracle_params *P, int64_t n, const double *u,
                 double *x, double *v, const float *tau, double *ring_x,
                 double *ring_d, const int32_t lo[3], const int32_t wn[3],
                 double *f, double *dout, double *am_hist, int32_t *am_valid,
                 double *bs_hist, int32_t *bs_valid)
{
    const int64_t np = P->np;
    const int32_t M = P->M;
    const int64_t lvl = (int64_t)3 * np; /* doubles per ring level */
    double *vs = (double *)calloc((size_t)(3 * np > 0 ? 3 * np : 1), sizeof(double));
    double *up = (double *)malloc(sizeof(double) * (size_t)(3 * np > 0 ? 3 * np : 1));
    double *ls = (double *)calloc((size_t)(3 * np > 0 ? 3 * np : 1), sizeof(double));
    double *lu = (double *)calloc((size_t)(3 * np > 0 ? 3 * np : 1), sizeof(double));
    const double fax = P->a_p * P->a_p / 6.0;
    /* added mass (eq. force_particle, second line): displaced mass and the
       Faxen coefficient of its d/dt term */
    const int am = P->a_am > 0.0;
    const double m_f = am ? P->rho_f * 4.0 / 3.0 * ORACLE_PI * P->a_am * P->a_am * P->a_am : 0.0;
    const double fam = P->a_am * P->a_am / 10.0;
    /* Basset term (eq. force_particle, third line): in the two-way coupled
       scheme the field carries the particle's earlier vorticity, so the memory
       integral covers the last step only (closing paragraph of Sec. 2.5).  With
       the bracket w = u~ + (a_b^2/6) lap u~ - v changing at the constant rate
       (w^n - w^{n-1})/dt over that step,
         6 pi mu a_b^2 int_{t-dt}^{t} [pi nu (t - s)]^{-1/2} ds (w^n - w^{n-1})/dt
         = 12 pi mu a_b^2 (w^n - w^{n-1}) / sqrt(pi nu dt). */
    const int bs = P->a_b > 0.0;
    const double fbs = P->a_b * P->a_b / 6.0;
    const double kbs = bs ? 12.0 * ORACLE_PI * P->rho_f * P->nu * P->a_b * P->a_b /
                                sqrt(ORACLE_PI * P->nu * P->dt)
                          : 0.0;
    int64_t p;

    /* 1. forcing from the drag delayed by eps_R = M dt */
    if (f) {
        if (n >= M) {
            int64_t slot = (n - M) % (M + 1);
            oracle_deposit(P, ring_x + slot * lvl, ring_d + slot * lvl, lo, wn, f);
        } else {
            int64_t wsz = (int64_t)wn[0] * wn[1] * wn[2];
            memset(f, 0, sizeof(double) * (size_t)(3 * wsz));
        }
    }
    /* 2. self-disturbance of the injection made at step n-1 (level n-1-M) */
    if (P->self_correction && n >= M + 1) {
        int64_t slot = (n - 1 - M) % (M + 1);
        oracle_self_disturbance(P, x, ring_x + slot * lvl, ring_d + slot * lvl, vs);
        if (fax != 0.0 || am || bs)
            oracle_self_laplacian(P, x, ring_x + slot * lvl, ring_d + slot * lvl, ls);
    }
    /* Faxen correction of the drag (eq. force_particle, first line):
       (a_p^2/6) lap u~ with u~ = u - v_self */
    if (fax != 0.0 || am || bs) oracle_grid_laplacian(P, u, x, lu);
    /* added mass: the gradient of u~ = u - v_self for the convective part of
       the fluid acceleration */
    double *gu = NULL, *gs = NULL;
    if (am) {
        size_t sz = (size_t)(9 * np > 0 ? 9 * np : 1);
        gu = (double *)malloc(sizeof(double) * sz);
        gs = (double *)calloc(sz, sizeof(double));
        oracle_grid_gradient(P, u, x, gu);
        if (P->self_correction && n >= M + 1) {
            int64_t slot = (n - 1 - M) % (M + 1);
            oracle_self_gradient(P, x, ring_x + slot * lvl, ring_d + slot * lvl, gs);
        }
    }
    /* Heun: the second stage sits at x* = x^n + dt v^n, where the carrier, the
       self term of the same injection (removed at each stage, Sec. 2.5) and the
       Faxen Laplacians are evaluated again */
    double *xs = NULL, *up2 = NULL, *vs2 = NULL, *lu2 = NULL, *ls2 = NULL;
    if (P->integrator == 2) {
        size_t sz = (size_t)(3 * np > 0 ? 3 * np : 1);
        xs = (double *)malloc(sizeof(double) * sz);
        up2 = (double *)malloc(sizeof(double) * sz);
        vs2 = (double *)calloc(sz, sizeof(double));
        lu2 = (double *)calloc(sz, sizeof(double));
        ls2 = (double *)calloc(sz, sizeof(double));
        for (p = 0; p < 3 * np; ++p) xs[p] = x[p] + P->dt * v[p];
        oracle_gather(P, u, xs, up2);
        if (P->self_correction && n >= M + 1) {
            int64_t slot = (n - 1 - M) % (M + 1);
            oracle_self_disturbance(P, xs, ring_x + slot * lvl, ring_d + slot * lvl, vs2);
            if (fax != 0.0)
                oracle_self_laplacian(P, xs, ring_x + slot * lvl, ring_d + slot * lvl, ls2);
        }
        if (fax != 0.0) oracle_grid_laplacian(P, u, xs, lu2);
    }
    /* 3. carrier velocity at the particles */
    oracle_gather(P, u, x, up);
    /* 4. drag, history, explicit Euler */
    {
        int64_t slot = n % (M + 1);
        double *hx = ring_x + slot * lvl;
        double *hd = ring_d + slot * lvl;
        for (p = 0; p < np; ++p) {
            double t = (double)tau[p];
            double D[3], xn[3];
            int d;
            int64_t k;
            if (am || bs) {
                /* eq. force_particle, explicit Euler with the particle's own
                   acceleration in the added-mass term moved to the left:
                     (m_p + m_f/2) dv/dt = S + m_f Du~/Dt + (m_f/2) dq/dt + B + m_p g_b,
                   S = m_p (u~ + (a_p^2/6) lap u~ - v) / tau_p,
                   q = u~ + (a_am^2/10) lap u~,
                   B = kbs (w^n - w^{n-1}),  w = u~ + (a_b^2/6) lap u~ - v,
                   d/dt along the path: (value^n - value^{n-1}) / dt, and B, zero on
                   the first step that has no previous value;
                   Du~/Dt = du~/dt + (u~ - v) . grad u~ (material derivative from
                   the path derivative).  D = m_p dv/dt - m_p g_b is the
                   hydrodynamic force handed to the fluid.  Without added mass
                   m_f = 0 and the scheme is explicit Euler with S + B. */
                double ut[3], q[3], S[3], w[3], Dm[3], acc[3];
                const int valid = am ? *am_valid : 0;
                const int bvalid = bs ? *bs_valid : 0;
                for (d = 0; d < 3; ++d) {
                    ut[d] = up[d * np + p] - vs[d * np + p];
                    q[d] = ut[d] + fam * (lu[d * np + p] - ls[d * np + p]);
                    S[d] = P->m_p * (ut[d] + fax * (lu[d * np + p] - ls[d * np + p]) -
                                     v[d * np + p]) / t;
                    w[d] = ut[d] + fbs * (lu[d * np + p] - ls[d * np + p]) - v[d * np + p];
                }
                for (d = 0; d < 3; ++d) {
                    double conv = 0.0, dut = 0.0, dq = 0.0, Bs = 0.0;
                    int jd;
                    if (am) {
                        for (jd = 0; jd < 3; ++jd)
                            conv += (ut[jd] - v[jd * np + p]) *
                                    (gu[(3 * d + jd) * np + p] - gs[(3 * d + jd) * np + p]);
                        dut = valid ? (ut[d] - am_hist[d * np + p]) / P->dt : 0.0;
                        dq = valid ? (q[d] - am_hist[(3 + d) * np + p]) / P->dt : 0.0;
                    }
                    if (bvalid) Bs = kbs * (w[d] - bs_hist[d * np + p]);
                    Dm[d] = dut + conv;
                    acc[d] = (S[d] + m_f * Dm[d] + 0.5 * m_f * dq + Bs + P->m_p * P->g[d]) /
                             (P->m_p + 0.5 * m_f);
                    D[d] = S[d] + m_f * Dm[d] + 0.5 * m_f * (dq - acc[d]) + Bs;
                }
                for (d = 0; d < 3; ++d) {
                    hx[d * np + p] = x[d * np + p];
                    hd[d * np + p] = D[d];
                    if (dout) dout[d * np + p] = D[d];
                    xn[d] = x[d * np + p] + P->dt * v[d * np + p];
                    v[d * np + p] += P->dt * acc[d];
                    if (am) {
                        am_hist[d * np + p] = ut[d];
                        am_hist[(3 + d) * np + p] = q[d];
                    }
                    if (bs) bs_hist[d * np + p] = w[d];
                }
            } else if (P->integrator == 0) {
                for (d = 0; d < 3; ++d) {
                    double ut = up[d * np + p] - vs[d * np + p];
                    ut += fax * (lu[d * np + p] - ls[d * np + p]);
                    D[d] = P->m_p * (ut - v[d * np + p]) / t;
                }
                for (d = 0; d < 3; ++d) {
                    hx[d * np + p] = x[d * np + p];
                    hd[d * np + p] = D[d];
                    if (dout) dout[d * np + p] = D[d];
                    xn[d] = x[d * np + p] + P->dt * v[d * np + p];
                }
                /* eq. particle_motion: m_p dv/dt = D + (m_p - m_f) g; the body
                   force is not part of D, so the fluid never receives it */
                for (d = 0; d < 3; ++d) {
                    v[d * np + p] += P->dt * D[d] / P->m_p;
                    v[d * np + p] += P->dt * P->g[d];
                }
            } else if (P->integrator == 2) {
                /* Heun: a_1 = (u~(x^n) - v^n)/tau + g, v* = v^n + dt a_1,
                   a_2 = (u~(x*) - v*)/tau + g; v^{n+1} = v^n + dt (a_1 + a_2)/2,
                   x^{n+1} = x^n + dt (v^n + v*)/2; the fluid gets the mean drag */
                for (d = 0; d < 3; ++d) {
                    double v0 = v[d * np + p];
                    double ut1 = up[d * np + p] - vs[d * np + p];
                    double ut2 = up2[d * np + p] - vs2[d * np + p];
                    ut1 += fax * (lu[d * np + p] - ls[d * np + p]);
                    ut2 += fax * (lu2[d * np + p] - ls2[d * np + p]);
                    double d1 = (ut1 - v0) / t;
                    double vst = v0 + P->dt * (d1 + P->g[d]);
                    double d2 = (ut2 - vst) / t;
                    double dm = 0.5 * (d1 + d2);
                    D[d] = P->m_p * dm;
                    hx[d * np + p] = x[d * np + p];
                    hd[d * np + p] = D[d];
                    if (dout) dout[d * np + p] = D[d];
                    xn[d] = x[d * np + p] + 0.5 * P->dt * (v0 + vst);
                    v[d * np + p] = v0 + P->dt * (dm + P->g[d]);
                }
            } else {
                /* dv/dt = (u~ - v)/tau + g with u~ held over the step has the
                   solution v(s) = w + (v^n - w) exp(-s/tau), w = u~ + tau g;
                   x advances by its integral; the fluid receives the
                   momentum the drag exchanged, divided by dt */
                double E = exp(-P->dt / t);
                double a = -expm1(-P->dt / t);   /* 1 - E without cancellation */
                for (d = 0; d < 3; ++d) {
                    double ut = up[d * np + p] - vs[d * np + p];
                    double v0 = v[d * np + p];
                    ut += fax * (lu[d * np + p] - ls[d * np + p]);
                    double w = ut + t * P->g[d];
                    double v1 = w + (v0 - w) * E;
                    hx[d * np + p] = x[d * np + p];
                    xn[d] = x[d * np + p] + P->dt * w + t * (v0 - w) * a;
                    D[d] = P->m_p * (v1 - v0) / P->dt - P->m_p * P->g[d];
                    hd[d * np + p] = D[d];
                    if (dout) dout[d * np + p] = D[d];
                    v[d * np + p] = v1;
                }
            }
            for (d = 0; d < 3; ++d) {
                double L = P->L[d];
                double w = xn[d] - L * floor(xn[d] / L);
                k = (int64_t)floor(xn[d] / L);
                if (w >= L) { w -= L; k += 1; }
                if (w < 0.0) w = 0.0;
                x[d * np + p] = w;
                if (d == 1 && P->shear != 0.0 && k != 0)
                    v[0 * np + p] -= (double)k * P->shear * L;
            }
        }
    }
    if (am) *am_valid = 1;
    if (bs) *bs_valid = 1;
    free(gu);
    free(gs);
    free(vs);
    free(up);
    free(ls);
    free(lu);
    free(xs);
    free(up2);
    free(vs2);
    free(lu2);
    free(ls2);
}
