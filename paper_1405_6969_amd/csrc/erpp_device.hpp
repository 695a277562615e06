// erpp_device.hpp -- device helpers of the ERPP coupling step (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "erpp_internal.hpp"

namespace erpp {

// Box of a block from the box-aligned block offsets (uniform per block).
template <typename F>
__device__ __forceinline__ int box_of_block(const DevBox *__restrict__ B, int nbox,
                                            int64_t blk, F key) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key(B[mid]) <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- FP64 cell --
// Periodic wrap into [0, L) and cell index / offset of a coordinate with nodes at
// i*dx.  Every operation rounded as written (same arithmetic as the reference
// definition: y = x - L floor(x/L); s = y/dx; b = min(floor(s), N-1); phi = s - b).
__device__ __forceinline__ double wrap_coord(double x, double L) {
#pragma clang fp contract(off)
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y = 0.0;
    return y;
}

__device__ __forceinline__ void cell_of(double x, double L, double dx, int N, int &b,
                                        double &phi) {
#pragma clang fp contract(off)
    double xh = wrap_coord(x, L);
    double s = xh / dx;
    double fb = floor(s);
    int i = (int)fb;
    if (i > N - 1) i = N - 1;
    if (i < 0) i = 0;
    b = i;
    phi = s - (double)i;
}

// Sphere membership of stencil node (mx,my,mz) in FP64, rounded exactly like the
// definition: d = (m - phi) dx per dimension, r2 = dx^2 + dy^2 + dz^2 <= R2.
__device__ __forceinline__ bool inside64(int mx, int my, int mz, double phx, double phy,
                                      double phz, const DevBox &B) {
#pragma clang fp contract(off)
    double ddx = ((double)mx - phx) * B.dx[0];
    double dy = ((double)my - phy) * B.dx[1];
    double dz = ((double)mz - phz) * B.dx[2];
    double r2 = ddx * ddx + dy * dy + dz * dz;
    return r2 <= B.R2;
}

// Sphere membership decided in FP64 for a particle whose FP32 test fell inside
// the guard band: re-read its delayed position from the ring (rare path).
__device__ __forceinline__ bool inside_exact(const DevBox *__restrict__ Bp, int64_t slot, int pid,
                                          int mx, int my, int mz) {
    const DevBox &B = *Bp;
    const int64_t np = B.np;
    const double *X = B.ring_x + slot * 3 * np;
    int b;
    double phx, phy, phz;
    cell_of(X[pid], B.L[0], B.dx[0], B.n[0], b, phx);
    cell_of(X[np + pid], B.L[1], B.dx[1], B.n[1], b, phy);
    cell_of(X[2 * np + pid], B.L[2], B.dx[2], B.n[2], b, phz);
    return inside64(mx, my, mz, phx, phy, phz, B);
}

// -------------------------------------------------------------- FP32 kernel --
// 1-D factor of the raw Gaussian: exp2(-t^2 cexp), t = (m - phi) dx.
__device__ __forceinline__ float g1(int m, float phi, float dxf, float cexp) {
    float t = ((float)m - phi) * dxf;
    return exp2f(-(t * t) * cexp);
}

__device__ __forceinline__ float d1(int m, float phi, float dxf) {
    float t = ((float)m - phi) * dxf;
    return t;
}

// Sphere decision for node mx of row (my, mz) in FP32 (ryz = dy^2 + dz^2 of the
// row, fused), with the FP64 decision inside the guard band around R2.
__device__ __forceinline__ bool inside32(int mx, float phx, float ryz, const DevBox &B,
                                         const DevBox *Bp, int64_t slot, int pid, int my,
                                         int mz) {
    float t = ((float)mx - phx) * B.dxf[0];
    float d2 = fmaf(t, t, ryz);
    if (d2 < B.R2f - B.guard) return true;
    if (d2 > B.R2f + B.guard) return false;
    return inside_exact(Bp, slot, pid, mx, my, mz);
}

// Contiguous range [lo, hi] of x offsets of row (my, mz) inside the sphere,
// within [mlo, mhi]; lo > hi when the row is empty.  Membership along a row is
// monotone in |mx - phi|, so the row is [ceil(phi - s*), floor(phi + s*)] for
// the exact half-width s* (in nodes).  Its estimate s = sqrt(R^2 - ryz) / dx
// (raw v_sqrt, multiply by 1/dx) has |s^2 - s*^2| <= E / dx^2, E the FP32 error
// of R^2 - ryz (below twice the guard band), so |s - s*| <= E / (dx^2 s); with
// the roundings of the sqrt and of phi -/+ s the estimated ends are off by less
// than gs / s, gs = 2 guard / dx^2 + 1e-6 smax (smax + 1).  When both estimated
// ends phi -/+ s lie farther than that from every node, ceil and floor of them
// are the exact ends.  Otherwise (rare: a few rows in 1e4) each end is
// settled by one exact decision (inside32 semantics) at the node k nearest the
// estimated end: the end is k if k is inside, else the next node inward; a row
// with s < 0.01 can hold only the node nearest phi, which both ends then test.
// The node set is therefore the exact one, the same in every kernel that calls
// this.
// The box constants row_range reads, held by value so that a kernel can keep
// them in registers across its loops.
struct RowK {
    float R2f, guard, idx0, dx0, gs;
    int mlo0, mhi0;
};

__device__ __forceinline__ RowK row_consts(const DevBox &B) {
    const float i2 = B.idxf0 * B.idxf0;
    const float smax = sqrtf(B.R2f * i2);
    return RowK{B.R2f, B.guard, B.idxf0, B.dxf[0], 2.0f * B.guard * i2 + 1e-6f * smax * (smax + 1.0f),
                B.mlo[0], B.mhi[0]};
}

__device__ __forceinline__ void row_range(float phx, float ryz, const RowK &K,
                                          const DevBox *Bp, int64_t slot, int pid, int my,
                                          int mz, int &lo, int &hi) {
    const float rem = fmaxf(K.R2f - ryz, 0.0f);
    const float s = __builtin_amdgcn_sqrtf(rem) * K.idx0;
    const float el = phx - s, eh = phx + s;
    const float kl = rintf(el), kh = rintf(eh);
    if (fminf(fabsf(el - kl), fabsf(eh - kh)) * s >= K.gs) {
        lo = max((int)ceilf(el), K.mlo0);
        hi = min((int)floorf(eh), K.mhi0);
        return;
    }
    const float tl = (kl - phx) * K.dx0, th = (kh - phx) * K.dx0;
    const float dl = fmaf(tl, tl, ryz), dh = fmaf(th, th, ryz);
    const float below = K.R2f - K.guard, above = K.R2f + K.guard;
    bool il = dl < below, ih = dh < below;
    if (dl >= below && dl <= above) il = inside_exact(Bp, slot, pid, (int)kl, my, mz);
    if (dh >= below && dh <= above) ih = inside_exact(Bp, slot, pid, (int)kh, my, mz);
    lo = max((int)kl + (il ? 0 : 1), K.mlo0);
    hi = min((int)kh - (ih ? 0 : 1), K.mhi0);
}

__device__ __forceinline__ void row_range(float phx, float ryz, const DevBox &B,
                                          const DevBox *Bp, int64_t slot, int pid, int my,
                                          int mz, int &lo, int &hi) {
    row_range(phx, ryz, row_consts(B), Bp, slot, pid, my, mz, lo, hi);
}

// ---------------------------------------------------------- self-disturbance --
// App. E closed form (with the -dt/rho_f prefactor), FP32.  r = x - X' (min
// image), D' the drag injected one step earlier.  Series for eta < 0.3.
__device__ __forceinline__ void self_disturbance32(float rx, float ry, float rz, float Dx,
                                                   float Dy, float Dz, float s2, float pref,
                                                   float &vx, float &vy, float &vz) {
    float rr = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
    float eta2 = rr / (2.0f * s2);
    float e = expf(-eta2);
    float Dr = fmaf(Dx, rx, fmaf(Dy, ry, Dz * rz));
    float F, Hr;
    if (eta2 < 0.09f) {
        // F = sum_j (-1)^j eta^2j/(j!(2j+3)),  (e - 3F)/eta^2 = sum_{j>=1} 2j (-1)^j eta^2(j-1)/(j!(2j+3))
        float t = 1.0f, q = -1.0f;
        F = 0.0f;
        Hr = 0.0f;
#pragma unroll
        for (int j = 0; j <= 5; ++j) {
            F = fmaf(t, 1.0f / (2.0f * j + 3.0f), F);
            t *= -eta2 / (float)(j + 1);
        }
#pragma unroll
        for (int j = 1; j <= 5; ++j) {
            Hr = fmaf((2.0f * j) / (2.0f * j + 3.0f), q, Hr);
            q *= -eta2 / (float)(j + 1);
        }
        Hr /= 2.0f * s2;
    } else {
        float eta = sqrtf(eta2);
        float fe = 0.88622692545275801f * erff(eta) - eta * e;
        F = fe / (2.0f * eta * eta2);
        Hr = (e - 3.0f * F) / rr;
    }
    float a = e - F;
    float b = Dr * Hr;
    vx = pref * (a * Dx - b * rx);
    vy = pref * (a * Dy - b * ry);
    vz = pref * (a * Dz - b * rz);
}

// FP64 version (plain path), series through j = 8 below eta = 0.3.
__device__ __forceinline__ void self_disturbance64(const double r[3], const double D[3],
                                                   double s2, double pref, double v[3]) {
    double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double eta2 = rr / (2.0 * s2);
    double eta = sqrt(eta2);
    double e = exp(-eta2);
    double Dr = D[0] * r[0] + D[1] * r[1] + D[2] * r[2];
    double F, Hr;
    if (eta < 0.3) {
        double t = 1.0, q = -1.0;
        F = 0.0;
        Hr = 0.0;
        for (int j = 0; j <= 8; ++j) {
            F += t / (2.0 * j + 3.0);
            t *= -eta2 / (double)(j + 1);
        }
        for (int j = 1; j <= 8; ++j) {
            Hr += (2.0 * j) * q / (2.0 * j + 3.0);
            q *= -eta2 / (double)(j + 1);
        }
        Hr /= 2.0 * s2;
    } else {
        double fe = 0.88622692545275801365 * erf(eta) - eta * e;
        F = fe / (2.0 * eta * eta2);
        Hr = (e - 3.0 * F) / rr;
    }
    for (int c = 0; c < 3; ++c) v[c] = pref * ((e - F) * D[c] - Dr * r[c] * Hr);
}

// Trilinear interpolation of a [3][Nz][Ny][Nx] field at x (FP64 weights).
template <typename T>
__device__ __forceinline__ void trilinear(const DevBox &B, const T *__restrict__ u,
                                          const double xp[3], double out[3]) {
    int b[3];
    double ph[3];
    for (int d = 0; d < 3; ++d) cell_of(xp[d], B.L[d], B.dx[d], B.n[d], b[d], ph[d]);
    const int64_t Nx = B.n[0], Ny = B.n[1], Nz = B.n[2];
    const int64_t ng = Nx * Ny * Nz;
    int64_t i0 = b[0], i1 = (b[0] + 1 == B.n[0]) ? 0 : b[0] + 1;
    int64_t j0 = b[1], j1 = (b[1] + 1 == B.n[1]) ? 0 : b[1] + 1;
    int64_t k0 = b[2], k1 = (b[2] + 1 == B.n[2]) ? 0 : b[2] + 1;
    double wx[2] = {1.0 - ph[0], ph[0]};
    double wy[2] = {1.0 - ph[1], ph[1]};
    double wz[2] = {1.0 - ph[2], ph[2]};
    int64_t ii[2] = {i0, i1}, jj[2] = {j0 * Nx, j1 * Nx}, kk[2] = {k0 * Nx * Ny, k1 * Nx * Ny};
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
        for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
            for (int c0 = 0; c0 < 2; ++c0) {
                double w = wx[c0] * wy[c1] * wz[c2];
                int64_t node = kk[c2] + jj[c1] + ii[c0];
                acc0 += w * (double)u[node];
                acc1 += w * (double)u[ng + node];
                acc2 += w * (double)u[2 * ng + node];
            }
    if (B.shear != 0.0) {
        double yh = wrap_coord(xp[1], B.L[1]);
        acc0 += B.shear * (yh - 0.5 * B.L[1]);
    }
    out[0] = acc0;
    out[1] = acc1;
    out[2] = acc2;
}

// index i in [-1, N] taken periodically into [0, N)
__device__ __forceinline__ int wrap_node(int i, int N) { return i < 0 ? i + N : (i >= N ? i - N : i); }

// Trilinear interpolation at xp of the 7-point nodal Laplacian of u (LAP: the
// grid part of the Faxen term; the mean shear is linear and adds nothing) and of
// its central-difference nodal gradient (GRAD, grad[3c + j] = d u_c / d x_j, plus
// the mean shear's d U_x / d y).  Both stencils read the 2x2x2 cell corners and
// their 24 face neighbours: 32 nodes per component, each loaded once.  FP64.
template <typename T, bool LAP, bool GRAD>
__device__ void trilinear_stencils(const DevBox &B, const T *__restrict__ u, const double xp[3],
                                   double lap[3], double grad[9]) {
    int b[3];
    double ph[3];
    for (int d = 0; d < 3; ++d) cell_of(xp[d], B.L[d], B.dx[d], B.n[d], b[d], ph[d]);
    const int Nx = B.n[0], Ny = B.n[1], Nz = B.n[2];
    const int64_t ng = (int64_t)Nx * Ny * Nz;
    int ix[4], iy[4], iz[4];   // nodes b - 1 .. b + 2
    for (int q = 0; q < 4; ++q) {
        ix[q] = wrap_node(b[0] + q - 1, Nx);
        iy[q] = wrap_node(b[1] + q - 1, Ny);
        iz[q] = wrap_node(b[2] + q - 1, Nz);
    }
    const double h0 = 1.0 / (B.dx[0] * B.dx[0]), h1 = 1.0 / (B.dx[1] * B.dx[1]),
                 h2 = 1.0 / (B.dx[2] * B.dx[2]);
    const double g0 = 0.5 / B.dx[0], g1 = 0.5 / B.dx[1], g2 = 0.5 / B.dx[2];
    for (int c = 0; c < 3; ++c) {
        const T *uc = u + c * ng;
        auto at = [&](int a, int bb, int cc) -> double {
            return (double)uc[((int64_t)iz[cc] * Ny + iy[bb]) * Nx + ix[a]];
        };
        double cube[2][2][2], xn[2][2][2], yn[2][2][2], zn[2][2][2];
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) cube[i][j][k] = at(1 + i, 1 + j, 1 + k);
        for (int s2 = 0; s2 < 2; ++s2)
            for (int t = 0; t < 2; ++t) {
                // the neighbour outside the cube: index 0 (s = 0) or 3 (s = 1)
                for (int s = 0; s < 2; ++s) {
                    xn[s][s2][t] = at(3 * s, 1 + s2, 1 + t);
                    yn[s][s2][t] = at(1 + s2, 3 * s, 1 + t);
                    zn[s][s2][t] = at(1 + s2, 1 + t, 3 * s);
                }
            }
        double accl = 0.0, accg[3] = {0.0, 0.0, 0.0};
        for (int c2 = 0; c2 < 2; ++c2)
            for (int c1 = 0; c1 < 2; ++c1)
                for (int c0 = 0; c0 < 2; ++c0) {
                    const double w = (c0 ? ph[0] : 1.0 - ph[0]) * (c1 ? ph[1] : 1.0 - ph[1]) *
                                     (c2 ? ph[2] : 1.0 - ph[2]);
                    const double u0 = cube[c0][c1][c2];
                    const double xm = c0 ? cube[0][c1][c2] : xn[0][c1][c2];
                    const double xq = c0 ? xn[1][c1][c2] : cube[1][c1][c2];
                    const double ym = c1 ? cube[c0][0][c2] : yn[0][c0][c2];
                    const double yq = c1 ? yn[1][c0][c2] : cube[c0][1][c2];
                    const double zm = c2 ? cube[c0][c1][0] : zn[0][c0][c1];
                    const double zq = c2 ? zn[1][c0][c1] : cube[c0][c1][1];
                    if (LAP) {
                        const double lx = (xq - 2.0 * u0 + xm) * h0;
                        const double ly = (yq - 2.0 * u0 + ym) * h1;
                        const double lz = (zq - 2.0 * u0 + zm) * h2;
                        accl += w * (lx + ly + lz);
                    }
                    if (GRAD) {
                        accg[0] += w * ((xq - xm) * g0);
                        accg[1] += w * ((yq - ym) * g1);
                        accg[2] += w * ((zq - zm) * g2);
                    }
                }
        if (LAP) lap[c] = accl;
        if (GRAD)
            for (int j = 0; j < 3; ++j) grad[3 * c + j] = accg[j];
    }
    if (GRAD) grad[1] += B.shear;
}

template <typename T>
__device__ __forceinline__ void trilinear_laplacian(const DevBox &B, const T *__restrict__ u,
                                                    const double xp[3], double out[3]) {
    trilinear_stencils<T, true, false>(B, u, xp, out, nullptr);
}

// Laplacian of the closed-form self-disturbance (the self part of the Faxen
// term): the disturbance is the projection of -(dt/rho_f) D g(r; s), and the
// Laplacian commutes with the projection, so with g's second derivatives
// lap v_c = pref e^{-r^2/(2s)} [D_c (r^2/s^2 - 2/s) - r_c (D.r)/s^2],
// pref = -(dt/rho_f)(2 pi s)^{-3/2}, s = sigma_s^2.  FP64.
__device__ __forceinline__ void self_laplacian64(const double r[3], const double D[3], double s,
                                                 double pref, double out[3]) {
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double e = pref * exp(-rr / (2.0 * s));
    const double Dr = D[0] * r[0] + D[1] * r[1] + D[2] * r[2];
    const double is = 1.0 / s;
    for (int c = 0; c < 3; ++c) out[c] = e * (D[c] * (rr * is * is - 2.0 * is) - r[c] * Dr * is * is);
}

// Gradient of the closed-form self-disturbance, out[3c + j] = d v_c / d x_j.
// Writing the disturbance as v_c = pref [A D_c - (D.r) r_c H] with A = e - F and
// H = (e - 3F) / r^2, functions of u = r^2 / (2s) (e = e^{-u}, s = sigma_s^2):
// dF/du = (e - 3F) / (2u), so dA/d(r^2) = -(e/s + H)/2 and dH/d(r^2) = -K/2 with
// K = (e/s + 5H) / r^2, and
//   d_j v_c = pref [-(e/s + H) r_j D_c - H D_j r_c - H (D.r) delta_cj + K (D.r) r_c r_j].
// Below eta = 0.3 (u < 0.09) H and K come from their power series in u, which
// stay finite at r = 0 where the closed forms cancel.
__device__ __forceinline__ void self_gradient64(const double r[3], const double D[3], double s,
                                                double pref, double out[9]) {
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double u = rr / (2.0 * s);
    const double e = exp(-u);
    const double Dr = D[0] * r[0] + D[1] * r[1] + D[2] * r[2];
    double H, K;
    if (u < 0.09) {
        // H = (1/2s) sum_{m>=1} (-u)^(m-1) (-2m) / (m! (2m+3)), K likewise with 2m+5, over 2s^2
        double c = -1.0;
        H = 0.0;
        K = 0.0;
        for (int m = 1; m <= 8; ++m) {
            H += (2.0 * m) * c / (2.0 * m + 3.0);
            K += (2.0 * m) * c / (2.0 * m + 5.0);
            c *= -u / (double)(m + 1);
        }
        H /= 2.0 * s;
        K /= 2.0 * s * s;
    } else {
        const double eta = sqrt(u);
        const double F = (0.88622692545275801365 * erf(eta) - eta * e) / (2.0 * eta * u);
        H = (e - 3.0 * F) / rr;
        K = (e / s + 5.0 * H) / rr;
    }
    const double a = e / s + H;
    for (int c = 0; c < 3; ++c)
        for (int j = 0; j < 3; ++j) {
            double t = -a * r[j] * D[c] - H * D[j] * r[c] + K * Dr * r[c] * r[j];
            if (c == j) t -= H * Dr;
            out[3 * c + j] = pref * t;
        }
}

// History write, position wrap (Lees-Edwards velocity jump in y when a mean
// shear is present) and the new state.  FP64.
__device__ __forceinline__ void finish_particle(const DevBox &B, int64_t p, const double xp[3],
                                                const double D[3], const double xn[3],
                                                double vn[3], double *hx, double *hdD,
                                                float *hdF) {
    const int64_t np = B.np;
    for (int d = 0; d < 3; ++d) {
        hx[d * np + p] = xp[d];
        if (hdD) hdD[d * np + p] = D[d];
        if (hdF) hdF[d * np + p] = (float)D[d];
    }
    for (int d = 0; d < 3; ++d) {
        double L = B.L[d];
        double fl = floor(xn[d] / L);
        double w = xn[d] - L * fl;
        int64_t k = (int64_t)fl;
        if (w >= L) { w -= L; k += 1; }
        if (w < 0.0) w = 0.0;
        B.x[d * np + p] = w;
        if (d == 1 && B.shear != 0.0 && k != 0) vn[0] -= (double)k * B.shear * L;
    }
    for (int d = 0; d < 3; ++d) B.v[d * np + p] = vn[d];
}

// Explicit Euler step with the memory terms of eq. force_particle: the added
// mass (second line) and the Basset term (third line), given u~ = u - v_self,
// lap u~ and grad u~ at x^n:
//   (m_p + m_f/2) dv/dt = S + m_f Du~/Dt + (m_f/2) dq/dt + B + m_p g_b,
//   S = m_p (u~ + fax lap u~ - v) / tau_p,   q = u~ + am_fax lap u~,
//   Du~/Dt = du~/dt + (u~ - v) . grad u~,
//   B = bs_k (w^n - w^{n-1}),   w = u~ + bs_fax lap u~ - v
// (the Basset memory integral over the last step only, with the bracket's
// derivative the difference over that step), with d/dt the difference along the
// particle path over the last step; each term is zero on the first step after
// it was switched on, and absent (m_f = 0, bs_k = 0) when off.  The fluid
// receives the hydrodynamic force D = m_p dv/dt - m_p g_b.  FP64.
__device__ __forceinline__ void update_particle_mem(const DevBox &B, int64_t p, double dt,
                                                    const double xp[3], const double ut[3],
                                                    const double lap[3], const double grad[9],
                                                    int am_valid, int bs_valid, double *hx,
                                                    double *hdD, float *hdF) {
#pragma clang fp contract(off)
    const int64_t np = B.np;
    const double t = (double)B.tau[p];
    const double mf = B.am_mf, mp = B.m_p;
    const bool am = mf != 0.0, bs = B.bs_k != 0.0;
    double v[3], q[3], S[3], w[3], D[3], xn[3], vn[3];
    for (int d = 0; d < 3; ++d) {
        v[d] = B.v[d * np + p];
        q[d] = ut[d] + B.am_fax * lap[d];
        S[d] = mp * (ut[d] + B.fax * lap[d] - v[d]) / t;
        w[d] = ut[d] + B.bs_fax * lap[d] - v[d];
    }
    for (int d = 0; d < 3; ++d) {
        double conv = 0.0, dut = 0.0, dq = 0.0, Bs = 0.0;
        if (am) {
            for (int j = 0; j < 3; ++j) conv += (ut[j] - v[j]) * grad[3 * d + j];
            dut = am_valid ? (ut[d] - B.am_hist[d * np + p]) / dt : 0.0;
            dq = am_valid ? (q[d] - B.am_hist[(3 + d) * np + p]) / dt : 0.0;
        }
        if (bs && bs_valid) Bs = B.bs_k * (w[d] - B.bs_hist[d * np + p]);
        const double Dm = dut + conv;
        const double acc = (S[d] + mf * Dm + 0.5 * mf * dq + Bs + mp * B.gb[d]) / (mp + 0.5 * mf);
        D[d] = S[d] + mf * Dm + 0.5 * mf * (dq - acc) + Bs;
        xn[d] = xp[d] + dt * v[d];
        vn[d] = v[d] + dt * acc;
    }
    for (int d = 0; d < 3; ++d) {
        if (am) {
            B.am_hist[d * np + p] = ut[d];
            B.am_hist[(3 + d) * np + p] = q[d];
        }
        if (bs) B.bs_hist[d * np + p] = w[d];
    }
    finish_particle(B, p, xp, D, xn, vn, hx, hdD, hdF);
}

// Drag, history write, explicit Euler and periodic wrap (Lees-Edwards velocity
// jump in y when a mean shear is present).  FP64.
__device__ __forceinline__ void update_particle(const DevBox &B, int64_t p, double dt,
                                                const double xp[3], const double up[3],
                                                const double vs[3], const double up2[3],
                                                const double vs2[3], double *hx, double *hdD,
                                                float *hdF) {
#pragma clang fp contract(off)
    const int64_t np = B.np;
    double t = (double)B.tau[p];
    double D[3], xn[3], vn[3];
    if (B.integ == 0) {
        // explicit Euler: drag at (x^n, v^n), positions with the old velocity
        for (int d = 0; d < 3; ++d) {
            double ut = up[d] - vs[d];
            double vd = B.v[d * np + p];
            D[d] = B.m_p * (ut - vd) / t;
            xn[d] = xp[d] + dt * vd;
            vn[d] = vd;
        }
        for (int d = 0; d < 3; ++d) {
            vn[d] += dt * D[d] / B.m_p;
            vn[d] += dt * B.gb[d];
        }
    } else if (B.integ == 2) {
        // Heun: stage 1 at (x^n, v^n), stage 2 at x* = x^n + dt v^n with
        // v* = v^n + dt a_1 (carrier and self term evaluated there by the
        // caller); the fluid gets the mean of the two stage drags
        for (int d = 0; d < 3; ++d) {
            const double v0 = B.v[d * np + p];
            const double ut1 = up[d] - vs[d];
            const double ut2 = up2[d] - vs2[d];
            const double d1 = (ut1 - v0) / t;
            const double vst = v0 + dt * (d1 + B.gb[d]);
            const double d2 = (ut2 - vst) / t;
            const double dm = 0.5 * (d1 + d2);
            D[d] = B.m_p * dm;
            xn[d] = xp[d] + 0.5 * dt * (v0 + vst);
            vn[d] = v0 + dt * (dm + B.gb[d]);
        }
    } else {
        // exponential integrator: dv/dt = (u~ - v)/tau + g_b solved exactly over
        // the step with u~ frozen; the fluid gets the step-averaged drag, the
        // momentum exchanged divided by dt
        const double e1 = -expm1(-dt / t);      // 1 - exp(-dt/tau)
        for (int d = 0; d < 3; ++d) {
            double ut = up[d] - vs[d];
            double vd = B.v[d * np + p];
            double w = ut + t * B.gb[d];         // velocity the particle relaxes to
            vn[d] = vd - (vd - w) * e1;
            xn[d] = xp[d] + dt * w + t * (vd - w) * e1;
            D[d] = B.m_p * (vn[d] - vd) / dt - B.m_p * B.gb[d];
        }
    }
    finish_particle(B, p, xp, D, xn, vn, hx, hdD, hdF);
}

}  // namespace erpp
