// plain.hip -- ERPP_F64_PLAIN path: every stage in FP64, no binning, the
// forcing accumulated with FP64 global atomics.  This is the straightforward
// single-pass formulation the tiled FP32 path is measured against.
#include <hip/hip_runtime.h>

#include "erpp_device.hpp"
#include "erpp_internal.hpp"

namespace erpp {
namespace {

// Per particle: FP64 cell/offset of X^{n-M}, amplitude -D/rho_f and the lattice
// normalisation Z = dV * sum of exp(-r^2/2 sigma^2) over the 3-sigma sphere.
__global__ void __launch_bounds__(kBlock) k_plain_eval(const DevBox *__restrict__ Bs, int nbox,
                                                       const int64_t *__restrict__ stepp, int M,
                                                       double *__restrict__ pamp,
                                                       double *__restrict__ pphi,
                                                       int32_t *__restrict__ pbase,
                                                       int64_t npt) {
    const int64_t n = *stepp;
    if (n < M) return;
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t np = B.np;
    const int64_t slot = (n - M) % (M + 1);
    const double *X = B.ring_x + slot * 3 * np;
    const double *D = (const double *)B.ring_d + slot * 3 * np;
    int b[3];
    double ph[3];
    for (int d = 0; d < 3; ++d) cell_of(X[d * np + p], B.L[d], B.dx[d], B.n[d], b[d], ph[d]);
    double Z = 0.0;
    for (int mz = B.mlo[2]; mz <= B.mhi[2]; ++mz) {
        for (int my = B.mlo[1]; my <= B.mhi[1]; ++my) {
            for (int mx = B.mlo[0]; mx <= B.mhi[0]; ++mx) {
#pragma clang fp contract(off)
                double ddx = ((double)mx - ph[0]) * B.dx[0];
                double dy = ((double)my - ph[1]) * B.dx[1];
                double dz = ((double)mz - ph[2]) * B.dx[2];
                double r2 = ddx * ddx + dy * dy + dz * dz;
                if (r2 <= B.R2) Z += exp(-r2 / B.two_s2);
            }
        }
    }
    const int64_t q = B.poff + p;
    pamp[q] = -D[p] / B.rho_f;
    pamp[npt + q] = -D[np + p] / B.rho_f;
    pamp[2 * npt + q] = -D[2 * np + p] / B.rho_f;
    pamp[3 * npt + q] = Z * B.dV;
    for (int d = 0; d < 3; ++d) {
        pphi[d * npt + q] = ph[d];
        pbase[d * npt + q] = b[d];
    }
}

__global__ void __launch_bounds__(kBlock) k_zero64(double *__restrict__ f, int64_t cnt) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * kBlock)
        f[i] = 0.0;
}

// One thread per (particle, stencil row (my, mz)); FP64 global atomics.
__global__ void __launch_bounds__(kBlock) k_plain_scatter(const DevBox *__restrict__ Bs, int nbox,
                                                          const int64_t *__restrict__ stepp,
                                                          int M,
                                                          const double *__restrict__ pamp,
                                                          const double *__restrict__ pphi,
                                                          const int32_t *__restrict__ pbase,
                                                          int64_t npt) {
    const int64_t n = *stepp;
    if (n < M) return;
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_r; });
    const DevBox &B = Bs[bi];
    const int64_t idx = (int64_t)(blockIdx.x - B.blk_r) * kBlock + threadIdx.x;
    if (idx >= B.np * B.rows) return;
    const int64_t p = idx / B.rows;
    const int r = (int)(idx - p * B.rows);
    const int ny = B.mhi[1] - B.mlo[1] + 1;
    const int my = B.mlo[1] + r % ny;
    const int mz = B.mlo[2] + r / ny;
    const int64_t q = B.poff + p;
    const double phx = pphi[q], phy = pphi[npt + q], phz = pphi[2 * npt + q];
    const int b0 = pbase[q], b1 = pbase[npt + q], b2 = pbase[2 * npt + q];
    const double a0 = pamp[q], a1 = pamp[npt + q], a2 = pamp[2 * npt + q];
    const double Z = pamp[3 * npt + q];
    int j = b1 + my, k = b2 + mz;
    j = (j % B.n[1] + B.n[1]) % B.n[1];
    k = (k % B.n[2] + B.n[2]) % B.n[2];
    const int64_t Nx = B.n[0];
    const int64_t ng = Nx * B.n[1] * B.n[2];
    const int64_t rowoff = ((int64_t)k * B.n[1] + j) * Nx;
    double *f = (double *)B.f;
    for (int mx = B.mlo[0]; mx <= B.mhi[0]; ++mx) {
        double r2;
        {
#pragma clang fp contract(off)
            double ddx = ((double)mx - phx) * B.dx[0];
            double dy = ((double)my - phy) * B.dx[1];
            double dz = ((double)mz - phz) * B.dx[2];
            r2 = ddx * ddx + dy * dy + dz * dz;
        }
        if (r2 > B.R2) continue;
        const double w = exp(-r2 / B.two_s2) / Z;
        int i = b0 + mx;
        i = (i % B.n[0] + B.n[0]) % B.n[0];
        const int64_t node = rowoff + i;
        atomicAdd(&f[node], a0 * w);
        atomicAdd(&f[ng + node], a1 * w);
        atomicAdd(&f[2 * ng + node], a2 * w);
    }
}

// Carrier, self term and Faxen terms of particle p at position pos (FP64):
// up = u(pos) + fax lap u(pos), vs = v_self(pos) + fax lap v_self(pos).
__device__ __forceinline__ void plain_terms(const DevBox &B, int64_t p, int64_t n, int M,
                                            int selfc, const double pos[3], double up[3],
                                            double vs[3]) {
    const int64_t np = B.np;
    trilinear<double>(B, (const double *)B.u, pos, up);
    vs[0] = vs[1] = vs[2] = 0.0;
    if (selfc && n >= M + 1) {
        const int64_t ss = (n - 1 - M) % (M + 1);
        const double *Xs = B.ring_x + ss * 3 * np;
        const double *Ds = (const double *)B.ring_d + ss * 3 * np;
        double r[3], D[3];
        for (int d = 0; d < 3; ++d) {
            double rd = pos[d] - Xs[d * np + p];
            rd -= B.L[d] * rint(rd / B.L[d]);
            r[d] = rd;
            D[d] = Ds[d * np + p];
        }
        self_disturbance64(r, D, B.s2s, B.pref, vs);
        if (B.fax != 0.0) {
            double ls[3];
            self_laplacian64(r, D, B.s2s, B.pref, ls);
            for (int d = 0; d < 3; ++d) vs[d] += B.fax * ls[d];
        }
    }
    if (B.fax != 0.0) {
        // Faxen term (a_p^2/6) lap u~, grid part (the self part is above)
        double lu[3];
        trilinear_laplacian<double>(B, (const double *)B.u, pos, lu);
        for (int d = 0; d < 3; ++d) up[d] += B.fax * lu[d];
    }
}

// Memory terms (added mass, Basset): u~ = u - v_self, lap u~ and grad u~ at pos, each the
// interpolated carrier stencil minus the closed form of the self-disturbance of
// the last injection (FP64).
__device__ void plain_am_terms(const DevBox &B, int64_t p, int64_t n, int M, int selfc,
                               const double pos[3], double ut[3], double lap[3],
                               double grad[9]) {
    const int64_t np = B.np;
    const double *u = (const double *)B.u;
    trilinear<double>(B, u, pos, ut);
    trilinear_stencils<double, true, true>(B, u, pos, lap, grad);
    if (selfc && n >= M + 1) {
        const int64_t ss = (n - 1 - M) % (M + 1);
        const double *Xs = B.ring_x + ss * 3 * np;
        const double *Ds = (const double *)B.ring_d + ss * 3 * np;
        double r[3], D[3], vs[3], ls[3], gs[9];
        for (int d = 0; d < 3; ++d) {
            double rd = pos[d] - Xs[d * np + p];
            rd -= B.L[d] * rint(rd / B.L[d]);
            r[d] = rd;
            D[d] = Ds[d * np + p];
        }
        self_disturbance64(r, D, B.s2s, B.pref, vs);
        self_laplacian64(r, D, B.s2s, B.pref, ls);
        self_gradient64(r, D, B.s2s, B.pref, gs);
        for (int d = 0; d < 3; ++d) {
            ut[d] -= vs[d];
            lap[d] -= ls[d];
        }
        for (int q = 0; q < 9; ++q) grad[q] -= gs[q];
    }
}

__global__ void __launch_bounds__(kBlock) k_plain_update(const DevBox *__restrict__ Bs, int nbox,
                                                         const int64_t *__restrict__ stepp, int M,
                                                         double dt, int selfc) {
    const int bi = box_of_block(Bs, nbox, blockIdx.x, [](const DevBox &b) { return b.blk_p; });
    const DevBox &B = Bs[bi];
    const int64_t p = (int64_t)(blockIdx.x - B.blk_p) * kBlock + threadIdx.x;
    if (p >= B.np) return;
    const int64_t n = *stepp;
    const int64_t np = B.np;
    double xp[3] = {B.x[p], B.x[np + p], B.x[2 * np + p]};
    const int64_t sw = n % (M + 1);
    if (B.am_mf != 0.0 || B.bs_k != 0.0) {
        double ut[3], lap[3], grad[9];
        plain_am_terms(B, p, n, M, selfc, xp, ut, lap, grad);
        update_particle_mem(B, p, dt, xp, ut, lap, grad, *B.am_valid, *B.bs_valid,
                            B.ring_x + sw * 3 * np, (double *)B.ring_d + sw * 3 * np, nullptr);
        return;
    }
    double up[3], vs[3];
    plain_terms(B, p, n, M, selfc, xp, up, vs);
    double up2[3] = {0.0, 0.0, 0.0}, vs2[3] = {0.0, 0.0, 0.0};
    if (B.integ == 2) {
        // Heun's second stage at x* = x^n + dt v^n
        const double xs[3] = {xp[0] + dt * B.v[p], xp[1] + dt * B.v[np + p],
                              xp[2] + dt * B.v[2 * np + p]};
        plain_terms(B, p, n, M, selfc, xs, up2, vs2);
    }
    update_particle(B, p, dt, xp, up, vs, up2, vs2, B.ring_x + sw * 3 * np,
                    (double *)B.ring_d + sw * 3 * np, nullptr);
}

}  // namespace

hipError_t plain_stage(erpp_plan *P, int k, hipStream_t st) {
    switch (k) {
        case 0:
            for (int b = 0; b < P->nbox; ++b) {
                const DevBox &H = P->hbox[b];
                const int64_t cnt = 3 * (int64_t)H.n[0] * H.n[1] * H.n[2];
                int64_t blocks = (cnt + kBlock - 1) / kBlock;
                if (blocks > 65536) blocks = 65536;
                hipLaunchKernelGGL(k_zero64, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                                   (double *)H.f, cnt);
            }
            break;
        case 1:
            break;
        case 2:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_plain_eval, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step, P->M, P->s.pamp, P->s.pphi,
                                   P->s.pbase, P->np_total);
            break;
        case 3:
            if (P->np_total > 0)
                hipLaunchKernelGGL(k_plain_scatter, dim3((unsigned)P->pblocks_rows), dim3(kBlock),
                                   0, st, P->dbox, P->nbox, P->s.step, P->M, P->s.pamp,
                                   P->s.pphi, P->s.pbase, P->np_total);
            break;
        case 4:
            if (P->np_total > 0) {
                hipLaunchKernelGGL(k_plain_update, dim3((unsigned)P->pblocks), dim3(kBlock), 0, st,
                                   P->dbox, P->nbox, P->s.step, P->M, P->dt, P->self_correction);
                for (const auto &B : P->hbox)
                    if (B.am_mf != 0.0 || B.bs_k != 0.0) return mark_memory_terms(P, st);
            }
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t plain_scatter_stages(erpp_plan *P, hipStream_t st) {
    for (int k = 0; k < 4; ++k) {
        hipError_t e = plain_stage(P, k, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t plain_update_stage(erpp_plan *P, hipStream_t st) { return plain_stage(P, 4, st); }

}  // namespace erpp
