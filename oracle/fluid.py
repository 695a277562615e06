"""FP64 CPU oracle of the fluid step that consumes the ERPP forcing.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/`` (and nothing in the product
package).  Shares no code with the HIP library.

The step is the operator splitting of App. E (arXiv:1405.6969) for the
unsteady Stokes equation of the regularised disturbance (Sec. 2.3,
eq. velo_reg_eq) on a triply periodic box:

1. forcing step (eq. forcing_step):      u~ = u^n + dt f^n
2. diffusion step (eq. diffusion_step):  u* = heat semigroup of u~ over dt,
   i.e. the convolution with g(., dt), done exactly in Fourier space
3. projection step:                      solve lap(phi) = -div(u*), then
   u^{n+1} = u* + grad(phi)

Fourier conventions: nodes x_i = i L/N; wavenumbers k = 2 pi m / L with m the
signed FFT index.  The mean (k = 0) is untouched by steps 2 and 3, so the
total momentum grows by exactly dt * sum(f) per step.

Nyquist index of an even N (the paper is silent; this is a reading): the grid
derivative of the Nyquist cosine vanishes at every node, so the first
derivatives of the projection (div and grad, and the Poisson operator div grad
built from them) use k_d with that component set to zero.  The diffusion keeps
the true |k|^2.  The projection is then exactly idempotent, its result has zero
grid divergence, and it does not depend on the sign given to the Nyquist index.

Also here, for the validation of Sec. 3.1 (a constant force held at a fixed
point of a fluid initially at rest):

* ``fixed_force_velocity``: the closed form along the force axis
  (eq. ref_velo_f_fixed), from the time convolution of the unsteady Green
  tensor (App. B) with the force;
* ``impulse``: the total impulse rho_f * integral(u) of the periodic box,
  which by the statement around eq. impulse_def equals F0 t exactly.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def wavenumbers(n, L, derivative=False):
    """(kx, ky, kz) broadcastable over a rfftn spectrum of a [Nz][Ny][Nx] field:
    kz along axis 0, ky along axis 1, kx (half spectrum) along axis 2.  With
    derivative=True the Nyquist component of an even N is zero."""
    nx, ny, nz = (int(a) for a in n)
    Lx, Ly, Lz = (float(a) for a in L)
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx, d=Lx / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=Ly / ny)
    kz = 2.0 * np.pi * np.fft.fftfreq(nz, d=Lz / nz)
    if derivative:
        if nx % 2 == 0:
            kx[nx // 2] = 0.0
        if ny % 2 == 0:
            ky[ny // 2] = 0.0
        if nz % 2 == 0:
            kz[nz // 2] = 0.0
    return kx[None, None, :], ky[None, :, None], kz[:, None, None]


def fluid_step(n, L, nu, dt, u, f):
    """One App. E step of the periodic unsteady Stokes equation.

    u, f: [3][Nz][Ny][Nx] FP64 (x fastest).  Returns u^{n+1} (new array)."""
    u = np.asarray(u, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    nx, ny, nz = (int(a) for a in n)
    assert u.shape == (3, nz, ny, nx) and f.shape == u.shape
    kx, ky, kz = wavenumbers(n, L)
    k2 = kx * kx + ky * ky + kz * kz
    dx_, dy_, dz_ = wavenumbers(n, L, derivative=True)
    kd2 = dx_ * dx_ + dy_ * dy_ + dz_ * dz_

    # 1. forcing step: explicit increment over dt
    ut = u + dt * f
    # 2. diffusion step: the heat kernel over dt multiplies mode k by exp(-nu k^2 dt)
    U = np.fft.rfftn(ut, axes=(1, 2, 3))
    U = U * np.exp(-nu * k2 * dt)
    # 3. projection step: lap(phi) = -div(u*)  ->  -kd^2 phi^ = -i kd.u*^,
    #    then u = u* + grad(phi)
    div = 1j * (dx_ * U[0] + dy_ * U[1] + dz_ * U[2])
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(kd2 > 0.0, div / np.where(kd2 > 0.0, kd2, 1.0), 0.0)
    U[0] = U[0] + 1j * dx_ * phi
    U[1] = U[1] + 1j * dy_ * phi
    U[2] = U[2] + 1j * dz_ * phi
    return np.fft.irfftn(U, s=(nz, ny, nx), axes=(1, 2, 3))


def fixed_force_velocity(r, t, nu, rho_f, F0=1.0):
    """Velocity component along a constant point force F0 switched on at t = 0
    in an unbounded fluid at rest, at distance r on the force axis
    (eq. ref_velo_f_fixed): with mu = rho_f nu and eta = r / sqrt(4 nu t),
    u = F0 / (4 pi mu r) [erf(eta) / (2 eta^2) - erf(eta)
                          - exp(-eta^2) / (sqrt(pi) eta) + 1]."""
    r = np.asarray(r, dtype=np.float64)
    mu = rho_f * nu
    eta = r / np.sqrt(4.0 * nu * t)
    e = erf(eta)
    br = e / (2.0 * eta * eta) - e - np.exp(-eta * eta) / (np.sqrt(np.pi) * eta) + 1.0
    return F0 / (4.0 * np.pi * mu * r) * br


def impulse(u, dV, rho_f):
    """Total impulse rho_f * sum(u) dV of a periodic field [3][...] (3-vector)."""
    u = np.asarray(u, dtype=np.float64)
    return rho_f * dV * u.reshape(3, -1).sum(axis=1)
