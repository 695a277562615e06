"""Pins of the fluid-step oracle (oracle/fluid.py) against facts fixed by the
paper and by mathematics: Fourier modes with closed-form evolution, the
projection of gradients, the momentum (impulse) balance, the App. E closed form
of the disturbance of one regularised impulse (eq. disturbance_velo, here in
its App. B Green-tensor form), and the constant-force solution of Sec. 3.1
(eq. ref_velo_f_fixed) through its limits and its time derivative."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute, fluid
from helpers import closed_form_sum, grid, min_image, periodic_gaussian


N_ANISO = (12, 10, 8)
L_ANISO = (3.0, 2.5, 1.7)


@pytest.mark.parametrize("m,A", [((2, -1, 3), None), ((0, 4, -1), None), ((6, 0, 0), (0.0, 1.0, 0.5)),
                                 ((1, -3, 2), None), ((5, 1, 0), None)])
def test_f1_solenoidal_mode_decays_by_heat_factor(m, A):
    """A divergence-free Fourier mode A cos(k.x + 0.3), A.k = 0, is an
    eigenfunction of the step with f = 0: diffusion multiplies it by
    exp(-nu |k|^2 dt) and the projection leaves it.  Distinct wavenumbers per
    axis and an anisotropic box catch swapped axes; m = (6,0,0) is the Nyquist
    index of Nx = 12 (transverse amplitude)."""
    nu, dt = 0.07, 0.3
    k = np.array([2 * math.pi * m[i] / L_ANISO[i] for i in range(3)])
    if A is None:
        A = np.cross(k, [0.3, -0.2, 0.9])
    A = np.asarray(A, dtype=np.float64)
    assert abs(A @ k) < 1e-12 * np.linalg.norm(A) * np.linalg.norm(k)
    x, y, z = grid(N_ANISO, L_ANISO)
    ph = np.cos(k[0] * x + k[1] * y + k[2] * z + 0.3)
    u0 = A[:, None, None, None] * ph[None]
    u1 = fluid.fluid_step(N_ANISO, L_ANISO, nu, dt, u0, np.zeros_like(u0))
    want = u0 * math.exp(-nu * (k @ k) * dt)
    assert np.max(np.abs(u1 - want)) < 1e-13 * np.max(np.abs(u0))


def test_f1b_nyquist_rule():
    """Nyquist reading: the grid derivative of the Nyquist cosine (-1)^j is zero
    at every node, so such a factor takes no part in div/grad of the projection,
    while the diffusion uses the full |k|^2.
    (a) (cos(pi i), 0, 0) has zero grid divergence: it only decays.
    (b) A cos(k1 x + 0.3) (-1)^j (y index at Nyquist) loses the x-component of A
        (its k_d is (k1, 0, 0)) and decays with k1^2 + k_Ny^2."""
    nu, dt = 0.1, 0.2
    x, y, z = grid(N_ANISO, L_ANISO)
    kNx = math.pi * N_ANISO[0] / L_ANISO[0]
    kNy = math.pi * N_ANISO[1] / L_ANISO[1]
    u0 = np.zeros((3,) + x.shape)
    u0[0] = np.cos(kNx * x)
    u1 = fluid.fluid_step(N_ANISO, L_ANISO, nu, dt, u0, np.zeros_like(u0))
    assert np.max(np.abs(u1 - u0 * math.exp(-nu * kNx ** 2 * dt))) < 1e-14
    k1 = 2 * math.pi / L_ANISO[0]
    A = np.array([0.4, 1.0, -0.7])
    ph = np.cos(k1 * x + 0.3) * np.cos(kNy * y)
    u0 = A[:, None, None, None] * ph[None]
    u1 = fluid.fluid_step(N_ANISO, L_ANISO, nu, dt, u0, np.zeros_like(u0))
    want = np.array([0.0, 1.0, -0.7])[:, None, None, None] * ph[None] \
        * math.exp(-nu * (k1 ** 2 + kNy ** 2) * dt)
    assert np.max(np.abs(u1 - want)) < 1e-14


def test_f2_gradient_forcing_is_projected_out():
    """f = grad(psi) + B cos(k'.x) with B.k' = 0 from rest: the gradient is
    removed by the projection step, the solenoidal part gains dt B cos(k'.x)
    times exp(-nu |k'|^2 dt)."""
    nu, dt = 0.05, 0.4
    k = np.array([2 * math.pi * v / L for v, L in zip((3, -2, 1), L_ANISO)])
    kp = np.array([2 * math.pi * v / L for v, L in zip((1, 2, -2), L_ANISO)])
    B = np.cross(kp, [1.0, 0.4, -0.3])
    x, y, z = grid(N_ANISO, L_ANISO)
    # psi = 0.7 sin(k.x): grad psi = 0.7 k cos(k.x)
    gpsi = 0.7 * k[:, None, None, None] * np.cos(k[0] * x + k[1] * y + k[2] * z)[None]
    sol = B[:, None, None, None] * np.cos(kp[0] * x + kp[1] * y + kp[2] * z)[None]
    u1 = fluid.fluid_step(N_ANISO, L_ANISO, nu, dt, np.zeros_like(sol), gpsi + sol)
    want = dt * sol * math.exp(-nu * (kp @ kp) * dt)
    assert np.max(np.abs(u1 - want)) < 1e-13 * np.max(np.abs(gpsi))


def test_f3_uniform_forcing_and_impulse_balance():
    """Sec. 3.1: in the periodic box the impulse rho_f * integral(u) grows by the
    applied force times the time.  A uniform f adds exactly dt f; for random
    u and f the discrete momentum grows by rho_f dV dt sum(f) per step."""
    rng = np.random.default_rng(11)
    nu, dt, rho = 0.02, 0.1, 1.7
    f = np.broadcast_to(np.array([0.3, -1.1, 2.0])[:, None, None, None], (3, 8, 10, 12)).copy()
    u1 = fluid.fluid_step(N_ANISO, L_ANISO, nu, dt, np.zeros_like(f), f)
    assert np.max(np.abs(u1 - dt * f)) < 1e-15
    dV = np.prod(L_ANISO) / np.prod(N_ANISO)
    u = rng.standard_normal((3, 8, 10, 12))
    I0 = fluid.impulse(u, dV, rho)
    applied = np.zeros(3)
    for _ in range(5):
        f = rng.standard_normal(u.shape)
        applied += rho * dV * dt * f.reshape(3, -1).sum(axis=1)
        u = fluid.fluid_step(N_ANISO, L_ANISO, nu, dt, u, f)
    assert np.allclose(fluid.impulse(u, dV, rho), I0 + applied, rtol=0, atol=1e-12)


@pytest.mark.parametrize("K", [1, 8])
def test_f4_regularised_impulse_matches_app_e_closed_form(K):
    """App. E: starting from rest, a forcing step with the regularised impulse
    -(dt/rho_f) D g(x - x_p, eps_R), exact diffusion over dt and the projection
    give eq. disturbance_velo with sigma^2 = sigma_R^2 + 2 nu dt (here in the
    App. B tensor form).  The forcing is the untruncated Gaussian, so the only
    difference is the periodic box: the mean flow -K dt D/(rho_f V) (the impulse
    spread over the box) and the field of the periodic images, whose size is of
    the same order; both are bounded by twice the mean."""
    n = (64, 56, 48)
    L = tuple(float(a) for a in n)
    sR, nu, dt, rho = 1.5, 0.5, 0.25, 1.3
    D = np.array([0.3, -0.7, 0.5])
    xp = np.array([20.3, 17.6, 15.2])
    f = -(D[:, None, None, None] * periodic_gaussian(n, L, xp, sR)[None]) / rho
    u = np.zeros_like(f)
    for _ in range(K):
        u = fluid.fluid_step(n, L, nu, dt, u, f)
    r = min_image(n, L, xp)
    ref, m = closed_form_sum(r, D, sR, nu, dt, rho, K)
    mean = -K * dt * D / (rho * np.prod(L))
    err = np.abs(u - ref - mean[:, None, None, None])[:, m]
    assert err.max() < 2.0 * np.abs(mean).max()
    # the bound is tight enough to matter: 1% of the peak disturbance
    assert 2.0 * np.abs(mean).max() < 0.01 * np.abs(ref).max()
    assert np.allclose(fluid.impulse(u, 1.0, rho), -K * dt * D, atol=1e-13)


def test_f5_fixed_force_closed_form_limits():
    """eq. ref_velo_f_fixed: for t -> infinity it tends to the steady Stokeslet
    on its axis, F/(4 pi mu r); for r >> sqrt(nu t) to the irrotational field of
    the impulse F t on its axis, F t/(2 pi rho_f r^3)."""
    nu, rho = 0.8, 1.4
    mu = nu * rho
    r = np.array([0.5, 1.0, 2.0])
    steady = fluid.fixed_force_velocity(r, 1e12, nu, rho)
    assert np.allclose(steady, 1 / (4 * math.pi * mu * r), rtol=1e-5)
    t = 1e-3
    far = np.array([3.0, 5.0])
    assert np.allclose(fluid.fixed_force_velocity(far, t, nu, rho), t / (2 * math.pi * rho * far ** 3),
                       rtol=1e-9)


@pytest.mark.parametrize("t", [0.01, 0.2, 3.0])
def test_f6_fixed_force_rate_is_the_unsteady_green_tensor(t):
    """The constant-force solution is the time integral of the unsteady Green
    tensor (App. B, eq. green_tensor) applied to F, so its time derivative on
    the axis equals that tensor at sigma^2 = 2 nu t (central differences)."""
    nu, rho = 0.6, 1.2
    r = np.array([0.05, 0.3, 1.0, 2.5])
    h = 1e-4 * t
    du = (fluid.fixed_force_velocity(r, t + h, nu, rho)
          - fluid.fixed_force_velocity(r, t - h, nu, rho)) / (2 * h)
    rr = np.stack([r, 0 * r, 0 * r])
    # the helper returns -dt G D / rho_f; a force F on the fluid is D = -F
    G = brute.green_tensor_velocity(rr, np.array([[-1.0], [0.0], [0.0]]), math.sqrt(2 * nu * t),
                                    1.0, rho)[0]
    assert np.allclose(du, G, rtol=2e-7)


def test_f7_stepped_impulses_converge_to_fixed_force_solution():
    """A constant force F applied through the regularised forcing from t = 0 is,
    in the continuum, u_ref(t + eps_R) - u_ref(eps_R) (the Green tensor
    convolved with g(eps_R) is the Green tensor eps_R later).  The App. E
    stepping replaces the time integral by a sum over steps; its error must be
    first order in dt."""
    nu, rho, eps = 1.0, 1.0, 0.01
    sR = math.sqrt(2 * nu * eps)
    t = 0.05
    r = np.array([0.5, 1.0, 2.0, 4.0, 8.0]) * sR
    rr = np.stack([r, 0 * r, 0 * r])
    F = np.array([-1.0, 0.0, 0.0])      # D = -F
    cont = fluid.fixed_force_velocity(r, t + eps, nu, rho) - fluid.fixed_force_velocity(r, eps, nu, rho)
    errs = []
    for K in (50, 100, 200):
        dt = t / K
        s, _ = closed_form_sum(rr, F, sR, nu, dt, rho, K)
        errs.append(np.max(np.abs(s[0] - cont) / cont))
    assert errs[-1] < 0.01
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


def test_f8_fixed_force_through_the_erpp_forcing():
    """Sec. 3.1 with the method's own forcing: a constant force at a fixed point,
    deposited with the 3 sigma_R cut and the lattice normalisation, stepped from
    rest.  The impulse equals F t exactly; the field follows the stepped App. E
    closed form within 3% of its peak (the cut of the Gaussian, largest next to
    the particle) and, beyond 6 sigma_R, within twice the periodic mean flow."""
    nu, rho, eps, M = 1.0, 1.0, 0.01, 10
    sR = math.sqrt(2 * nu * eps)
    N, Lb = 48, 2 * math.pi
    n, L, dx = (N,) * 3, (Lb,) * 3, Lb / N
    dt = eps / M
    P = oracle.make_params(n, L, 1, 1.0, rho, nu, sR, 3.0, 0.0, M, dt)
    xp = np.array([N // 2 * dx + 0.3 * dx, N // 2 * dx, N // 2 * dx])
    D = np.array([-1.0, 0.0, 0.0])
    f = oracle.deposit(P, xp[:, None], D[:, None])
    K = 50
    u = np.zeros_like(f)
    for _ in range(K):
        u = fluid.fluid_step(n, L, nu, dt, u, f)
    assert np.allclose(fluid.impulse(u, dx ** 3, rho), [K * dt, 0, 0], atol=1e-13)
    r = min_image(n, L, xp)
    ref, m = closed_form_sum(r, D, sR, nu, dt, rho, K)
    mean = K * dt / (rho * Lb ** 3)
    err = np.abs(u - ref)
    err[0] = np.abs(u[0] - ref[0] - mean)
    rn = np.sqrt(np.sum(r * r, axis=0))
    assert err[:, m].max() < 0.03 * np.abs(ref).max()
    far = m & (rn > 6 * sR)
    assert err[:, far].max() < 2.0 * mean
