"""Pins of the oracle's added-mass terms (eq. force_particle, second line) and of
the two new ingredients they need: the gradient of the App. E disturbance (the
self part of grad u~) and the interpolated nodal gradient of the carrier.

What fixes each value:
* am1  the closed-form gradient equals central differences of the closed-form
       disturbance itself (a separately pinned oracle function), on both sides of
       the series/closed-form switch, and its trace vanishes (solenoidal field);
* am2  the interpolated central-difference gradient of a trigonometric field is
       second-order accurate, and the mean shear adds S to d u_x / d y;
* am3  settling from rest in fluid at rest: the relaxation time becomes
       tau_p (m_p + m_f/2) / m_p (first-order convergence in dt) and the terminal
       velocity stays tau_p g_b;
* am4  a transverse wave whose amplitude grows linearly in time: the steady slip
       of the Maxey-Riley equation with added mass, Faxen corrections a^2/6
       (drag) and a^2/10 (added mass), in closed form;
* am5  a Taylor-Green carrier: the convective part of D u~/Dt converges at second
       order to (u . grad) u, which differs from the transposed product.
"""
import math

import numpy as np
import pytest

import oracle

RHO, NU = 1.0, 0.1


def _params(n, L, m_p, sigma, dt, a_am, a_p=0.0, self_correction=0, g=(0.0, 0.0, 0.0),
            shear=0.0, integrator=0, M=2):
    return oracle.make_params(n, L, 1, m_p, RHO, NU, sigma, 3.0, shear, M, dt,
                              self_correction, g=g, integrator=integrator, a_p=a_p, a_am=a_am)


@pytest.mark.parametrize("eta", [0.0, 0.05, 0.2, 0.29, 0.31, 0.6, 1.3, 2.7])
def test_am1_self_gradient_is_the_derivative_of_the_disturbance(eta):
    P = _params((16,) * 3, (1.0,) * 3, 1.0, 0.1, 1e-3, 0.0)
    s = math.sqrt(P.sigma ** 2 + 2 * P.nu * P.dt)
    rng = np.random.default_rng(int(eta * 100))
    dirn = rng.standard_normal(3)
    dirn /= np.linalg.norm(dirn)
    r = dirn * eta * math.sqrt(2) * s
    X0 = np.full((3, 1), 0.5)
    D = rng.standard_normal((3, 1))
    x = X0 + r[:, None]
    gs = oracle.self_gradient(P, x, X0, D)[:, :, 0]
    h = 1e-4 * s
    fd = np.empty((3, 3))
    for j in range(3):
        e = np.zeros((3, 1))
        e[j] = h
        fd[:, j] = (oracle.self_disturbance(P, x + e, X0, D) -
                    oracle.self_disturbance(P, x - e, X0, D))[:, 0] / (2 * h)
    scale = np.max(np.abs(fd))
    assert np.max(np.abs(gs - fd)) <= 1e-7 * scale
    assert abs(np.trace(gs)) <= 1e-12 * scale


def test_am2_grid_gradient_second_order_and_shear():
    errs = []
    for N in (32, 64, 128):
        L = (2 * math.pi,) * 3
        P = _params((N,) * 3, L, 1.0, 1.5 * L[0] / N, 1e-3, 0.0)
        ax = np.arange(N) * (L[0] / N)
        Zg, Yg, Xg = np.meshgrid(ax, ax, ax, indexing="ij")
        u = np.stack([np.sin(Xg) * np.cos(2 * Yg), np.cos(Yg + Zg), np.sin(3 * Zg) * np.cos(Xg)])
        rng = np.random.default_rng(3)
        x = rng.uniform(0, L[0], (3, 40))
        gu = oracle.grid_gradient(P, u, x)
        X, Y, Z = x
        ex = np.zeros((3, 3, 40))
        ex[0, 0] = np.cos(X) * np.cos(2 * Y)
        ex[0, 1] = -2 * np.sin(X) * np.sin(2 * Y)
        ex[1, 1] = -np.sin(Y + Z)
        ex[1, 2] = -np.sin(Y + Z)
        ex[2, 0] = -np.sin(3 * Z) * np.sin(X)
        ex[2, 2] = 3 * np.cos(3 * Z) * np.cos(X)
        errs.append(np.max(np.abs(gu - ex)))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    # the mean shear U_x = S (y - Ly/2) adds S to d u_x / d y and nothing else
    P0 = _params((16,) * 3, (1.0,) * 3, 1.0, 0.1, 1e-3, 0.0)
    Ps = _params((16,) * 3, (1.0,) * 3, 1.0, 0.1, 1e-3, 0.0, shear=0.7)
    u = np.random.default_rng(4).standard_normal((3, 16, 16, 16))
    x = np.random.default_rng(5).uniform(0, 1, (3, 7))
    d = oracle.grid_gradient(Ps, u, x) - oracle.grid_gradient(P0, u, x)
    want = np.zeros_like(d)
    want[0, 1] = 0.7
    assert np.allclose(d, want, rtol=0, atol=1e-14)


def _settle(dt, T, m_p, tau, a_am, gb):
    N, L = 16, 1.0
    P = _params((N,) * 3, (L,) * 3, m_p, 0.1, dt, a_am, g=(gb, 0.0, 0.0))
    run = oracle.Run(P, np.zeros((3, N, N, N)), np.full((3, 1), 0.5), np.zeros((3, 1)),
                     np.array([tau], np.float32))
    K = int(round(T / dt))
    for _ in range(K):
        run.step(want_f=False)
    return run.v[0, 0], K * dt


def test_am3_settling_relaxation_time_with_added_mass():
    tau = float(np.float32(0.05))
    a = 0.05
    m_f = RHO * 4 / 3 * math.pi * a ** 3
    m_p = 2.0 * m_f                               # rho_p = 2 rho_f: added mass matters
    gb = 3.0
    taup = tau * (m_p + 0.5 * m_f) / m_p
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        v, t = _settle(dt, 0.1, m_p, tau, a, gb)
        errs.append(v - tau * gb * (1 - math.exp(-t / taup)))
    assert 1.9 < errs[0] / errs[1] < 2.1 and 1.9 < errs[1] / errs[2] < 2.1
    assert abs(errs[2]) < 2e-3 * tau * gb
    # terminal velocity tau_p g_b, independent of the added mass
    v, _ = _settle(2e-3, 2.0, m_p, tau, a, gb)
    assert abs(v / (tau * gb) - 1) < 1e-12
    # without the term the relaxation time is tau_p: the two differ clearly
    v0, t = _settle(5e-4, 0.1, m_p, tau, 0.0, gb)
    assert abs(v0 - tau * gb * (1 - math.exp(-t / tau))) < 2e-3 * tau * gb
    assert abs(v0 - v) > 0.05 * tau * gb


@pytest.mark.parametrize("a_p_on", [False, True])
def test_am4_steady_slip_in_an_accelerating_wave(a_p_on):
    """u = (0, alpha t sin(k x), 0): no convective term, the particle moves in y
    only, and at the particle u~ = alpha t s_p, lap u~ = -k_h^2 u~ (k_h^2 =
    (2 - 2 cos k dx) / dx^2, exact for the nodal stencil and kept by the
    interpolation).  The Maxey-Riley equation then has a steady state with
    dv/dt = (1 - k6) alpha s_p and slip (1 - k6) u~ - v equal to
      tau_p alpha s_p [(m_p + m_f/2)(1 - k6) - m_f - (m_f/2)(1 - k10)] / m_p,
    k6 = (a_p^2/6) k_h^2, k10 = (a^2/10) k_h^2."""
    N, L = 32, 2 * math.pi
    dx = L / N
    k = 3.0
    a = 0.15
    m_f = RHO * 4 / 3 * math.pi * a ** 3
    m_p = 1.5 * m_f
    tau = float(np.float32(0.02))
    dt, alpha = 1e-3, 2.0
    a_p = a if a_p_on else 0.0
    P = _params((N,) * 3, (L,) * 3, m_p, 2 * dx, dt, a, a_p=a_p)
    ax = np.arange(N) * dx
    wave = np.zeros((3, N, N, N))
    wave[1] = np.sin(k * ax)[None, None, :]
    x0 = np.array([[1.234], [2.0], [3.0]])
    run = oracle.Run(P, 0 * wave, x0, np.zeros((3, 1)), np.array([tau], np.float32))
    K = 1000                                      # transient factor 0.9625^K < 1e-16
    for n in range(K):
        run.u = alpha * n * dt * wave
        run.step(want_f=False)
    sp = oracle.gather(P, wave, x0)[1, 0]
    kh2 = (2 - 2 * math.cos(k * dx)) / dx ** 2
    k6 = a_p ** 2 / 6 * kh2
    k10 = a ** 2 / 10 * kh2
    ut = alpha * (K - 1) * dt * sp                # u~ seen by the last step
    vK = run.v[1, 0]
    # slip measured against the field of the last step, advanced by one step
    slip = (1 - k6) * ut - (vK - (1 - k6) * alpha * dt * sp)
    want = tau * alpha * sp * ((m_p + 0.5 * m_f) * (1 - k6) - m_f - 0.5 * m_f * (1 - k10)) / m_p
    assert abs(run.x[0, 0] - x0[0, 0]) < 1e-15 and run.v[0, 0] == 0.0
    assert abs(slip / want - 1) < 1e-9
    # a^2/6 in place of a^2/10 in the added-mass term would move the slip by
    wrong = tau * alpha * sp * (0.5 * m_f * (a ** 2 / 6 - a ** 2 / 10) * kh2) / m_p
    assert abs(wrong) > 1e-4 * abs(want)


def test_am5_convective_term_is_u_dot_grad_u():
    a = 0.05
    m_f = RHO * 4 / 3 * math.pi * a ** 3
    m_p = 3 * m_f
    tau = float(np.float32(0.05))
    dt = 1e-4
    x0 = np.array([[0.7], [2.1], [1.3]])
    errs = []
    for N in (16, 32, 64):
        L = 2 * math.pi
        ax = np.arange(N) * (L / N)
        Zg, Yg, Xg = np.meshgrid(ax, ax, ax, indexing="ij")
        u = np.stack([np.sin(Xg) * np.cos(Yg), -np.cos(Xg) * np.sin(Yg), 0 * Xg])
        P = _params((N,) * 3, (L,) * 3, m_p, 2 * L / N, dt, a)
        run = oracle.Run(P, u, x0, np.zeros((3, 1)), np.array([tau], np.float32))
        run.step(want_f=False)
        ut = oracle.gather(P, u, x0)[:, 0]
        # first step: no history, v = 0, so (m_p + m_f/2) dv/dt = m_p u~/tau + m_f (u~.grad) u~
        conv = ((m_p + 0.5 * m_f) * run.v[:, 0] / dt - m_p * ut / tau) / m_f
        X, Y = x0[0, 0], x0[1, 0]
        want = np.array([0.5 * math.sin(2 * X), 0.5 * math.sin(2 * Y), 0.0])
        errs.append(np.max(np.abs(conv - want)))
    assert errs[-1] < 5e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
    # the transposed product (grad u) . u = grad |u|^2 / 2 differs at this point
    X, Y = x0[0, 0], x0[1, 0]
    transposed = np.array([0.5 * math.sin(2 * X) * math.cos(2 * Y),
                           0.5 * math.sin(2 * Y) * math.cos(2 * X), 0.0])
    assert np.max(np.abs(transposed - want)) > 0.1


def test_am_rejects_other_integrators_and_shear():
    with pytest.raises(ValueError):
        _params((16,) * 3, (1.0,) * 3, 1.0, 0.1, 1e-3, 0.05, integrator=1)
    with pytest.raises(ValueError):
        _params((16,) * 3, (1.0,) * 3, 1.0, 0.1, 1e-3, 0.05, shear=0.5)
