"""Pins of the oracle's Basset term (Sec. 2.5, eq. force_particle, third line).

In the two-way coupled scheme the field already carries the vorticity the
particle produced before the current step, so the memory integral covers the
last step only (closing paragraph of Sec. 2.5).  The reading: over that step the
bracket w = u~ + (a_b^2/6) lap u~ - v changes at the constant rate
(w^n - w^{n-1})/dt, which gives B^n = K_B (w^n - w^{n-1}) with
K_B = 6 pi mu a_b^2 (1/dt) int_0^dt [pi nu s]^{-1/2} ds, and B = 0 on the first
step (no previous value).  What fixes each value here:
* b1  the one-step kernel integral is computed by adaptive quadrature with the
      algebraic end-point weight (scipy), not from its closed form; settling
      from rest then follows the closed-form solution of the second-order linear
      recurrence of the scheme (two characteristic roots), at every step, and
      the drag handed to the fluid is m_p dv/dt - m_p g_b;
* b2  a transverse wave whose amplitude grows linearly in time (no convective
      term, particle fixed in x): the second step's velocity carries K_B times
      (1 - (a_b^2/6) k_h^2), k_h^2 the symbol of the interpolated nodal
      Laplacian -- the Faxen factor a_b^2/6 of the Basset bracket, not a_b^2/10;
* b3  the self-disturbance is removed inside the bracket: at the first step with
      a self term, switching the removal on changes the drag by
      -(m_p/tau) v_R - K_B (v_R + (a_b^2/6) lap v_R), with v_R from the App. B
      Green tensor and its Laplacian by fourth-order finite differences;
* b4  the reading's limits: the terminal velocity does not depend on the term,
      the transient is slowed by it, and its effect on the velocity at a fixed
      time vanishes as sqrt(dt) (the window shrinks with the step).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import brute

RHO, NU = 1.0, 0.1
A = 0.05                                  # particle radius
RHO_P = 10.0                              # heavy particle, rho_p / rho_f = 10
M_F = RHO * 4.0 / 3.0 * math.pi * A ** 3
M_P = RHO_P * M_F
TAU = float(np.float32(M_P / (6 * math.pi * RHO * NU * A)))   # 6 pi mu a = m_p / tau_p


def k_basset(dt, a=A):
    """6 pi mu a^2 (1/dt) int_0^dt (pi nu s)^(-1/2) ds by quadrature."""
    val, _ = integrate.quad(lambda s: 1.0 / math.sqrt(math.pi * NU), 0.0, dt,
                            weight="alg", wvar=(-0.5, 0.0))
    return 6 * math.pi * RHO * NU * a * a * val / dt


def _params(n, L, sigma, dt, a_b, s=0, g=(0.0, 0.0, 0.0), a_p=0.0, M=2, np_=1):
    return oracle.make_params(n, L, np_, M_P, RHO, NU, sigma, 3.0, 0.0, M, dt, s, g=g,
                              a_p=a_p, a_b=a_b)


def _settle(dt, steps, a_b, gb=2.0):
    P = _params((16,) * 3, (1.0,) * 3, 0.1, dt, a_b, g=(gb, 0.0, 0.0))
    run = oracle.Run(P, np.zeros((3, 16, 16, 16)), np.full((3, 1), 0.5), np.zeros((3, 1)),
                     np.array([TAU], np.float32))
    vs, Ds = [run.v[0, 0]], []
    for _ in range(steps):
        _, D = run.step(want_f=False)
        Ds.append(D[0, 0])
        vs.append(run.v[0, 0])
    return np.array(vs), np.array(Ds)


def test_b1_settling_follows_the_recurrence_with_the_quadrature_coefficient():
    dt = 0.2 * TAU
    gb = 2.0
    K = k_basset(dt)
    # the quadrature agrees with the closed form 2 sqrt(dt / (pi nu)) of the integral
    assert abs(K * dt / (6 * math.pi * RHO * NU * A * A) - 2 * math.sqrt(dt / (math.pi * NU))) \
        < 1e-12 * K
    h, beta = dt / TAU, K * dt / M_P
    assert 0.2 < beta < 0.6                  # the explicit scheme is stable here
    vs, Ds = _settle(dt, 60, A, gb)
    # v^{n+1} = (1 - h - beta) v^n + beta v^{n-1} + dt g_b for n >= 1; v^0 = 0, v^1 = dt g_b
    c1, c0 = 1 - h - beta, beta
    r = np.roots([1.0, -c1, -c0])
    vinf = TAU * gb
    Amat = np.array([[1.0, 1.0], [r[0], r[1]]])
    coef = np.linalg.solve(Amat, np.array([-vinf, dt * gb - vinf]))
    n = np.arange(vs.size)
    closed = vinf + coef[0] * r[0] ** n + coef[1] * r[1] ** n
    assert np.max(np.abs(vs - closed)) <= 1e-12 * vinf
    # the fluid receives the hydrodynamic force m_p dv/dt - m_p g_b
    assert np.allclose(Ds, M_P * np.diff(vs) / dt - M_P * gb, rtol=0, atol=1e-12 * M_P * gb)


def test_b2_faxen_factor_inside_the_bracket_is_a_squared_over_six():
    N, L = 32, 2 * math.pi
    dx = L / N
    k = 3.0
    dt, alpha = 2e-3, 2.0
    a_b = 0.15
    P = _params((N,) * 3, (L,) * 3, 2 * dx, dt, a_b)
    ax = np.arange(N) * dx
    wave = np.zeros((3, N, N, N))
    wave[1] = np.sin(k * ax)[None, None, :]
    x0 = np.array([[1.234], [2.0], [3.0]])
    run = oracle.Run(P, 0 * wave, x0, np.zeros((3, 1)), np.array([TAU], np.float32))
    for n in range(2):
        run.u = alpha * n * dt * wave
        run.step(want_f=False)
    sp = oracle.gather(P, wave, x0)[1, 0]
    kh2 = (2 - 2 * math.cos(k * dx)) / dx ** 2
    K = k_basset(dt, a_b)
    ut1 = alpha * dt * sp
    want = dt * ut1 * (1.0 / TAU + K * (1 - a_b * a_b / 6 * kh2) / M_P)
    assert abs(run.v[1, 0] / want - 1) < 1e-12
    other = dt * ut1 * (1.0 / TAU + K * (1 - a_b * a_b / 10 * kh2) / M_P)
    assert abs(other / want - 1) > 1e-4
    assert run.v[0, 0] == 0.0 and run.v[2, 0] == 0.0


def _sigma_s(P):
    return math.sqrt(P.sigma ** 2 + P.nu * 2 * P.dt)


def test_b3_self_disturbance_removed_inside_the_bracket():
    N, L, M = 16, 2.0, 3
    dx = L / N
    dt = 0.2 * TAU
    U0 = np.array([1.5, -1.0, 0.6])
    x0 = np.array([[0.4, 1.3], [0.7, 0.2], [1.1, 1.6]])
    v0 = U0[:, None] + np.array([[-0.5, 0.3], [0.4, -0.2], [0.2, 0.25]])
    D, X, P = {}, {}, None
    for s in (0, 1):
        P = _params((N,) * 3, (L,) * 3, 1.5 * dx, dt, A, s=s, M=M, np_=2)
        u = np.zeros((3, N, N, N)) + U0[:, None, None, None]
        run = oracle.Run(P, u, x0, v0, np.full(2, TAU, np.float32))
        out = [run.step(want_f=False)[1] for _ in range(M + 1)]
        X[s] = run.x.copy()
        out.append(run.step(want_f=False)[1])
        D[s] = out
    for n in range(M + 1):
        assert np.array_equal(D[0][n], D[1][n])
    assert np.array_equal(X[0], X[1])
    D0 = M_P * (U0[:, None] - v0) / TAU
    assert np.allclose(D[0][0], D0, rtol=1e-13, atol=0)
    sig = _sigma_s(P)

    def vself(x):
        r = x - x0
        r -= L * np.round(r / L)
        return brute.green_tensor_velocity(r, D0, sig, dt, RHO)

    xa = X[0]
    vr = vself(xa)
    h = 1e-3 * sig
    lap = np.zeros_like(vr)
    for j in range(3):
        e = np.zeros((3, 1))
        e[j] = h
        lap += (-vself(xa + 2 * e) + 16 * vself(xa + e) - 30 * vr + 16 * vself(xa - e)
                - vself(xa - 2 * e)) / (12 * h * h)
    K = k_basset(dt)
    want = -(M_P / TAU) * vr - K * (vr + A * A / 6 * lap)
    got = D[1][M + 1] - D[0][M + 1]
    tol = 1e-7 * np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= tol
    flipped = -(M_P / TAU) * vr - K * (vr - A * A / 6 * lap)
    assert np.max(np.abs(flipped - want)) > 1e2 * tol


def test_b4_terminal_velocity_transient_and_vanishing_window():
    gb = 2.0
    T = 3 * TAU
    # same terminal velocity, slower transient
    vb, _ = _settle(0.2 * TAU, 200, A, gb)
    v0, _ = _settle(0.2 * TAU, 200, 0.0, gb)
    assert abs(vb[-1] / (TAU * gb) - 1) < 1e-9 and abs(v0[-1] / (TAU * gb) - 1) < 1e-9
    assert np.all(vb[2:15] < v0[2:15])
    # the effect at t = 3 tau shrinks as sqrt(dt)
    eff = []
    for dt in (0.1 * TAU, 0.025 * TAU):
        steps = int(round(T / dt))
        eff.append(_settle(dt, steps, 0.0, gb)[0][-1] - _settle(dt, steps, A, gb)[0][-1])
    ratio = eff[0] / eff[1]
    assert 1.7 < ratio < 2.3                 # sqrt(4) = 2


def test_b_rejects_other_integrators_and_shear():
    with pytest.raises(ValueError):
        oracle.make_params((16,) * 3, (1.0,) * 3, 1, M_P, RHO, NU, 0.1, integrator=2, a_b=A)
    with pytest.raises(ValueError):
        oracle.make_params((16,) * 3, (1.0,) * 3, 1, M_P, RHO, NU, 0.1, shear=0.5, a_b=A)
