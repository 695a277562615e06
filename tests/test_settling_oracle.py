"""Pins of the two-way coupled oracle loop (oracle.Run for the coupling step,
oracle.fluid.fluid_step for the fluid) on the settling particle of Sec. 3.2
(particle motion in the coupled regime): a heavy particle released from rest
under gravity in a periodic box at rest, Stokes drag with the self-disturbance
removed (eq. drag_coupled, Sec. 2.5).

What the paper fixes and these tests check:
* the particle relaxes to the uncoupled solution v_t (1 - e^{-t/tau_p})
  (eq. uncoupled_solution) up to an error that vanishes with d_p / sigma_R, and
  is first order in it (the regularised history of the particle's own
  disturbance, older than one step, stays in the field it sees);
* the removal takes out exactly the App. E disturbance of the last injection,
  whose value at the particle tends to (2/3) dt |D| / rho_f (2 pi sigma_s^2)^(-3/2)
  with D = m_p g at terminal velocity (the limit eta -> 0 of eq. disturbance_velo);
* at fixed sigma_R the result does not depend on the grid.
Velocities are measured relative to the box-mean fluid velocity, which grows by
the impulse the particle hands to the periodic box.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fluid

NU, RHO, TAU, G, M = 1.0, 1.0, 0.2, 0.5, 4
L = 2 * math.pi
SIGMA = L / 16


def settle(N, ratio, self_correction, sigma=SIGMA, T=6 * TAU, integrator=0):
    """Terminal-velocity error of the settling particle after T, against the
    discrete uncoupled solution v_t (1 - (1 - dt/tau)^K)."""
    dx = L / N
    eps = sigma ** 2 / (2 * NU)
    dt = eps / M
    K = int(round(T / dt))
    d = ratio * sigma
    m_p = 3 * math.pi * RHO * NU * d * TAU          # 6 pi mu a = m_p / tau_p
    P = oracle.make_params((N,) * 3, (L,) * 3, 1, m_p, RHO, NU, sigma, 3.0, 0.0, M, dt,
                           self_correction, g=(G, 0.0, 0.0), integrator=integrator)
    x = np.array([[L / 2 + 0.3 * dx], [L / 2], [L / 2]])
    run = oracle.Run(P, np.zeros((3, N, N, N)), x, np.zeros((3, 1)), np.array([TAU], np.float32))
    for _ in range(K):
        f, _ = run.step(want_f=True)
        run.u = fluid.fluid_step((N,) * 3, (L,) * 3, NU, dt, run.u, f)
    tau32 = float(np.float32(TAU))
    h = dt / tau32
    q = 1 - h if integrator == 0 else 1 - h + h * h / 2
    v_ref = tau32 * G * (1 - q ** K)
    return (run.v[0, 0] - run.u[0].mean()) / v_ref - 1.0, dt, m_p


def test_s1_error_first_order_in_dp_over_sigma():
    e1, _, _ = settle(16, 0.25, 1)
    e2, _, _ = settle(16, 0.125, 1)
    assert 0.0 < e2 < e1 < 0.06
    assert 1.9 < e1 / e2 < 2.1


def test_s2_removal_is_the_app_e_disturbance_of_the_last_injection():
    e_on, dt, m_p = settle(16, 0.25, 1)
    e_off, _, _ = settle(16, 0.25, 0)
    s2 = SIGMA ** 2 + 2 * NU * dt
    v_self = (2.0 / 3.0) * dt * m_p * G / RHO * (2 * math.pi * s2) ** -1.5
    removed = (e_off - e_on) * TAU * G
    assert removed > 0
    assert abs(removed / v_self - 1) < 0.1


def test_s3_grid_independent_at_fixed_sigma():
    e16, _, _ = settle(16, 0.25, 1)
    e32, _, _ = settle(32, 0.25, 1)
    assert abs(e16 - e32) < 5e-3


def test_s4_heun_stages_with_self_removal():
    """The paper extends the removal to each stage of a Runge-Kutta scheme
    (Sec. 2.5).  With Heun and the removal at both stages the settling error
    keeps the behaviour of the Euler scheme: first order in d_p / sigma_R, and
    lower than without the removal."""
    e1, _, _ = settle(16, 0.25, 1, integrator=2)
    e2, _, _ = settle(16, 0.125, 1, integrator=2)
    e_off, _, _ = settle(16, 0.25, 0, integrator=2)
    assert 0.0 < e2 < e1 < 0.06
    assert 1.9 < e1 / e2 < 2.1
    assert e_off > e1
