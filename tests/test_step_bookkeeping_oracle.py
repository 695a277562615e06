"""Pins of the oracle's step composition: which history level each stage reads,
which position is stored with a drag, where Heun's second stage removes the self
term, and the sign with which the self parts enter the Faxen and added-mass terms.

The definitions pinned are Sec. 2.3 eq. velo_reg_eq and Sec. 2.4
eq. ns_regularized_filtered (the fluid is forced at time t by the drag of time
t - eps_R, spread around the position of that same time), App. E
eqs. forcing_step and disturbance_velo (the injection made one step earlier is
what the fluid turned into the disturbance the particle sees), and Sec. 2.5
(that disturbance is removed from every term of the force, at every stage).
With eps_R = M dt the forcing of step n is the drag D^{n-M} at x^{n-M}, and the
self term of step n is the disturbance of the injection (x^{n-1-M}, D^{n-1-M}).

Nothing here re-runs the oracle's own arithmetic.  A carrier that is uniform in
space makes the trajectory a closed form until the first self term (the
geometric series of explicit Euler, of Heun and of the added-mass scheme), the
nodal Laplacian and gradient of such a field vanish exactly, so:
* the forcing is compared with the node-by-node brute force (oracle/brute.py) of
  the closed-form delayed position and drag;
* the first self terms are built from the App. B Green tensor (a formula of the
  paper independent of the App. E form the oracle uses), and its Laplacian and
  gradient from fourth-order finite differences of that tensor.
Particles move 0.4 sigma per step, so reading a neighbouring level, or storing
the next position, moves every checked value far outside its bar.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute

N = 16
L = 2.0
DX = L / N
SIGMA = 1.5 * DX
NU, RHO, M_P = 0.01, 1.0, 1.0
DT = 5e-3
TAU = float(np.float32(0.025))      # Stokes times are stored in float32
H = DT / TAU                        # 0.2
M = 3
U0 = np.array([12.0, -8.0, 5.0])    # |U0| dt = 0.41 sigma
SLIP0 = np.array([-5.0, 3.0, 2.0])
NP = 5


def _start():
    rng = np.random.default_rng(20240)
    x0 = rng.uniform(0.0, L, (3, NP))
    v0 = U0[:, None] + SLIP0[:, None] * rng.uniform(0.6, 1.4, (1, NP))
    return x0, v0


def _run(s, integrator=0, a_p=0.0, a_am=0.0):
    P = oracle.make_params((N,) * 3, (L,) * 3, NP, M_P, RHO, NU, SIGMA, 3.0, 0.0, M, DT, s,
                           integrator=integrator, a_p=a_p, a_am=a_am)
    u = np.zeros((3, N, N, N)) + U0[:, None, None, None]
    x0, v0 = _start()
    return oracle.Run(P, u, x0, v0, np.full(NP, TAU, np.float32)), x0, v0


def _closed_form(k, q, xfac):
    """v^k = U0 + (v0 - U0) q^k, x^k = x0 + k dt U0 + xfac (v0 - U0)(1 - q^k)."""
    x0, v0 = _start()
    w = U0[:, None]
    v = w + (v0 - w) * q ** k
    x = x0 + k * DT * w + xfac * (v0 - w) * (1 - q ** k)
    return x, v


def _euler(k):
    return _closed_form(k, 1 - H, TAU)


def _heun(k):
    q = 1 - H + H * H / 2
    return _closed_form(k, q, DT * (1 - H / 2) / (1 - q))


def _am(k, beta):
    q = 1 - H * beta
    return _closed_form(k, q, DT / (1 - q))


def _sigma_s():
    return math.sqrt(SIGMA ** 2 + 2 * NU * DT)


def _min_image(r):
    return r - L * np.round(r / L)


def _v_self(x, X, D):
    """App. B Green tensor form of the disturbance of the injection (X, D)."""
    return brute.green_tensor_velocity(_min_image(x - X), D, _sigma_s(), DT, RHO)


def _fd_derivatives(x, X, D):
    """Laplacian and gradient (grad[c, j] = d v_c / d x_j) of _v_self in x by
    fourth-order central differences."""
    h = 1e-3 * _sigma_s()
    lap = np.zeros((3, x.shape[1]))
    grad = np.zeros((3, 3, x.shape[1]))
    f0 = _v_self(x, X, D)
    for j in range(3):
        e = np.zeros((3, 1))
        e[j] = h
        fp1, fm1 = _v_self(x + e, X, D), _v_self(x - e, X, D)
        fp2, fm2 = _v_self(x + 2 * e, X, D), _v_self(x - 2 * e, X, D)
        lap += (-fp2 + 16 * fp1 - 30 * f0 + 16 * fm1 - fm2) / (12 * h * h)
        grad[:, j] = (-fp2 + 8 * fp1 - 8 * fm1 + fm2) / (12 * h)
    return lap, grad


def _close(got, want, scale, rtol):
    return np.max(np.abs(got - want)) <= rtol * scale


# ------------------------------------------------------------ (a) forcing ----

def test_b1_forcing_is_the_drag_of_level_n_minus_M_at_its_own_position():
    """s = 0: every level is the closed-form Euler state.  The forcing of steps
    M .. M+3 equals the brute-force deposit of (x^{n-M}, D^{n-M}); the one of a
    neighbouring level, or of the next position beside the same drag, does not."""
    run, _, _ = _run(0)
    for n in range(M + 4):
        f, D = run.step(want_f=True)
        if n < M:
            assert not np.any(f)
            continue
        k = n - M
        xk, vk = _euler(k)
        Dk = M_P * (U0[:, None] - vk) / TAU
        want = brute.deposit((N,) * 3, (L,) * 3, SIGMA, 3.0, RHO, np.mod(xk, L), Dk)
        scale = np.max(np.abs(want))
        assert _close(f, want, scale, 1e-12), n
        # the alternatives are far outside the bar
        x1, v1 = _euler(k + 1)
        D1 = M_P * (U0[:, None] - v1) / TAU
        for Xa, Da in ((x1, D1), (x1, Dk)):
            alt = brute.deposit((N,) * 3, (L,) * 3, SIGMA, 3.0, RHO, np.mod(Xa, L), Da)
            assert np.max(np.abs(alt - want)) > 0.1 * scale


# --------------------------------------------------------- (b) self term ----

def test_b2_self_term_is_the_injection_of_level_n_minus_1_minus_M():
    """s = 1, explicit Euler.  Steps 0..M have no self term, so x, v, D follow
    the closed form.  Step M+1 removes the disturbance of (x^0, D^0) at x^{M+1};
    step M+2 that of (x^1, D^1) at x^{M+2} (x^{M+2} = x^{M+1} + dt v^{M+1} is
    still closed form, v^{M+2} follows from the pinned D^{M+1})."""
    run, _, _ = _run(1)
    Ds = []
    for n in range(M + 3):
        _, D = run.step(want_f=False)
        Ds.append(D)
    levels = [_euler(k) for k in range(M + 2)]
    Dl = [M_P * (U0[:, None] - v) / TAU for _, v in levels]
    for n in range(M + 1):
        assert _close(Ds[n], Dl[n], np.max(np.abs(Dl[n])), 1e-12), n
    xa, va = levels[M + 1]
    vr = _v_self(xa, levels[0][0], Dl[0])
    want1 = M_P * (U0[:, None] - vr - va) / TAU
    tol1 = 1e-11 * np.max(np.abs(want1))
    assert _close(Ds[M + 1], want1, np.max(np.abs(want1)), 1e-11)
    # reading level n - M instead moves D^{M+1} by far more than the bar
    wrong = M_P * (U0[:, None] - _v_self(xa, levels[1][0], Dl[1]) - va) / TAU
    assert np.max(np.abs(wrong - want1)) > 1e6 * tol1
    vb = va + DT * want1 / M_P
    xb = xa + DT * va
    want2 = M_P * (U0[:, None] - _v_self(xb, levels[1][0], Dl[1]) - vb) / TAU
    assert _close(Ds[M + 2], want2, np.max(np.abs(want2)), 1e-11)


# ----------------------------------------------- (c) Heun's second stage ----

@pytest.mark.parametrize("a_p", [0.0, DX])
def test_b3_heun_second_stage_removes_the_self_term_at_x_star(a_p):
    """Heun with the removal at each stage (Sec. 2.5): at step M+1 stage 1 sees
    u~ = U0 - v_R(x^{M+1}) and stage 2 u~ = U0 - v_R(x*), x* = x^{M+1} + dt v^{M+1},
    both from the same injection (x^0, D^0).  With a Faxen radius the stages add
    (a_p^2/6) lap u~ = -(a_p^2/6) lap v_R at their own positions."""
    run, _, _ = _run(1, integrator=2, a_p=a_p)
    Ds = [run.step(want_f=False)[1] for _ in range(M + 2)]
    fax = a_p * a_p / 6.0
    x0l, v0l = _heun(0)
    D0 = M_P * (U0[:, None] - v0l) * (1 - H / 2) / TAU
    assert _close(Ds[0], D0, np.max(np.abs(D0)), 1e-12)
    xa, va = _heun(M + 1)
    xs = xa + DT * va

    def drag(x2):
        u1 = U0[:, None] - _v_self(xa, x0l, D0) - fax * _fd_derivatives(xa, x0l, D0)[0]
        u2 = U0[:, None] - _v_self(x2, x0l, D0) - fax * _fd_derivatives(x2, x0l, D0)[0]
        d1 = (u1 - va) / TAU
        vst = va + DT * d1
        d2 = (u2 - vst) / TAU
        return M_P * 0.5 * (d1 + d2)

    want = drag(xs)
    tol = 1e-9 * np.max(np.abs(want))
    assert np.max(np.abs(Ds[M + 1] - want)) <= tol
    assert np.max(np.abs(drag(xa) - want)) > 1e4 * tol     # stage 2 at x^n instead


# ------------------------------------ (d) Faxen and added-mass self parts ----

@pytest.mark.parametrize("integrator", [0, 1])
def test_b4_faxen_self_laplacian_enters_with_a_minus_sign(integrator):
    """A Faxen radius on the uniform carrier: at step M+1 the drag sees
    u~ + (a_p^2/6) lap u~ with u~ = U0 - v_R and lap u~ = -lap v_R
    (eq. force_particle, first line), lap v_R from finite differences of the
    App. B tensor; the grid Laplacian of the uniform field is exactly zero.
    Explicit Euler: D = m_p (u~ + (a_p^2/6) lap u~ - v)/tau.  Exponential
    integrator: the step-average drag m_p (w - v)(1 - e^{-dt/tau})/dt with w the
    same corrected velocity, on its own closed-form trajectory."""
    a_p = DX
    fax = a_p * a_p / 6.0
    run, _, _ = _run(1, integrator=integrator, a_p=a_p)
    Ds = [run.step(want_f=False)[1] for _ in range(M + 2)]
    if integrator == 0:
        traj, gain = _euler, 1.0 / TAU
    else:
        E = math.exp(-H)
        traj, gain = (lambda k: _closed_form(k, E, TAU)), -math.expm1(-H) / DT
    x0l, v0l = traj(0)
    D0 = M_P * (U0[:, None] - v0l) * gain
    assert _close(Ds[0], D0, np.max(np.abs(D0)), 1e-12)
    xa, va = traj(M + 1)
    lap, _ = _fd_derivatives(xa, x0l, D0)
    base = U0[:, None] - _v_self(xa, x0l, D0) - va
    want = M_P * (base - fax * lap) * gain
    tol = 1e-9 * np.max(np.abs(want))
    assert np.max(np.abs(Ds[M + 1] - want)) <= tol
    assert np.max(np.abs(M_P * (base + fax * lap) * gain - want)) > 1e4 * tol


def test_b5_added_mass_self_parts_enter_with_a_minus_sign():
    """Added mass (eq. force_particle, second line; explicit Euler with the
    particle's own acceleration on the left, path derivatives over the last
    step).  On the uniform carrier the state is a geometric series until step
    M+1 (u~ is constant, so every d/dt and the convective term vanish and the
    effective mass is m_p + m_f/2).  At step M+1, u~ = U0 - v_R and its
    Laplacian and gradient are minus those of v_R (finite differences of the
    App. B tensor): the drag of that step follows, and flipping the sign of the
    self parts moves it far outside the bar."""
    a = 0.8 * DX
    m_f = RHO * 4.0 / 3.0 * math.pi * a ** 3
    beta = M_P / (M_P + 0.5 * m_f)
    fax, fam = a * a / 6.0, a * a / 10.0
    run, _, _ = _run(1, a_p=a, a_am=a)
    Ds = [run.step(want_f=False)[1] for _ in range(M + 2)]
    x0l, v0l = _am(0, beta)
    D0 = beta * M_P * (U0[:, None] - v0l) / TAU
    for k in range(M + 1):
        _, vk = _am(k, beta)
        Dk = beta * M_P * (U0[:, None] - vk) / TAU
        assert _close(Ds[k], Dk, np.max(np.abs(Dk)), 1e-12), k
    xa, va = _am(M + 1, beta)
    vr = _v_self(xa, x0l, D0)
    lap, grad = _fd_derivatives(xa, x0l, D0)

    def drag(sign):
        ut = U0[:, None] - vr
        lapu = -sign * lap
        gradu = -sign * grad
        q = ut + fam * lapu
        S = M_P * (ut + fax * lapu - va) / TAU
        dut = (ut - U0[:, None]) / DT
        dq = (q - U0[:, None]) / DT
        conv = np.einsum("j...,cj...->c...", ut - va, gradu)
        Dm = dut + conv
        acc = (S + m_f * Dm + 0.5 * m_f * dq) / (M_P + 0.5 * m_f)
        return S + m_f * Dm + 0.5 * m_f * (dq - acc)

    want = drag(1.0)
    tol = 1e-9 * np.max(np.abs(want))
    assert np.max(np.abs(Ds[M + 1] - want)) <= tol
    assert np.max(np.abs(drag(-1.0) - want)) > 1e3 * tol
