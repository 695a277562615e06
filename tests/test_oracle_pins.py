"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage (arXiv:1405.6969) or the mathematical fact it
relies on.  None of them re-types the oracle's own formula: they use closed
forms, limits, invariants, an independent formula from another part of the
paper (App. B vs App. E), brute force on tiny boxes, or 60-digit arithmetic.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads


def _params(box, M=2, dt=1e-3, s=1, **kw):
    return oracle.params_for_box(box, M=M, dt=dt, self_correction=s, **kw)


# --------------------------------------------------------------- kernel -----

@pytest.mark.parametrize("sigma_dx", [1.5, 2.0])
def test_p1_lattice_sum_of_gaussian_is_its_integral(sigma_dx):
    """Sec. 2.3, eq. known_integral: the Gaussian integrates to one.  On a
    lattice (Poisson summation) the sum with a wide cut-off equals the
    continuum integral (2 pi sigma^2)^(3/2) up to ~1e-19 aliasing."""
    box = workloads.tiny_box(3, n=(48, 48, 48), np_=20, sigma_dx=sigma_dx)
    P = oracle.params_for_box(box, M=1, dt=1e-3)
    P.cutoff = 8.0
    Z = oracle.normalisation(P, box.x)
    cont = (2 * math.pi * box.sigma ** 2) ** 1.5
    assert np.max(np.abs(Z / cont - 1.0)) < 1e-12


def test_p2_truncated_sphere_mass_band():
    """The 3 sigma sphere keeps erf(3/sqrt2) - 3 sqrt(2/pi) e^-4.5 = 0.97071 of
    the mass in the continuum; on the lattice it scatters around that value."""
    box = workloads.tiny_box(4, n=(32, 32, 32), np_=200, sigma_dx=1.5)
    P = oracle.params_for_box(box, M=1, dt=1e-3)
    Z = oracle.normalisation(P, box.x)
    frac = Z / (2 * math.pi * box.sigma ** 2) ** 1.5
    cont = math.erf(3 / math.sqrt(2)) - 3 * math.sqrt(2 / math.pi) * math.exp(-4.5)
    assert abs(cont - 0.970709) < 1e-6
    assert np.all(frac > 0.955) and np.all(frac < 0.985)
    assert abs(np.mean(frac) - cont) < 5e-3


# -------------------------------------------------------------- scatter -----

@pytest.mark.parametrize("seed,n,sigma_dx,placement", [
    (11, (12, 13, 14), 1.5, "uniform"),
    (12, (16, 12, 13), 1.5, "clustered"),
    (13, (14, 14, 14), 2.0, "uniform"),
    (14, (13, 15, 12), 1.5, "uniform"),
])
def test_p5_deposit_equals_brute_force(seed, n, sigma_dx, placement):
    """Sec. 2.4, eq. ns_regularized_filtered, evaluated node by node with the
    minimum-image distance (oracle/brute.py) on tiny periodic boxes."""
    box = workloads.tiny_box(seed, n=n, np_=23, sigma_dx=sigma_dx, placement=placement)
    rng = np.random.default_rng(seed)
    D = rng.normal(size=(3, box.np_))
    P = _params(box)
    f = oracle.deposit(P, box.x, D)
    fb = brute.deposit(box.n, box.L, box.sigma, 3.0, box.spec.rho_f, box.x, D)
    assert np.max(np.abs(f - fb)) <= 1e-13 * np.max(np.abs(fb))


def test_p3_momentum_balance():
    """Momentum balance (Sec. 1: all vorticity the particle generates reaches the
    fluid): rho_f dV sum_c f_c = - sum_p D_p."""
    box = workloads.tiny_box(21, n=(32, 24, 28), np_=400, placement="clustered")
    rng = np.random.default_rng(1)
    D = rng.normal(size=(3, box.np_))
    P = _params(box)
    f = oracle.deposit(P, box.x, D)
    dV = np.prod(box.dx)
    lhs = box.spec.rho_f * dV * f.reshape(3, -1).sum(axis=1)
    assert np.allclose(lhs, -D.sum(axis=1), rtol=1e-13, atol=1e-13 * np.abs(D).sum())


def test_p4_single_particle_closed_form():
    """One particle: f = -(D/rho_f) g / sum(g dV) on the nodes of the 3 sigma
    ball and zero elsewhere (Sec. 2.4 with the per-particle normalisation)."""
    box = workloads.tiny_box(5, n=(20, 20, 20), np_=1)
    D = np.array([[0.3], [-1.2], [0.7]])
    P = _params(box)
    f = oracle.deposit(P, box.x, D)
    dx = box.dx[0]
    X = box.x[:, 0]
    cnt = 0
    gam = np.zeros((20, 20, 20))
    for k in range(20):
        for j in range(20):
            for i in range(20):
                r = np.array([i, j, k]) * dx - X
                r -= box.L[0] * np.round(r / box.L[0])
                r2 = float(r @ r)
                if r2 <= (3 * box.sigma) ** 2:
                    gam[k, j, i] = math.exp(-r2 / (2 * box.sigma ** 2))
                    cnt += 1
    Z = gam.sum() * dx ** 3
    for c in range(3):
        assert np.allclose(f[c], -D[c, 0] * gam / Z, rtol=1e-13, atol=1e-16)
    # sphere of radius 4.5 dx: 360-393 nodes depending on the offset
    assert 355 <= cnt <= 400


def test_p6_linearity_and_superposition():
    """The forcing is linear in the drags and additive over particles (the
    disturbance equation is linear, Sec. 2.1, eq. unsteady_stokes)."""
    box = workloads.tiny_box(31, n=(16, 16, 16), np_=30)
    rng = np.random.default_rng(2)
    D1, D2 = rng.normal(size=(2, 3, box.np_))
    P = _params(box)
    f1 = oracle.deposit(P, box.x, D1)
    f2 = oracle.deposit(P, box.x, D2)
    f12 = oracle.deposit(P, box.x, 2.5 * D1 - 0.75 * D2)
    assert np.allclose(f12, 2.5 * f1 - 0.75 * f2, rtol=0, atol=1e-13 * np.abs(f12).max())
    fa = oracle.deposit(P, box.x[:, :12], D1[:, :12])
    fb = oracle.deposit(P, box.x[:, 12:], D1[:, 12:])
    assert np.allclose(fa + fb, f1, rtol=0, atol=1e-13 * np.abs(f1).max())


def test_p7_translation_reflection_permutation():
    """Symmetries of the periodic problem: shifting every particle by whole
    node vectors shifts f by the same node offsets; mirroring x -> L - x with
    D_x -> -D_x mirrors f with f_x -> -f_x; swapping axes of a cubic box swaps
    the components of f."""
    box = workloads.tiny_box(41, n=(16, 16, 16), np_=25)
    rng = np.random.default_rng(3)
    D = rng.normal(size=(3, box.np_))
    P = _params(box)
    f = oracle.deposit(P, box.x, D)
    tol = 1e-11 * np.abs(f).max()
    dx = box.dx[0]
    L = box.L[0]
    # translation by (3, -2, 5) nodes
    sh = np.array([3, -2, 5])
    Xs = np.mod(box.x + (sh * dx)[:, None], L)
    fs = oracle.deposit(P, Xs, D)
    assert np.allclose(fs, np.roll(f, shift=(5, -2, 3), axis=(1, 2, 3)), atol=tol, rtol=0)
    # reflection in x
    Xr = box.x.copy()
    Xr[0] = np.mod(L - Xr[0], L)
    Dr = D.copy()
    Dr[0] *= -1
    fr = oracle.deposit(P, Xr, Dr)
    idx = (-np.arange(16)) % 16
    fm = f[:, :, :, idx].copy()
    fm[0] *= -1
    assert np.allclose(fr, fm, atol=tol, rtol=0)
    # swap x and y
    Xp = box.x[[1, 0, 2]]
    Dp = D[[1, 0, 2]]
    fp = oracle.deposit(P, Xp, Dp)
    ft = np.transpose(f[[1, 0, 2]], (0, 1, 3, 2))
    assert np.allclose(fp, ft, atol=tol, rtol=0)


def test_deposit_window_matches_full_grid():
    box = workloads.tiny_box(42, n=(24, 20, 22), np_=60, placement="clustered")
    rng = np.random.default_rng(4)
    D = rng.normal(size=(3, box.np_))
    P = _params(box)
    f = oracle.deposit(P, box.x, D)
    lo, wn = (18, 3, 15), (9, 7, 10)   # wraps in x and z
    fw = oracle.deposit(P, box.x, D, lo=lo, wn=wn)
    iz = (np.arange(wn[2]) + lo[2]) % 22
    iy = (np.arange(wn[1]) + lo[1]) % 20
    ix = (np.arange(wn[0]) + lo[0]) % 24
    ref = f[:, iz][:, :, iy][:, :, :, ix]
    assert np.array_equal(fw, ref)


# ------------------------------------------------------- self-disturbance ---

def _sd_setup(seed=7):
    box = workloads.tiny_box(seed, n=(32, 32, 32), np_=1)
    P = _params(box, M=3, dt=2e-3)
    sig_s = math.sqrt(box.sigma ** 2 + 2 * box.spec.nu * 2e-3)
    return box, P, sig_s


def _vs(P, r, Dp, base=None):
    x0 = np.array([[1.0], [1.1], [0.9]]) if base is None else base
    x = x0 + np.asarray(r, dtype=np.float64).reshape(3, 1)
    return oracle.self_disturbance(P, x, x0, np.asarray(Dp, float).reshape(3, 1))[:, 0]


def test_p8i_self_disturbance_equals_app_b_green_tensor():
    """App. E closed form (eq. disturbance_velo) with the -dt/rho_f prefactor
    equals -dt G_ik(r; sigma_s) D_k with the unsteady Stokeslet of App. B
    (eq. green_tensor), a formula derived independently in the paper."""
    box, P, sig_s = _sd_setup()
    rng = np.random.default_rng(8)
    for eta in [0.31, 0.5, 1.0, 2.0, 3.5]:
        for _ in range(3):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            r = d * eta * math.sqrt(2) * sig_s
            Dp = rng.normal(size=3)
            v = _vs(P, r, Dp)
            ref = brute.green_tensor_velocity(r.reshape(3, 1), Dp.reshape(3, 1), sig_s,
                                              P.dt, P.rho_f)[:, 0]
            assert np.allclose(v, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_p8i_series_branch_against_60_digit_green_tensor():
    """Below eta = 0.3 the oracle sums Maclaurin series; compare with the App. B
    Green tensor and the App. E closed form in 60-digit arithmetic."""
    box, P, sig_s = _sd_setup()
    rng = np.random.default_rng(9)
    for eta in [1e-6, 1e-3, 0.017, 0.1, 0.2999, 0.3001]:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = d * eta * math.sqrt(2) * sig_s
        Dp = rng.normal(size=3)
        v = _vs(P, r, Dp)
        ref_b = brute.green_tensor_velocity_hp(r, Dp, sig_s, P.dt, P.rho_f)
        ref_e = brute.disturbance_velo_hp(r, Dp, sig_s, P.dt, P.rho_f)
        assert np.allclose(ref_b, ref_e, rtol=1e-25, atol=0)
        assert np.allclose(v, ref_b, rtol=2e-14, atol=1e-15 * np.abs(ref_b).max())


def test_p8ii_self_disturbance_is_divergence_free():
    """The projection step of App. E makes the field solenoidal."""
    box, P, sig_s = _sd_setup()
    rng = np.random.default_rng(10)
    Dp = rng.normal(size=3)
    h = 1e-4 * sig_s
    for rr in [0.2, 0.6, 1.3]:
        r0 = rng.normal(size=3)
        r0 *= rr * sig_s / np.linalg.norm(r0)
        div = 0.0
        scale = 0.0
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            dv = (_vs(P, r0 + e, Dp)[c] - _vs(P, r0 - e, Dp)[c]) / (2 * h)
            div += dv
            scale = max(scale, abs(dv))
        grad_scale = np.abs(_vs(P, r0, Dp)).max() / sig_s
        assert abs(div) < 1e-6 * max(scale, grad_scale)


def test_p8iii_limits():
    """r -> 0: the transverse projection keeps 2/3 of the Gaussian peak;
    r >> sigma_s: the potential dipole -(dt/rho_f)[3(D.rh)rh - D]/(4 pi r^3)."""
    box, P, sig_s = _sd_setup()
    Dp = np.array([0.4, -1.1, 0.25])
    v0 = _vs(P, [0.0, 0.0, 0.0], Dp)
    peak = -(P.dt / P.rho_f) * (2 * math.pi * sig_s ** 2) ** -1.5 * (2.0 / 3.0)
    assert np.allclose(v0, peak * Dp, rtol=1e-14)
    r = np.array([0.6, -0.3, 0.45])
    r *= 9.0 * sig_s / np.linalg.norm(r)   # eta ~ 6.4, e^-eta^2 ~ 1e-18
    rn = np.linalg.norm(r)
    rh = r / rn
    far = -(P.dt / P.rho_f) * (3 * (Dp @ rh) * rh - Dp) / (4 * math.pi * rn ** 3)
    assert np.allclose(_vs(P, r, Dp), far, rtol=1e-12)


def test_self_disturbance_continuous_at_series_switch():
    box, P, sig_s = _sd_setup()
    d = np.array([0.3, 0.5, -0.81])
    d /= np.linalg.norm(d)
    Dp = np.array([1.0, 0.2, -0.7])
    a = _vs(P, d * 0.3 * (1 - 1e-12) * math.sqrt(2) * sig_s, Dp)
    b = _vs(P, d * 0.3 * (1 + 1e-12) * math.sqrt(2) * sig_s, Dp)
    assert np.allclose(a, b, rtol=1e-13)


def test_self_disturbance_minimum_image():
    box, P, sig_s = _sd_setup()
    L = box.L[0]
    Dp = np.array([0.1, 0.2, 0.3])
    base = np.array([[0.01], [L - 0.02], [0.5]])
    r = np.array([-0.02, 0.03, 0.001])
    x = np.mod(base + r.reshape(3, 1), L)
    v = oracle.self_disturbance(P, x, base, Dp.reshape(3, 1))[:, 0]
    assert np.allclose(v, _vs(P, r, Dp), rtol=1e-12)


# ----------------------------------------------------------------- gather ---

def test_p9_gather_exact_cases_and_brute_force():
    """Trilinear interpolation reproduces nodal values at nodes and constants
    everywhere, and equals the hat-function sum over all nodes."""
    box = workloads.tiny_box(51, n=(12, 14, 13), np_=40, shear=0.7)
    P = _params(box)
    up = oracle.gather(P, box.u, box.x)
    ref = brute.gather(box.n, box.L, box.u, box.x, shear=0.7)
    assert np.allclose(up, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    # at nodes
    ii = np.array([0, 5, 11, 3])
    jj = np.array([0, 13, 7, 2])
    kk = np.array([12, 0, 6, 9])
    xn = np.stack([ii * box.dx[0], jj * box.dx[1], kk * box.dx[2]])
    P0 = _params(box)
    P0.shear = 0.0
    un = oracle.gather(P0, box.u, xn)
    assert np.array_equal(un, box.u[:, kk, jj, ii])
    # constant field, fields affine within one cell
    uc = np.ones_like(box.u) * np.array([1.5, -2.0, 0.25])[:, None, None, None]
    assert np.allclose(oracle.gather(P0, uc, box.x), np.array([1.5, -2.0, 0.25])[:, None],
                       rtol=0, atol=1e-14)
    Nx, Ny, Nz = box.n
    zz, yy, xx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    ua = np.stack([1 + 0.5 * xx - 0.25 * yy + 0.125 * zz] * 3).astype(np.float64)
    xin = np.stack([np.linspace(0.1, Nx - 1.2, 9) * box.dx[0],
                    np.linspace(0.3, Ny - 1.1, 9) * box.dx[1],
                    np.linspace(0.2, Nz - 1.4, 9) * box.dx[2]])
    want = 1 + 0.5 * xin[0] / box.dx[0] - 0.25 * xin[1] / box.dx[1] + 0.125 * xin[2] / box.dx[2]
    assert np.allclose(oracle.gather(P0, ua, xin)[0], want, rtol=1e-14)


# ----------------------------------------------------------------- update ---

def _uniform_carrier_run(steps, dt, tau, u0, s=0, M=3):
    box = workloads.tiny_box(61, n=(16, 16, 16), np_=8, carrier="zero", tau=(tau,))
    u = np.zeros_like(box.u) + np.asarray(u0)[:, None, None, None]
    P = _params(box, M=M, dt=dt, s=s)
    run = oracle.Run(P, u, box.x, box.v, box.tau)
    x0, v0 = box.x.copy(), box.v.copy()
    for _ in range(steps):
        run.step(want_f=False)
    return box, run, x0, v0


def test_p10_update_geometric_series():
    """Explicit Euler on dv/dt = (u0 - v)/tau (Sec. 2.5, eq. force_stokes_drag,
    Sec. 3.2, eq. Drag_one_way) has the exact discrete solution
    v^n = u0 + (v0-u0) q^n, x^n = x0 + n dt u0 + tau (v0-u0)(1-q^n), q = 1-dt/tau."""
    u0 = np.array([0.3, -0.2, 0.1])
    dt, tau, n = 1e-3, 0.05, 37
    box, run, x0, v0 = _uniform_carrier_run(n, dt, tau, u0)
    tau = float(np.float32(tau))       # Stokes times are stored in float32
    q = 1 - dt / tau
    v_ref = u0[:, None] + (v0 - u0[:, None]) * q ** n
    x_ref = x0 + n * dt * u0[:, None] + tau * (v0 - u0[:, None]) * (1 - q ** n)
    assert np.allclose(run.v, v_ref, rtol=1e-12, atol=1e-14)
    L = box.L[0]
    dxw = run.x - x_ref
    dxw -= L * np.round(dxw / L)
    assert np.max(np.abs(dxw)) < 1e-12


def test_p10g_body_force_geometric_series():
    """With a body acceleration g_b (eq. particle_motion: (m_p - m_f) g / m_p)
    explicit Euler relaxes to w = u0 + tau g_b: v^n = w + (v0 - w) q^n,
    x^n = x0 + n dt w + tau (v0 - w)(1 - q^n).  The drag handed to the fluid is
    the hydrodynamic force alone, m_p (u0 - v^n)/tau, which tends to -m_p g_b
    (eq. drag_coupled: at terminal velocity the drag balances gravity)."""
    u0 = np.array([0.3, -0.2, 0.1])
    gb = np.array([-0.9, 0.4, 2.0])
    dt, tau, n, M = 1e-3, 0.05, 800, 3
    box = workloads.tiny_box(61, n=(16, 16, 16), np_=8, carrier="zero", tau=(tau,))
    u = np.zeros_like(box.u) + u0[:, None, None, None]
    P = _params(box, M=M, dt=dt, s=0)
    P.g = (type(P.g))(*gb)
    run = oracle.Run(P, u, box.x, box.v, box.tau)
    x0, v0 = box.x.copy(), box.v.copy()
    for _ in range(n - 1):
        run.step(want_f=False)
    v_before = run.v.copy()
    _, D = run.step(want_f=False)
    tau32 = float(np.float32(tau))
    q = 1 - dt / tau32
    w = (u0 + tau32 * gb)[:, None]
    assert np.allclose(run.v, w + (v0 - w) * q ** n, rtol=1e-12, atol=1e-13)
    x_ref = x0 + n * dt * w + tau32 * (v0 - w) * (1 - q ** n)
    dxw = run.x - x_ref
    dxw -= box.L[0] * np.round(dxw / box.L[0])
    assert np.max(np.abs(dxw)) < 1e-12
    assert np.allclose(D, box.m_p * (u0[:, None] - v_before) / tau32, rtol=1e-13, atol=0)
    assert np.allclose(D, -box.m_p * gb[:, None], rtol=1e-5)   # q^n ~ 1e-7


@pytest.mark.parametrize("dt_over_tau", [0.02, 3.0])
def test_p10e_exponential_integrator_is_exact_for_a_uniform_carrier(dt_over_tau):
    """With u~ uniform the exponential integrator reproduces the continuous
    solution of m_p dv/dt = m_p (u0 - v)/tau + m_p g_b at every step
    (eq. uncoupled_solution with an initial slip): v = w + (v0 - w) e^{-t/tau},
    x = x0 + w t + tau (v0 - w)(1 - e^{-t/tau}), w = u0 + tau g_b, also for
    dt = 3 tau where explicit Euler diverges.  The drag handed to the fluid is
    the momentum the drag exchanged over the step divided by dt."""
    u0 = np.array([0.3, -0.2, 0.1])
    gb = np.array([-0.9, 0.4, 2.0])
    tau = 0.05
    tau32 = float(np.float32(tau))
    dt = dt_over_tau * tau32
    n = 30
    box = workloads.tiny_box(61, n=(16, 16, 16), np_=8, carrier="zero", tau=(tau,))
    u = np.zeros_like(box.u) + u0[:, None, None, None]
    P = _params(box, M=3, dt=dt, s=0)
    P.g = (type(P.g))(*gb)
    P.integrator = 1
    run = oracle.Run(P, u, box.x, box.v, box.tau)
    x0, v0 = box.x.copy(), box.v.copy()
    for _ in range(n - 1):
        run.step(want_f=False)
    vb = run.v.copy()
    _, D = run.step(want_f=False)
    t = n * dt
    w = (u0 + tau32 * gb)[:, None]
    assert np.allclose(run.v, w + (v0 - w) * math.exp(-t / tau32), rtol=1e-12, atol=1e-13)
    x_ref = x0 + w * t + tau32 * (v0 - w) * (1 - math.exp(-t / tau32))
    dxw = run.x - x_ref
    dxw -= box.L[0] * np.round(dxw / box.L[0])
    assert np.max(np.abs(dxw)) < 1e-12
    assert np.allclose(D * dt, box.m_p * (run.v - vb) - box.m_p * gb[:, None] * dt,
                       rtol=0, atol=1e-14)


def test_p10h_heun_integrator_exact_discrete_solution_and_order():
    """Heun (two stages) on a uniform carrier with a body force relaxes as
    v^n = w + (v0 - w) q^n, q = 1 - h + h^2/2 (h = dt/tau), with
    x^n = x0 + n dt w + dt (1 - h/2)(v0 - w)(1 - q^n)/(1 - q); its error against
    the continuous solution (eq. uncoupled_solution with an initial slip) is
    second order in dt.  The fluid receives the mean of the two stage drags."""
    u0 = np.array([0.3, -0.2, 0.1])
    gb = np.array([-0.9, 0.4, 2.0])
    tau = 0.05
    tau32 = float(np.float32(tau))
    w = (u0 + tau32 * gb)[:, None]
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        n = int(round(0.1 / dt))
        box = workloads.tiny_box(61, n=(16, 16, 16), np_=8, carrier="zero", tau=(tau,))
        u = np.zeros_like(box.u) + u0[:, None, None, None]
        P = _params(box, M=3, dt=dt, s=0)
        P.g = (type(P.g))(*gb)
        P.integrator = 2
        run = oracle.Run(P, u, box.x, box.v, box.tau)
        x0, v0 = box.x.copy(), box.v.copy()
        for _ in range(n - 1):
            run.step(want_f=False)
        vb = run.v.copy()
        _, D = run.step(want_f=False)
        h = dt / tau32
        q = 1 - h + h * h / 2
        assert np.allclose(run.v, w + (v0 - w) * q ** n, rtol=1e-12, atol=1e-13)
        x_ref = x0 + n * dt * w + dt * (1 - h / 2) * (v0 - w) * (1 - q ** n) / (1 - q)
        dxw = run.x - x_ref
        dxw -= box.L[0] * np.round(dxw / box.L[0])
        assert np.max(np.abs(dxw)) < 1e-12
        assert np.allclose(D * dt, box.m_p * (run.v - vb) - box.m_p * gb[:, None] * dt,
                           rtol=0, atol=1e-14)
        exact = w + (v0 - w) * math.exp(-n * dt / tau32)
        errs.append(np.max(np.abs(run.v - exact)))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_p10_continuum_limit_uncoupled_solution():
    """As dt -> 0 the discrete relaxation converges to the paper's one-way
    solution v = v_t (1 - e^{-t/tau_p}) (eq. uncoupled_solution), here for a
    particle released from rest in a uniform stream v_t."""
    tau = 0.05
    T = 0.1
    errs = []
    for dt in [1e-3, 5e-4]:
        n = int(round(T / dt))
        box = workloads.tiny_box(62, n=(16, 16, 16), np_=4, carrier="zero", tau=(tau,))
        u = np.zeros_like(box.u)
        u[0] = 0.8
        P = _params(box, M=2, dt=dt, s=0)
        run = oracle.Run(P, u, box.x, np.zeros_like(box.v), box.tau)
        for _ in range(n):
            run.step(want_f=False)
        exact = 0.8 * (1 - math.exp(-T / tau))
        errs.append(abs(run.v[0, 0] - exact))
    assert errs[0] < 2e-2 * 0.8
    assert 1.8 < errs[0] / errs[1] < 2.2      # first order in dt


def test_p11_startup_zero_forcing_and_no_self_correction():
    """No history before t=0: f = 0 for n < M, the self term vanishes for n <= M."""
    box = workloads.tiny_box(71, n=(16, 16, 16), np_=20)
    M = 3
    runs = []
    for s in (0, 1):
        P = _params(box, M=M, dt=1e-3, s=s)
        run = oracle.Run(P, box.u, box.x, box.v, box.tau)
        out = [run.step() for _ in range(M + 3)]
        runs.append(out)
    for n in range(M + 3):
        f0, D0 = runs[0][n]
        f1, D1 = runs[1][n]
        if n < M:
            assert not np.any(f0) and not np.any(f1)
        else:
            assert np.any(f0)
        if n <= M:
            assert np.array_equal(D0, D1)
        else:
            assert not np.array_equal(D0, D1)


def test_lees_edwards_velocity_jump():
    box = workloads.tiny_box(72, n=(16, 16, 16), np_=2, carrier="zero", shear=1.0)
    L = box.L[1]
    x = np.array([[0.5, 0.5], [L - 1e-4, 1e-4], [0.5, 0.5]])
    v = np.array([[0.0, 0.0], [1.0, -1.0], [0.0, 0.0]])
    P = _params(box, M=2, dt=1e-3, s=0)
    run = oracle.Run(P, box.u, x, v, box.tau)
    run.step(want_f=False)
    assert run.x[1, 0] < 0.01 and run.x[1, 1] > L - 0.01
    # the drag pulls v_x towards the mean flow; the jump adds -S L / +S L
    assert run.v[0, 0] < -0.9 * L and run.v[0, 1] > 0.9 * L


# -------------------------------------------------------------------- bin ---

def test_p12_bin_invariants():
    box = workloads.tiny_box(81, n=(24, 20, 18), np_=500, placement="clustered")
    P = _params(box)
    x = box.x.copy()
    x[0, :3] = [0.0, box.L[0] * (1 - 1e-17), -1e-18]   # edges
    key, start, perm = oracle.bin_cells(P, x)
    nc = 24 * 20 * 18
    assert start[0] == 0 and start[-1] == box.np_
    assert np.all(np.diff(start) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(box.np_))
    for c in np.unique(key):
        members = perm[start[c]:start[c + 1]]
        assert np.all(key[members] == c)
        assert np.all(np.diff(members) > 0)             # stable
    i = key % 24
    j = (key // 24) % 20
    k = key // (24 * 20)
    xw = np.mod(x, np.array(box.L)[:, None])
    xw = np.where(xw >= np.array(box.L)[:, None], xw - np.array(box.L)[:, None], xw)
    for d, idx in enumerate((i, j, k)):
        lo = idx * box.dx[d]
        assert np.all(xw[d] >= lo - 1e-12)
        assert np.all(xw[d] < lo + box.dx[d] + 1e-12)
    assert np.all((key >= 0) & (key < nc))


# --------------------------------------------------------------- workloads --

def test_k53_field_is_divergence_free_and_scaled():
    spec = workloads.BoxSpec(n=(32, 32, 32), L=(2 * math.pi,) * 3, np_=10, urms=0.7,
                             kmax=10.0, seed=5)
    box = workloads.make_box(spec)
    u = box.u
    assert abs(math.sqrt(np.mean(np.sum(u * u, axis=0)) / 3) - 0.7) < 1e-12
    k = np.fft.fftfreq(32, 1.0 / 32)
    uh = [np.fft.fftn(u[c]) for c in range(3)]
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    div = KX * uh[0] + KY * uh[1] + KZ * uh[2]
    assert np.max(np.abs(div)) < 1e-9 * np.max(np.abs(uh[0]))


# ------------------------------------------------------------- Faxen term --

def test_p13_self_laplacian_is_the_laplacian_of_the_app_e_closed_form():
    """The Faxen term needs lap v_self.  Its closed form (the Gaussian's second
    derivatives through the projection) against a fourth-order finite-difference
    Laplacian of the App. B tensor form of the App. E disturbance."""
    box = workloads.tiny_box(81, n=(32, 32, 32), np_=1, sigma_dx=1.5)
    dt = 2e-3
    P = _params(box, M=2, dt=dt)
    s = math.sqrt(P.sigma ** 2 + 2 * P.nu * dt)
    rng = np.random.default_rng(5)
    D = np.array([0.7, -0.4, 1.1])
    h = 2e-3 * s
    for _ in range(12):
        r = rng.normal(size=3)
        r *= rng.uniform(0.2, 3.0) * s / np.linalg.norm(r)
        x = (np.array([0.5, 0.5, 0.5]) * np.array(box.L) + r)[:, None]
        Xp = (np.array([0.5, 0.5, 0.5]) * np.array(box.L))[:, None]
        got = oracle.self_laplacian(P, x, Xp, D[:, None])[:, 0]

        def v(rr):
            return brute.green_tensor_velocity(rr[:, None], D[:, None], s, dt, P.rho_f)[:, 0]
        lap = np.zeros(3)
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            lap += (-v(r + 2 * e) + 16 * v(r + e) - 30 * v(r) + 16 * v(r - e) - v(r - 2 * e)) \
                / (12 * h * h)
        assert np.allclose(got, lap, rtol=1e-5, atol=1e-6 * np.max(np.abs(lap)))


def test_p14_grid_laplacian_of_a_fourier_mode():
    """On the grid, the 7-point Laplacian of a Fourier mode is the mode times
    -sum_d (4/h_d^2) sin^2(k_d h_d/2); the interpolated value is that times the
    trilinear interpolation of the mode, and the symbol tends to -|k|^2 at
    second order in h."""
    errs = []
    for N in (16, 32):
        n, L = (N, N + 4, N - 2), (2.0, 2.5, 1.8)
        box = workloads.tiny_box(82, n=n, L=L, np_=50, carrier="zero")
        P = _params(box, M=2, dt=1e-3)
        m = (2, -1, 1)
        k = np.array([2 * math.pi * m[d] / L[d] for d in range(3)])
        h = np.array([L[d] / n[d] for d in range(3)])
        ax = [np.arange(n[d]) * h[d] for d in range(3)]
        z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        ph = np.cos(k[0] * x + k[1] * y + k[2] * z + 0.4)
        u = np.stack([ph, 2 * ph, -ph])
        sym = -np.sum(4 / h ** 2 * np.sin(k * h / 2) ** 2)
        got = oracle.grid_laplacian(P, u, box.x)
        want = sym * oracle.gather(P, u, box.x)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.max(np.abs(want)))
        errs.append(abs(sym / -(k @ k) - 1))
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_p15_faxen_term_enters_the_drag():
    """eq. force_particle, first line: D = m_p (u~ + (a_p^2/6) lap u~ - v)/tau.
    Before any self term exists (n <= M) a step with radius a_p differs from
    one without by m_p (a_p^2/6) lap u / tau in the drag."""
    box = workloads.tiny_box(83, n=(24, 24, 24), np_=30)
    dt, a = 1e-3, 0.05
    Ds = []
    for ap in (0.0, a):
        P = _params(box, M=3, dt=dt)
        P.a_p = ap
        run = oracle.Run(P, box.u, box.x, box.v, box.tau)
        _, D = run.step(want_f=False)
        Ds.append(D)
    P = _params(box, M=3, dt=dt)
    lap = oracle.grid_laplacian(P, box.u, box.x)
    tau = box.tau.astype(np.float64)[None, :]
    want = box.m_p * (a * a / 6.0) * lap / tau
    assert np.allclose(Ds[1] - Ds[0], want, rtol=1e-10, atol=1e-12 * np.max(np.abs(want)))
