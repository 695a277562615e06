"""The settling particle of Sec. 3.2 in the coupled regime, through the C ABI:
erpp_plan_set_body_force for gravity, erpp_run_coupled for the coupling step
plus the App. E fluid step.

* Parity: the velocity history of the particle and the final fluid field
  against the oracle's coupled loop (bars: FP64 1e-12, FP32 1e-6 on v and
  1e-5 on u).
* The paper's figure cases (box 2 pi, sigma_R fixed by a 24^3 grid): the
  terminal velocity approaches v_t as d_p / sigma_R decreases, first order;
  removing the self-disturbance lowers the error; the result is the same on
  24^3 and 48^3 grids; with sigma_R below the grid spacing it stays small.
Velocities are relative to the box-mean fluid velocity.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fluid as ofluid
from helpers import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

erpp = pytest.importorskip("paper_1405_6969_amd")

NU, RHO, TAU, G, M = 1.0, 1.0, 0.2, 0.5, 4
L = 2 * math.pi


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(N, sigma, ratio, prec, self_correction=1):
    dx = L / N
    eps = sigma ** 2 / (2 * NU)
    dt = eps / M
    m_p = 3 * math.pi * RHO * NU * ratio * sigma * TAU
    x = np.array([[L / 2 + 0.3 * dx], [L / 2], [L / 2]])
    db = erpp.device_box((N,) * 3, (L,) * 3, x, np.zeros((3, 1)), np.array([TAU], np.float32),
                         np.zeros((3, N, N, N)), M, m_p, RHO, NU, sigma, precision=prec)
    plan = erpp.Plan([db], M, dt, precision=prec, self_correction=self_correction)
    plan.set_body_force(0, (G, 0.0, 0.0))
    fl = erpp.Fluid((N,) * 3, (L,) * 3, NU, dt, precision=prec)
    return db, plan, fl, dt, m_p, x


def _terminal_error(N, sigma, ratio, prec=erpp.F32_FAST, self_correction=1, T=6 * TAU,
                    integrator=None):
    db, plan, fl, dt, _, _ = _setup(N, sigma, ratio, prec, self_correction)
    K = int(round(T / dt))
    with plan, fl:
        if integrator is not None:
            plan.set_integrator(integrator)
        plan.run_coupled([fl], 0, K, graph=True)
        torch.cuda.synchronize()
    tau32 = float(np.float32(TAU))
    h = dt / tau32
    # the discrete uncoupled solution of the scheme: amplification 1 - h (Euler),
    # 1 - h + h^2/2 (Heun)
    q = 1 - h + h * h / 2 if integrator == erpp.HEUN else 1 - h
    v_ref = tau32 * G * (1 - q ** K)
    v = db.v[0, 0].item() - db.u[0].double().mean().item()
    return v / v_ref - 1.0


@pytest.mark.parametrize("prec", [erpp.F32_FAST, erpp.F64_PLAIN])
def test_settling_matches_oracle(prec):
    _cuda()
    N, sigma, ratio = 32, L / 16, 0.25
    db, plan, fl, dt, m_p, x = _setup(N, sigma, ratio, prec)
    P = oracle.make_params((N,) * 3, (L,) * 3, 1, m_p, RHO, NU, sigma, 3.0, 0.0, M, dt, 1,
                           g=(G, 0.0, 0.0))
    run = oracle.Run(P, np.zeros((3, N, N, N)), x, np.zeros((3, 1)), np.array([TAU], np.float32))
    K = 40
    vg, vo = [], []
    with plan, fl:
        for n in range(K):
            plan.run_coupled([fl], n, 1, graph=False)
            vg.append(db.v[:, 0].cpu().numpy().copy())
            f, _ = run.step(want_f=True)
            run.u = ofluid.fluid_step((N,) * 3, (L,) * 3, NU, dt, run.u, f)
            vo.append(run.v[:, 0].copy())
        torch.cuda.synchronize()
        u = db.u.double().cpu().numpy()
    vg, vo = np.array(vg), np.array(vo)
    ev, eu = rel_l2(vg, vo), rel_l2(u, run.u)
    print(f"prec {prec}: velocity history rel-L2 {ev:.3e}, fluid {eu:.3e}")
    if prec == erpp.F64_PLAIN:
        assert ev <= 1e-12 and eu <= 1e-12
    else:
        assert ev <= 1e-6 and eu <= 1e-5


def test_settling_error_vs_dp_over_sigma():
    """Terminal-velocity error against d_p / sigma_R (0.5 .. 0.0625), sigma_R =
    2 pi / 24 on a 24^3 grid, with and without the removal of the
    self-disturbance (FP32 path)."""
    _cuda()
    sigma = L / 24
    ratios = [0.5, 0.25, 0.125, 0.0625]
    on = [_terminal_error(24, sigma, r) for r in ratios]
    off = [_terminal_error(24, sigma, r, self_correction=0) for r in ratios]
    print("d_p/sigma_R:", ratios)
    print("error with removal:   ", [f"{e:.4f}" for e in on])
    print("error without removal:", [f"{e:.4f}" for e in off])
    for a, b in zip(on, on[1:]):
        assert 1.8 < a / b < 2.2                       # first order in d_p / sigma_R
    assert on[-1] < 0.02
    assert all(b > a > 0 for a, b in zip(on, off))    # the removal lowers the error


def test_settling_grid_independent_at_fixed_sigma():
    """Same sigma_R on 24^3 (sigma_R/Dx = 1) and 48^3 (sigma_R/Dx = 2, the
    widest stencil the library takes at this sigma_R)."""
    _cuda()
    sigma = L / 24
    e24 = _terminal_error(24, sigma, 0.25)
    e48 = _terminal_error(48, sigma, 0.25)
    print(f"24^3: {e24:.4f}, 48^3: {e48:.4f}")
    assert abs(e24 - e48) < 5e-3


def test_settling_unresolved_sigma():
    """d_p / sigma_R = 0.0625 on a 48^3 grid with sigma_R / Dx = 1, 0.5, 0.3
    (0.3 is about the smallest ratio whose 3 sigma sphere always holds a node).
    The paper reports a loss of accuracy once the kernel is not resolved.  With
    the per-particle lattice normalisation used here the deposited impulse stays
    exact, and the measured terminal-velocity error stays at the resolved
    level (1.8%, 2.0%, 1.8%); the test keeps it below 3%."""
    _cuda()
    dx = L / 48
    errs = [_terminal_error(48, s * dx, 0.0625) for s in (1.0, 0.5, 0.3)]
    print("sigma_R/Dx 1, 0.5, 0.3:", [f"{e:.4f}" for e in errs])
    assert all(0.0 < e < 0.03 for e in errs)


@pytest.mark.parametrize("prec", [erpp.F32_FAST, erpp.F64_PLAIN])
def test_exponential_integrator_matches_oracle(prec):
    """ERPP_EXPONENTIAL through the coupling step (frozen k^-5/3 carrier, gravity,
    Stokes times 0.01 and 0.05 with dt = 0.03, where explicit Euler diverges for
    the first population), 12 steps, against the oracle with the same
    integrator.  Bars of the coupling step: f 1e-5 / 1e-12, v 1e-6 / 1e-13;
    x within steps * dt * (v bar) * max|v| (FP32) and 1e-12 (FP64)."""
    _cuda()
    import workloads
    from helpers import assert_forcing_matches, carrier_for, periodic_diff, tolerances, upload
    spec = workloads.BoxSpec(n=(32, 28, 24), L=(2 * math.pi, 2 * math.pi * 28 / 32,
                                                 2 * math.pi * 24 / 32), np_=1500,
                             carrier="k53", kmax=6.0, tau=(0.01, 0.05), nu=0.05,
                             mass_loading=0.5, placement="clustered", n_blobs=5,
                             blob_radius_dx=3.0, seed=workloads.SEED_BASE + 77)
    box = workloads.make_box(spec)
    M, dt, steps = 3, 0.03, 12
    gb = (0.3, -1.0, 0.2)
    db = upload(box, M, prec)
    P = oracle.params_for_box(box, M, dt, 1)
    P.g = (type(P.g))(*gb)
    P.integrator = 1
    run = oracle.Run(P, carrier_for(box, prec), box.x, box.v, box.tau)
    tf, tv = tolerances(prec)
    with erpp.Plan([db], M, dt, precision=prec) as plan:
        plan.set_body_force(0, gb)
        plan.set_integrator(erpp.EXPONENTIAL)
        for n in range(steps):
            plan.step(n)
            fo, _ = run.step(want_f=True)
            if n >= M:
                assert_forcing_matches(db.f.double().cpu().numpy(), fo, prec, n)
        torch.cuda.synchronize()
    assert rel_l2(db.v.cpu().numpy(), run.v) <= tv
    # positions take dt (u~ + tau g_b) directly: the displacement the velocity bar allows
    ex = np.max(np.abs(periodic_diff(db.x.cpu().numpy(), run.x, box.L)))
    assert ex <= (1e-12 if prec == erpp.F64_PLAIN else steps * dt * tv * np.max(np.abs(run.v)))


def test_exponential_integrator_settles_with_large_steps():
    """The coupled settling particle with tau_p = dt / 3 (explicit Euler would
    diverge): the exponential integrator relaxes to the continuous uncoupled
    solution v_t (1 - e^{-t/tau_p}) within the d_p / sigma_R error of the
    scheme (d_p / sigma_R = 0.125)."""
    _cuda()
    N, sigma, ratio = 24, L / 24, 0.125
    eps = sigma ** 2 / (2 * NU)
    dt = eps / M
    tau = dt / 3
    m_p = 3 * math.pi * RHO * NU * ratio * sigma * tau
    dx = L / N
    x = np.array([[L / 2 + 0.3 * dx], [L / 2], [L / 2]])
    db = erpp.device_box((N,) * 3, (L,) * 3, x, np.zeros((3, 1)), np.array([tau], np.float32),
                         np.zeros((3, N, N, N)), M, m_p, RHO, NU, sigma)
    K = 60
    with erpp.Plan([db], M, dt) as plan, erpp.Fluid((N,) * 3, (L,) * 3, NU, dt) as fl:
        plan.set_body_force(0, (G, 0.0, 0.0))
        plan.set_integrator(erpp.EXPONENTIAL)
        plan.run_coupled([fl], 0, K, graph=True)
        torch.cuda.synchronize()
    tau32 = float(np.float32(tau))
    v_t = tau32 * G
    v = db.v[0, 0].item() - db.u[0].double().mean().item()
    err = v / (v_t * (1 - math.exp(-K * dt / tau32))) - 1
    print(f"exponential integrator, dt/tau = 3: terminal error {err:.4f}")
    assert np.isfinite(err) and 0.0 < err < 0.06


@pytest.mark.parametrize("prec", [erpp.F32_FAST, erpp.F64_PLAIN])
def test_faxen_term_matches_oracle(prec):
    """The Faxen correction (eq. force_particle, first line) in the two-way
    coupled loop: k^-5/3 carrier, particle radius 0.6 dx, 12 coupled steps,
    against the oracle's coupled loop with the same radius.  Bars: the coupled
    test's (v 1e-6 / 1e-12, u 1e-5 / 1e-12).  The term must matter: the run
    without it differs by far more than the bar."""
    _cuda()
    import workloads
    from helpers import carrier_for, upload
    n = (32, 32, 32)
    spec = workloads.BoxSpec(n=n, L=(L,) * 3, np_=1500, carrier="k53", kmax=10.0,
                             tau=(0.02, 0.05), nu=0.05, mass_loading=2.0, placement="clustered",
                             n_blobs=6, blob_radius_dx=3.0, seed=workloads.SEED_BASE + 91)
    box = workloads.make_box(spec)
    Mx, dt, steps = 3, 2e-3, 12
    a_p = 0.6 * box.dx[0]
    out = {}
    for ap in (0.0, a_p):
        db = upload(box, Mx, prec)
        with erpp.Plan([db], Mx, dt, precision=prec) as plan, \
                erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=prec) as fl:
            if ap > 0:
                # a graph captured before the radius is set must not be reused
                plan.run_coupled([fl], 0, 0, graph=True)
            plan.set_faxen(0, ap)
            plan.run_coupled([fl], 0, steps, graph=True)
            torch.cuda.synchronize()
        out[ap] = (db.v.cpu().numpy(), db.u.double().cpu().numpy())
    P = oracle.params_for_box(box, Mx, dt, 1)
    P.a_p = a_p
    run = oracle.Run(P, carrier_for(box, prec), box.x, box.v, box.tau)
    for _ in range(steps):
        f, _ = run.step(want_f=True)
        run.u = ofluid.fluid_step(box.n, box.L, box.spec.nu, dt, run.u, f)
    v, u = out[a_p]
    ev, eu = rel_l2(v, run.v), rel_l2(u, run.u)
    effect = rel_l2(out[0.0][0], run.v)
    print(f"prec {prec}: Faxen v {ev:.3e}, u {eu:.3e}; without the term v differs by {effect:.3e}")
    tv, tu = (1e-12, 1e-12) if prec == erpp.F64_PLAIN else (1e-6, 1e-5)
    assert ev <= tv and eu <= tu
    assert effect > 100 * tv


@pytest.mark.parametrize("prec", [erpp.F32_FAST, erpp.F64_PLAIN])
@pytest.mark.parametrize("a_p_dx", [0.0, 0.6])
def test_heun_integrator_matches_oracle(prec, a_p_dx):
    """ERPP_HEUN (two stages, the self term removed at each, Sec. 2.5) in the
    two-way coupled loop: k^-5/3 carrier, gravity, with and without the Faxen
    correction (evaluated at both stages), 12 coupled steps against the
    oracle's coupled loop with the same integrator.  Bars: v 1e-6 / 1e-12,
    u 1e-5 / 1e-12; x within steps * dt * (v bar) * max|v| (FP32) and 1e-12
    (FP64).  A graph captured under Euler must not be replayed afterwards."""
    _cuda()
    import workloads
    from helpers import carrier_for, periodic_diff, upload
    spec = workloads.BoxSpec(n=(32, 28, 24), L=(L, L * 28 / 32, L * 24 / 32), np_=1500,
                             carrier="k53", kmax=8.0, tau=(0.02, 0.05), nu=0.05,
                             mass_loading=1.0, placement="clustered", n_blobs=5,
                             blob_radius_dx=3.0, seed=workloads.SEED_BASE + 123)
    box = workloads.make_box(spec)
    Mx, dt, steps = 3, 4e-3, 12
    gb = (0.3, -1.0, 0.2)
    a_p = a_p_dx * box.dx[0]
    db = upload(box, Mx, prec)
    with erpp.Plan([db], Mx, dt, precision=prec) as plan, \
            erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=prec) as fl:
        plan.set_body_force(0, gb)
        plan.run_coupled([fl], 0, 0, graph=True)
        plan.set_integrator(erpp.HEUN)
        if a_p > 0:
            plan.set_faxen(0, a_p)
        plan.run_coupled([fl], 0, steps, graph=True)
        torch.cuda.synchronize()
        v, u, x = db.v.cpu().numpy(), db.u.double().cpu().numpy(), db.x.cpu().numpy()
    P = oracle.params_for_box(box, Mx, dt, 1)
    P.g = (type(P.g))(*gb)
    P.integrator = 2
    P.a_p = a_p
    run = oracle.Run(P, carrier_for(box, prec), box.x, box.v, box.tau)
    for _ in range(steps):
        f, _ = run.step(want_f=True)
        run.u = ofluid.fluid_step(box.n, box.L, box.spec.nu, dt, run.u, f)
    ev, eu = rel_l2(v, run.v), rel_l2(u, run.u)
    ex = np.max(np.abs(periodic_diff(x, run.x, box.L)))
    print(f"prec {prec}, a_p/dx {a_p_dx}: Heun v {ev:.3e}, u {eu:.3e}, x {ex:.3e}")
    tv, tu = (1e-12, 1e-12) if prec == erpp.F64_PLAIN else (1e-6, 1e-5)
    assert ev <= tv and eu <= tu
    assert ex <= (1e-12 if prec == erpp.F64_PLAIN else steps * dt * tv * np.max(np.abs(run.v)))


def test_heun_settling_error_first_order():
    """The settling particle with Heun and the stage-wise removal (24^3,
    sigma_R = 2 pi / 24): the terminal-velocity error against the scheme's
    discrete uncoupled solution is first order in d_p / sigma_R, and lower than
    without the removal."""
    _cuda()
    sigma = L / 24
    on = [_terminal_error(24, sigma, r, integrator=erpp.HEUN) for r in (0.25, 0.125)]
    off = _terminal_error(24, sigma, 0.25, self_correction=0, integrator=erpp.HEUN)
    print(f"Heun: error {on[0]:.4f}, {on[1]:.4f} at d_p/sigma_R 0.25, 0.125; "
          f"{off:.4f} without removal")
    assert 0.0 < on[1] < on[0] < 0.06
    assert 1.8 < on[0] / on[1] < 2.2
    assert off > on[0]


def test_heun_rejects_sheared_box():
    _cuda()
    import workloads
    from helpers import upload
    spec = workloads.BoxSpec(n=(16, 16, 16), L=(L, L, L), np_=50, carrier="k53",
                             kmax=4.0, tau=(0.05, 0.05), nu=0.05, mass_loading=0.1,
                             placement="uniform", shear=1.0, seed=workloads.SEED_BASE + 5)
    db = upload(workloads.make_box(spec), 2, erpp.F32_FAST)
    with erpp.Plan([db], 2, 1e-3) as plan:
        with pytest.raises(erpp.ErppError) as e:
            plan.set_integrator(erpp.HEUN)
        assert e.value.status == erpp.ERPP_EUNSUPPORTED
        plan.set_integrator(erpp.EXPONENTIAL)
