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


def _terminal_error(N, sigma, ratio, prec=erpp.F32_FAST, self_correction=1, T=6 * TAU):
    db, plan, fl, dt, _, _ = _setup(N, sigma, ratio, prec, self_correction)
    K = int(round(T / dt))
    with plan, fl:
        plan.run_coupled([fl], 0, K, graph=True)
        torch.cuda.synchronize()
    tau32 = float(np.float32(TAU))
    v_ref = tau32 * G * (1 - (1 - dt / tau32) ** K)
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
