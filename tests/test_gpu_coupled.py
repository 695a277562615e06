"""Two-way coupled steps (erpp_run_coupled): the coupling step of every box
followed by its fluid step, against the FP64 oracle running the same loop
(oracle.Run for the coupling, oracle.fluid.fluid_step for the fluid).

Bars (written here): ERPP_F64_PLAIN rel-L2 of v and u <= 1e-12;
ERPP_F32_FAST rel-L2(v) <= 1e-6 and rel-L2(u) <= 1e-5 after 14 steps, positions
within steps * dt * 1e-6 * max|v|.
The momentum balance of the coupled system is checked on the GPU result:
particles plus fluid change by dt times the drag still in the history ring.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import fluid as ofluid
from helpers import carrier_for, oracle_run, periodic_diff, rel_l2, upload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

erpp = pytest.importorskip("paper_1405_6969_amd")
PRECS = [erpp.F32_FAST, erpp.F64_PLAIN]


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _box(seed=3, n=(32, 32, 32), np_=1500, carrier="taylor_green", loading=2.0):
    spec = workloads.BoxSpec(n=n, L=tuple(2 * math.pi * s / n[0] for s in n), np_=np_,
                             carrier=carrier, kmax=6.0, tau=(0.02, 0.05), nu=0.05,
                             mass_loading=loading, placement="clustered", n_blobs=6,
                             blob_radius_dx=3.0, seed=workloads.SEED_BASE + seed)
    return workloads.make_box(spec)


def _momentum(db, box, rho):
    dV = np.prod(box.dx)
    v = db.v.double().cpu().numpy()
    u = db.u.double().cpu().numpy()
    return box.m_p * v.sum(axis=1) + rho * dV * u.reshape(3, -1).sum(axis=1), \
        box.m_p * np.abs(v).sum() + rho * dV * np.abs(u).sum()


@pytest.mark.parametrize("prec", PRECS)
def test_coupled_steps_match_oracle(prec):
    _cuda()
    box = _box()
    M, dt, steps = 4, 2e-3, 14
    db = upload(box, M, prec)
    run = oracle_run(box, M, dt, 1, prec)
    P0, _ = _momentum(db, box, box.spec.rho_f)
    with erpp.Plan([db], M, dt, precision=prec) as plan, \
            erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=prec) as fl:
        plan.run_coupled([fl], 0, steps, graph=False)
        torch.cuda.synchronize()
    for _ in range(steps):
        f, _D = run.step(want_f=True)
        run.u = ofluid.fluid_step(box.n, box.L, box.spec.nu, dt, run.u, f)
    v = db.v.cpu().numpy()
    x = db.x.cpu().numpy()
    u = db.u.double().cpu().numpy()
    ev, eu = rel_l2(v, run.v), rel_l2(u, run.u)
    ex = np.max(np.abs(periodic_diff(x, run.x, box.L)))
    print(f"prec {prec}: rel-L2 v {ev:.3e}, u {eu:.3e}, max |dx| {ex:.3e}")
    if prec == erpp.F64_PLAIN:
        assert ev <= 1e-12 and eu <= 1e-12 and ex <= 1e-12
    else:
        # positions: the displacement that the velocity bar allows, per particle
        assert ev <= 1e-6 and eu <= 1e-5
        assert ex <= steps * dt * 1e-6 * np.max(np.abs(run.v))
    # the disturbance is not negligible: the fluid moved away from the carrier
    assert rel_l2(u, carrier_for(box, prec)) > 1e-3
    # momentum: particles + fluid change by dt * (drag levels not yet injected),
    # i.e. every ring level except the oldest one (n = steps - M - 1)
    P1, scale = _momentum(db, box, box.spec.rho_f)
    ring = db.ring_d.double().cpu().numpy()
    oldest = (steps - M - 1) % (M + 1)
    inflight = dt * (ring.sum(axis=(0, 2)) - ring[oldest].sum(axis=1))
    # FP32: each transform rounds the mean at ~eps32 log2(nodes) of sum |u|
    tol = 1e-13 if prec == erpp.F64_PLAIN else 2e-5
    assert np.allclose(P1 - P0, inflight, rtol=0, atol=tol * scale), (P1 - P0, inflight)


@pytest.mark.parametrize("prec", PRECS)
def test_coupled_graph_replays_match_eager(prec):
    """The captured coupled step, replayed in three chunks with unrelated eager
    work and synchronisation in between, gives the eager result after every
    chunk (bit for bit on the deterministic FP32 path; to 1e-13 on the FP64
    path, whose global atomics add in any order)."""
    _cuda()
    box = _box(seed=9, n=(40, 36, 32), np_=2000, carrier="k53")
    M, dt = 3, 1e-3
    da, dg = upload(box, M, prec), upload(box, M, prec)
    with erpp.Plan([da], M, dt, precision=prec) as pa, erpp.Plan([dg], M, dt, precision=prec) as pg, \
            erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=prec) as fa, \
            erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=prec) as fg:
        step = 0
        for chunk in range(3):
            pa.run_coupled([fa], step, 4, graph=False)
            pg.run_coupled([fg], step, 4, graph=True)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
            torch.cuda.synchronize()
            step += 4
            for name in ("u", "v", "x"):
                a = getattr(da, name).double().cpu().numpy()
                g = getattr(dg, name).double().cpu().numpy()
                if prec == erpp.F32_FAST:
                    assert np.array_equal(a, g), (chunk, name)
                else:
                    assert rel_l2(g, a) <= 1e-13, (chunk, name)
        del junk


def test_coupled_rejects_mismatched_fluid():
    _cuda()
    box = _box()
    M, dt = 2, 1e-3
    db = upload(box, M, erpp.F32_FAST)
    with erpp.Plan([db], M, dt) as plan:
        bad = [erpp.Fluid(box.n, box.L, box.spec.nu * 2, dt),           # viscosity
               erpp.Fluid(box.n, box.L, box.spec.nu, dt * 2),           # step
               erpp.Fluid((32, 32, 30), box.L, box.spec.nu, dt),        # grid
               erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=erpp.F64_PLAIN)]
        for fl in bad:
            with pytest.raises(erpp.ErppError) as ei:
                plan.run_coupled([fl], 0, 1)
            assert ei.value.status == erpp.ERPP_EINVAL
            fl.close()
