"""The Basset history term (eq. force_particle, third line, its memory integral
over the last step only as Sec. 2.5 closes) through the C ABI
(erpp_plan_set_basset), against the oracle with the same term.

* Parity, coupling step alone (frozen k^-5/3 carrier, gravity, self-correction
  on, Faxen term on; alone and together with the added mass): forcing every step
  with the rel-L2 and node-by-node bars, velocities every step, positions at the
  end (FP32 f 1e-5, v 1e-6; FP64 1e-12, 1e-13).
* Parity in the two-way coupled loop (one graph per step), the term switched on
  after a few steps on both sides: v 1e-6 / 1e-12, u 1e-5 / 1e-12 rel-L2.
* The term must matter: without it the velocities differ by far more than the bar.
* Rejections: a sheared box, another integrator, a NULL history.
"""
import ctypes as C
import math

import numpy as np
import pytest

import oracle
from oracle import fluid as ofluid
from helpers import (assert_forcing_matches, carrier_for, periodic_diff, rel_l2,
                     tolerances, upload)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

erpp = pytest.importorskip("paper_1405_6969_amd")
import workloads  # noqa: E402

L = 2 * math.pi


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _box(seed, n=(32, 28, 24), np_=1500):
    spec = workloads.BoxSpec(n=n, L=(L, L * n[1] / n[0], L * n[2] / n[0]), np_=np_,
                             carrier="k53", kmax=8.0, tau=(0.02, 0.05), nu=0.05,
                             mass_loading=1.0, placement="clustered", n_blobs=5,
                             blob_radius_dx=3.0, seed=workloads.SEED_BASE + seed)
    return workloads.make_box(spec)


@pytest.mark.parametrize("prec", [erpp.F32_FAST, erpp.F64_PLAIN])
@pytest.mark.parametrize("added_mass", [False, True])
def test_basset_step_matches_oracle(prec, added_mass):
    _cuda()
    box = _box(301)
    M, dt, steps = 3, 2e-3, 12
    gb = (0.3, -1.0, 0.2)
    a = 1.5 * box.dx[0]
    db = upload(box, M, prec)
    P = oracle.params_for_box(box, M, dt, 1)
    P.g = (type(P.g))(*gb)
    P.a_p = a
    P.a_b = a
    if added_mass:
        P.a_am = a
    run = oracle.Run(P, carrier_for(box, prec), box.x, box.v, box.tau)
    tf, tv = tolerances(prec)
    with erpp.Plan([db], M, dt, precision=prec) as plan:
        plan.set_body_force(0, gb)
        plan.set_faxen(0, a)
        plan.set_basset(0, a)
        if added_mass:
            plan.set_added_mass(0, a)
        for n in range(steps):
            plan.step(n)
            fo, _ = run.step(want_f=True)
            if n >= M:
                assert_forcing_matches(db.f.double().cpu().numpy(), fo, prec, n)
            assert rel_l2(db.v.cpu().numpy(), run.v) <= tv, n
        torch.cuda.synchronize()
    ex = np.max(np.abs(periodic_diff(db.x.cpu().numpy(), run.x, box.L)))
    assert ex <= (1e-12 if prec == erpp.F64_PLAIN else steps * dt * tv * np.max(np.abs(run.v)))


@pytest.mark.parametrize("prec", [erpp.F32_FAST, erpp.F64_PLAIN])
def test_basset_coupled_matches_oracle(prec):
    _cuda()
    box = _box(302, n=(32, 32, 32))
    M, dt, steps, on_at = 3, 2e-3, 12, 4
    a = 1.2 * box.dx[0]
    out = {}
    for use in (False, True):
        db = upload(box, M, prec)
        with erpp.Plan([db], M, dt, precision=prec) as plan, \
                erpp.Fluid(box.n, box.L, box.spec.nu, dt, precision=prec) as fl:
            plan.set_faxen(0, a)
            plan.run_coupled([fl], 0, on_at, graph=True)
            if use:
                plan.set_basset(0, a)
            plan.run_coupled([fl], on_at, steps - on_at, graph=True)
            torch.cuda.synchronize()
            out[use] = (db.v.cpu().numpy(), db.u.double().cpu().numpy())
    P = oracle.params_for_box(box, M, dt, 1)
    P.a_p = a
    run = oracle.Run(P, carrier_for(box, prec), box.x, box.v, box.tau)
    for n in range(steps):
        if n == on_at:
            run.P.a_b = a
        f, _ = run.step(want_f=True)
        run.u = ofluid.fluid_step(box.n, box.L, box.spec.nu, dt, run.u, f)
    v, u = out[True]
    ev, eu = rel_l2(v, run.v), rel_l2(u, run.u)
    effect = rel_l2(out[False][0], run.v)
    print(f"prec {prec}: Basset v {ev:.3e}, u {eu:.3e}; without it v differs by {effect:.3e}")
    tv, tu = (1e-12, 1e-12) if prec == erpp.F64_PLAIN else (1e-6, 1e-5)
    assert ev <= tv and eu <= tu
    assert effect > 100 * tv


def test_basset_rejections():
    _cuda()
    spec = workloads.BoxSpec(n=(16, 16, 16), L=(L, L, L), np_=50, carrier="k53", kmax=4.0,
                             tau=(0.05, 0.05), nu=0.05, mass_loading=0.1, placement="uniform",
                             shear=1.0, seed=workloads.SEED_BASE + 7)
    db = upload(workloads.make_box(spec), 2, erpp.F32_FAST)
    with erpp.Plan([db], 2, 1e-3) as plan:
        with pytest.raises(erpp.ErppError) as e:
            plan.set_basset(0, 0.1)
        assert e.value.status == erpp.ERPP_EUNSUPPORTED
    box = _box(303, n=(16, 16, 16), np_=50)
    db = upload(box, 2, erpp.F32_FAST)
    with erpp.Plan([db], 2, 1e-3) as plan:
        plan.set_integrator(erpp.HEUN)
        with pytest.raises(erpp.ErppError) as e:
            plan.set_basset(0, 0.1)
        assert e.value.status == erpp.ERPP_EUNSUPPORTED
        plan.set_integrator(erpp.EULER)
        plan.set_basset(0, 0.1)
        with pytest.raises(erpp.ErppError) as e:
            plan.set_integrator(erpp.EXPONENTIAL)
        assert e.value.status == erpp.ERPP_EUNSUPPORTED
        lib = erpp.load()
        assert lib.erpp_plan_set_basset(plan.h, 0, C.c_double(0.1), None) == erpp.ERPP_EINVAL
        assert lib.erpp_plan_set_basset(plan.h, 0, C.c_double(-0.1), None) == erpp.ERPP_EINVAL
        plan.set_basset(0, 0.0)
