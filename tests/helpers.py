"""Shared helpers of the GPU parity tests: upload a seeded box, run the oracle
on the same arrays, compare."""
from __future__ import annotations

import numpy as np

import oracle
import workloads


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return 0.0 if np.linalg.norm(a) == 0.0 else np.inf
    return float(np.linalg.norm(a - b) / nb)


def carrier_for(box, precision):
    """The carrier both sides consume: FP32-rounded for the FP32 path."""
    import paper_1405_6969_amd as erpp
    if precision == erpp.F32_FAST:
        return box.u.astype(np.float32).astype(np.float64)
    return box.u


def upload(box, M, precision, device="cuda"):
    import paper_1405_6969_amd as erpp
    s = box.spec
    return erpp.device_box(box.n, box.L, box.x, box.v, box.tau, carrier_for(box, precision), M,
                           box.m_p, s.rho_f, s.nu, box.sigma, s.cutoff, s.shear,
                           precision=precision, device=device)


def oracle_run(box, M, dt, self_correction, precision):
    P = oracle.params_for_box(box, M, dt, self_correction)
    return oracle.Run(P, carrier_for(box, precision), box.x, box.v, box.tau)


def tolerances(precision):
    import paper_1405_6969_amd as erpp
    if precision == erpp.F32_FAST:
        return 1e-5, 1e-6
    return 1e-12, 1e-13


def periodic_diff(a, b, L):
    d = np.asarray(a) - np.asarray(b)
    Ls = np.asarray(L, dtype=np.float64)[:, None]
    return d - Ls * np.round(d / Ls)
