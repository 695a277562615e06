"""Shared helpers of the GPU parity tests: upload a seeded box, run the oracle
on the same arrays, compare."""
from __future__ import annotations

import math

import numpy as np

import oracle
from oracle import brute
import workloads


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return 0.0 if np.linalg.norm(a) == 0.0 else np.inf
    return float(np.linalg.norm(a - b) / nb)


def forcing_errors(fg, fo):
    """Node-by-node comparison of a GPU forcing with the oracle's: the largest
    error over nodes and components relative to the largest oracle value, the
    nodes where the oracle is exactly zero but the GPU is not, and the nodes
    where the oracle exceeds 1e-6 of its largest value but the GPU is zero."""
    fg = np.asarray(fg, dtype=np.float64)
    fo = np.asarray(fo, dtype=np.float64)
    mo = float(np.max(np.abs(fo))) if fo.size else 0.0
    if mo == 0.0:
        return (0.0 if not np.any(fg) else np.inf), int(np.count_nonzero(fg)), 0
    err = float(np.max(np.abs(fg - fo))) / mo
    extra = int(np.count_nonzero((fo == 0) & (fg != 0)))
    lost = int(np.count_nonzero((np.abs(fo) > 1e-6 * mo) & (fg == 0)))
    return err, extra, lost


def node_tolerance(precision):
    """Per-node bar on the forcing, relative to the largest oracle value."""
    import paper_1405_6969_amd as erpp
    return 1e-5 if precision == erpp.F32_FAST else 1e-12


def assert_forcing_matches(fg, fo, precision, what=""):
    """rel-L2 and node-by-node bars, and the same set of touched nodes."""
    tol_f, _ = tolerances(precision)
    e2 = rel_l2(fg, fo)
    assert e2 <= tol_f, (what, "rel-L2", e2)
    err, extra, lost = forcing_errors(fg, fo)
    assert err <= node_tolerance(precision), (what, "max node error", err)
    assert extra == 0 and lost == 0, (what, "node set", extra, lost)
    return e2, err


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


def window_particles(box, lo, wn, margin):
    """Indices of the particles whose position lies within `margin` of the node
    window [lo, lo + wn) (periodic), the only ones whose stencil can reach it."""
    keep = np.ones(box.np_, bool)
    for d in range(3):
        c = (lo[d] + 0.5 * (wn[d] - 1)) * box.dx[d]
        dd = box.x[d] - c
        dd -= box.L[d] * np.round(dd / box.L[d])
        keep &= np.abs(dd) <= 0.5 * (wn[d] - 1) * box.dx[d] + margin
    return np.nonzero(keep)[0]


def sampled_parity(box, db, M, dt, steps, precision, rng, nsample=4000, wn=(24, 24, 24),
                   self_correction=1):
    """Oracle on subsets after `steps` steps of the GPU path on the whole box.

    The carrier is frozen, so particles are independent: the oracle run on a
    subset reproduces that subset exactly.  (a) v and x of `nsample` random
    particles; (b) the forcing of the last step on a node window, from every
    particle that can reach it (3 sigma plus the largest drift over the run).
    Returns (rel-L2 of v, max periodic |dx|, rel-L2 of f on the window, largest
    node error of f on the window relative to its largest oracle value); the
    window's touched-node set is asserted equal."""
    import torch
    P = oracle.params_for_box(box, M, dt, self_correction)
    u = carrier_for(box, precision)
    sample = rng.choice(box.np_, size=min(nsample, box.np_), replace=False)
    run = oracle.Run(P, u, box.x[:, sample], box.v[:, sample], box.tau[sample])
    for _ in range(steps):
        run.step(want_f=False)
    torch.cuda.synchronize()
    ev = rel_l2(db.v.cpu().numpy()[:, sample], run.v)
    ex = float(np.max(np.abs(periodic_diff(db.x.cpu().numpy()[:, sample], run.x, box.L))))
    wn = tuple(min(wn[d], box.n[d]) for d in range(3))
    lo = tuple(int(rng.integers(0, n)) for n in box.n)
    vmax = float(np.max(np.abs(box.v))) + float(np.max(np.abs(box.u))) \
        + abs(box.spec.shear) * box.L[1]
    margin = box.spec.cutoff * box.sigma + 2.0 * vmax * steps * dt + 2 * max(box.dx)
    idx = window_particles(box, lo, wn, margin)
    run2 = oracle.Run(P, u, box.x[:, idx], box.v[:, idx], box.tau[idx])
    for _ in range(steps - 1):
        run2.step(want_f=False)
    fo, _ = run2.step(want_f=True, lo=lo, wn=wn)
    fg = db.f.double().cpu().numpy()
    iz = (np.arange(wn[2]) + lo[2]) % box.n[2]
    iy = (np.arange(wn[1]) + lo[1]) % box.n[1]
    ix = (np.arange(wn[0]) + lo[0]) % box.n[0]
    fw = fg[:, iz][:, :, iy][:, :, :, ix]
    err, extra, lost = forcing_errors(fw, fo)
    assert extra == 0 and lost == 0, ("window node set", extra, lost)
    return ev, ex, rel_l2(fw, fo), err


# ------------------------------------------------ fluid-step helpers ----

def grid(n, L):
    ax = [np.arange(m) * (Li / m) for m, Li in zip(n, L)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x, y, z


def periodic_gaussian(n, L, xp, s):
    """Normalised Gaussian of variance s^2 at xp, summed over the 27 nearest
    periodic images (the next shell is below exp(-L^2/(8 s^2)) ~ 1e-60 here)."""
    x, y, z = grid(n, L)
    out = np.zeros_like(x)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                r2 = ((x - xp[0] + a * L[0]) ** 2 + (y - xp[1] + b * L[1]) ** 2
                      + (z - xp[2] + c * L[2]) ** 2)
                out += np.exp(-r2 / (2 * s * s))
    return out / (2 * math.pi * s * s) ** 1.5


def min_image(n, L, xp):
    x, y, z = grid(n, L)
    r = np.stack([x - xp[0], y - xp[1], z - xp[2]])
    for i in range(3):
        r[i] -= L[i] * np.round(r[i] / L[i])
    return r


def closed_form_sum(r, D, sR, nu, dt, rho, K):
    """Sum over the last K forcing steps of the App. E disturbance of one step,
    the k-th one diffused k dt longer: sigma_k^2 = sigma_R^2 + 2 nu k dt."""
    rn = np.sqrt(np.sum(r * r, axis=0))
    m = rn > 1e-9
    out = np.zeros_like(r)
    for k in range(1, K + 1):
        ss = math.sqrt(sR * sR + 2 * nu * k * dt)
        out[:, m] += brute.green_tensor_velocity(r[:, m], D[:, None], ss, dt, rho)
    return out, m
