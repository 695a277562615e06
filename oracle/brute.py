"""Brute-force checkers for tiny boxes (TEST INFRASTRUCTURE ONLY).

These are *independent formulations* of the quantities the oracle computes, used
to pin the oracle itself:

* ``deposit``: loops over every grid node for every particle and measures the
  minimum-image distance node - particle directly (the oracle instead walks a
  stencil of offsets around the particle's cell);
* ``gather``: sums every node's value times the product of 1-D hat functions of
  the minimum-image separation (the oracle instead picks the 8 corners of the
  cell);
* ``green_tensor_velocity``: the self-disturbance written with the unsteady
  Stokeslet of App. B (eq. green_tensor, built from g and G = -erf/(4 pi r)),
  not with the f(eta) form of App. E that the oracle uses;
* ``*_hp``: the same App. E / App. B expressions in 60-digit decimal arithmetic
  (erf from its Maclaurin series), free of the cancellation that forces the
  oracle onto a series branch near r = 0.
"""
from __future__ import annotations

import math
from decimal import Decimal, getcontext

import numpy as np


def _min_image(d, L):
    return d - L * np.round(d / L)


def deposit(n, L, sigma, cutoff, rho_f, X, D):
    Nx, Ny, Nz = n
    dx = [L[d] / n[d] for d in range(3)]
    dV = dx[0] * dx[1] * dx[2]
    zz, yy, xx = np.meshgrid(np.arange(Nz) * dx[2], np.arange(Ny) * dx[1],
                             np.arange(Nx) * dx[0], indexing="ij")
    f = np.zeros((3, Nz, Ny, Nx))
    rc2 = (cutoff * sigma) ** 2
    for p in range(X.shape[1]):
        rx = _min_image(xx - X[0, p], L[0])
        ry = _min_image(yy - X[1, p], L[1])
        rz = _min_image(zz - X[2, p], L[2])
        r2 = rx * rx + ry * ry + rz * rz
        gam = np.where(r2 <= rc2, np.exp(-r2 / (2 * sigma * sigma)), 0.0)
        Z = dV * gam.sum()
        for c in range(3):
            f[c] += (-D[c, p] / rho_f) * gam / Z
    return f


def gather(n, L, u, x, shear=0.0):
    Nx, Ny, Nz = n
    dx = [L[d] / n[d] for d in range(3)]
    out = np.zeros((3, x.shape[1]))
    nodes = [np.arange(n[d]) * dx[d] for d in range(3)]
    for p in range(x.shape[1]):
        h = []
        for d in range(3):
            t = _min_image(nodes[d] - x[d, p], L[d]) / dx[d]
            h.append(np.maximum(0.0, 1.0 - np.abs(t)))
        w = h[2][:, None, None] * h[1][None, :, None] * h[0][None, None, :]
        for c in range(3):
            out[c, p] = np.sum(w * u[c])
        if shear != 0.0:
            yh = np.mod(x[1, p], L[1])
            out[0, p] += shear * (yh - 0.5 * L[1])
    return out


def green_tensor_velocity(r, Dp, sigma_s, dt, rho_f):
    """-dt * G_ik(r; sigma_s) D_k with App. B, eq. green_tensor (FP64)."""
    r = np.asarray(r, dtype=np.float64)
    Dp = np.asarray(Dp, dtype=np.float64)
    from scipy.special import erf
    rn = np.sqrt(np.sum(r * r, axis=0))
    s2 = sigma_s * sigma_s
    g = (2 * np.pi * s2) ** -1.5 * np.exp(-rn * rn / (2 * s2))
    G = -erf(rn / (np.sqrt(2.0) * sigma_s)) / (4 * np.pi * rn)
    A = (1 + s2 / rn ** 2) * g + G / rn ** 2
    B = (1 + 3 * s2 / rn ** 2) * g + 3 * G / rn ** 2
    Dr = np.sum(Dp * r, axis=0)
    Gd = (A * Dp - B * Dr * r / rn ** 2) / rho_f
    return -dt * Gd


# ------------------------------------------------------ high precision -------

def _erf_dec(x: Decimal) -> Decimal:
    # erf(x) = 2/sqrt(pi) sum_k (-1)^k x^(2k+1) / (k! (2k+1))
    getcontext().prec = 60
    term = x
    total = Decimal(0)
    k = 0
    x2 = x * x
    eps = Decimal(10) ** -58
    while True:
        add = term / (2 * k + 1)
        total += add
        if abs(add) < eps:
            break
        k += 1
        term = -term * x2 / k
    return 2 * total / _pi_dec().sqrt()


def _pi_dec() -> Decimal:
    getcontext().prec = 60
    return Decimal("3.14159265358979323846264338327950288419716939937510582097494459")


def green_tensor_velocity_hp(r, Dp, sigma_s, dt, rho_f):
    """App. B Green tensor velocity in 60-digit arithmetic (one particle)."""
    getcontext().prec = 60
    r = [Decimal(float(v)) for v in r]
    Dp = [Decimal(float(v)) for v in Dp]
    s = Decimal(float(sigma_s))
    s2 = s * s
    pi = _pi_dec()
    rr = sum(v * v for v in r)
    rn = rr.sqrt()
    g = (2 * pi * s2) ** Decimal(-1.5) * (-rr / (2 * s2)).exp()
    G = -_erf_dec(rn / (Decimal(2).sqrt() * s)) / (4 * pi * rn)
    A = (1 + s2 / rr) * g + G / rr
    B = (1 + 3 * s2 / rr) * g + 3 * G / rr
    Dr = sum(a * b for a, b in zip(Dp, r))
    out = []
    for c in range(3):
        Gd = (A * Dp[c] - B * Dr * r[c] / rr) / Decimal(float(rho_f))
        out.append(float(-Decimal(float(dt)) * Gd))
    return np.array(out)


def disturbance_velo_hp(r, Dp, sigma_s, dt, rho_f):
    """App. E closed form (eq. disturbance_velo, with the -dt/rho_f prefactor)
    in 60-digit arithmetic, no series (one particle, r != 0)."""
    getcontext().prec = 60
    r = [Decimal(float(v)) for v in r]
    Dp = [Decimal(float(v)) for v in Dp]
    s = Decimal(float(sigma_s))
    pi = _pi_dec()
    rr = sum(v * v for v in r)
    rn = rr.sqrt()
    eta = rn / (Decimal(2).sqrt() * s)
    e = (-eta * eta).exp()
    fe = pi.sqrt() / 2 * _erf_dec(eta) - eta * e
    F = fe / (2 * eta ** 3)
    rh = [v / rn for v in r]
    Drh = sum(a * b for a, b in zip(Dp, rh))
    pref = -Decimal(float(dt)) / Decimal(float(rho_f)) * (2 * pi * s * s) ** Decimal(-1.5)
    return np.array([float(pref * ((e - F) * Dp[c] - Drh * (e - 3 * F) * rh[c]))
                     for c in range(3)])
