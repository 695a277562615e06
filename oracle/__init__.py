"""FP64 CPU oracle of the ERPP coupling step (ctypes wrapper of erpp_oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; the product package never imports
it.  It shares no code with the HIP library: inputs are plain NumPy arrays from
``workloads``.

Every entry point follows a definition of the paper (arXiv:1405.6969); the
citations are in erpp_oracle.c next to each stage.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "erpp_oracle.c")
_LIB = os.path.join(_HERE, "liberpp_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wextra", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3), ("np", C.c_int64),
                ("m_p", C.c_double), ("rho_f", C.c_double), ("nu", C.c_double),
                ("sigma", C.c_double), ("cutoff", C.c_double), ("shear", C.c_double),
                ("M", C.c_int32), ("dt", C.c_double), ("self_correction", C.c_int32),
                ("g", C.c_double * 3), ("integrator", C.c_int32), ("a_p", C.c_double),
                ("a_am", C.c_double), ("a_b", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER(Params)
        d = C.POINTER(C.c_double)
        i32 = C.POINTER(C.c_int32)
        f32 = C.POINTER(C.c_float)
        lib.oracle_bin.argtypes = [P, d, i32, i32, i32]
        lib.oracle_deposit.argtypes = [P, d, d, i32, i32, d]
        lib.oracle_normalisation.argtypes = [P, d, d]
        lib.oracle_self_disturbance.argtypes = [P, d, d, d, d]
        lib.oracle_gather.argtypes = [P, d, d, d]
        lib.oracle_step.argtypes = [P, C.c_int64, d, d, d, f32, d, d, i32, i32, d, d, d, i32,
                                    d, i32]
        lib.oracle_self_gradient.argtypes = [P, d, d, d, d]
        lib.oracle_grid_gradient.argtypes = [P, d, d, d]
        lib.oracle_self_laplacian.argtypes = [P, d, d, d, d]
        lib.oracle_grid_laplacian.argtypes = [P, d, d, d]
        for fn in (lib.oracle_bin, lib.oracle_deposit, lib.oracle_normalisation,
                   lib.oracle_self_disturbance, lib.oracle_gather, lib.oracle_step,
                   lib.oracle_self_laplacian, lib.oracle_grid_laplacian,
                   lib.oracle_self_gradient, lib.oracle_grid_gradient):
            fn.restype = None
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(n, L, np_, m_p, rho_f, nu, sigma, cutoff=3.0, shear=0.0, M=1,
                dt=1e-3, self_correction=1, g=(0.0, 0.0, 0.0), integrator=0,
                a_p=0.0, a_am=0.0, a_b=0.0) -> Params:
    P = Params()
    P.n = (C.c_int32 * 3)(*[int(v) for v in n])
    P.L = (C.c_double * 3)(*[float(v) for v in L])
    P.np = int(np_)
    P.m_p, P.rho_f, P.nu, P.sigma = float(m_p), float(rho_f), float(nu), float(sigma)
    P.cutoff, P.shear = float(cutoff), float(shear)
    P.M, P.dt, P.self_correction = int(M), float(dt), int(self_correction)
    P.g = (C.c_double * 3)(*[float(a) for a in g])
    P.integrator = int(integrator)
    P.a_p = float(a_p)
    P.a_am = float(a_am)
    P.a_b = float(a_b)
    if (P.a_am > 0.0 or P.a_b > 0.0) and (P.integrator != 0 or P.shear != 0.0):
        raise ValueError("the added-mass and Basset terms are defined for the explicit Euler "
                         "integrator in a box without mean shear")
    for d in range(3):
        dxd = P.L[d] / P.n[d]
        R = int(np.ceil(P.cutoff * P.sigma / dxd))
        if P.n[d] < 2 * R + 2:
            raise ValueError(f"grid too small: N[{d}]={P.n[d]} < 2*{R}+2")
    rc = P.cutoff * P.sigma
    if rc * rc < 0.25 * sum((P.L[d] / P.n[d]) ** 2 for d in range(3)):
        raise ValueError("cutoff * sigma below half the cell diagonal: a sphere can miss "
                         "every node and the normalisation vanishes")
    if P.M < 1:
        raise ValueError("M must be >= 1")
    return P


def params_for_box(box, M, dt, self_correction=1, np_=None) -> Params:
    p = box.params()
    return make_params(p["n"], p["L"], p["np"] if np_ is None else np_, p["m_p"],
                       p["rho_f"], p["nu"], p["sigma"], p["cutoff"], p["shear"], M, dt,
                       self_correction)


def _with_np(P: Params, np_: int) -> Params:
    Q = Params()
    C.pointer(Q)[0] = P
    Q.np = int(np_)
    return Q


def bin_cells(P: Params, x):
    x = _f64(x)
    np_ = x.shape[1]
    Q = _with_np(P, np_)
    nc = P.n[0] * P.n[1] * P.n[2]
    key = np.empty(np_, np.int32)
    start = np.empty(nc + 1, np.int32)
    perm = np.empty(np_, np.int32)
    _load().oracle_bin(C.byref(Q), _ptr(x, C.c_double), _ptr(key, C.c_int32),
                       _ptr(start, C.c_int32), _ptr(perm, C.c_int32))
    return key, start, perm


def _window(P, lo, wn):
    if lo is None:
        lo = (0, 0, 0)
    if wn is None:
        wn = tuple(P.n)
    return np.asarray(lo, np.int32), np.asarray(wn, np.int32)


def deposit(P: Params, X, D, lo=None, wn=None):
    """Forcing (acceleration) [3][wn_z][wn_y][wn_x] from delayed (X, D)."""
    X, D = _f64(X), _f64(D)
    Q = _with_np(P, X.shape[1])
    lo, wn = _window(P, lo, wn)
    f = np.empty((3, wn[2], wn[1], wn[0]))
    _load().oracle_deposit(C.byref(Q), _ptr(X, C.c_double), _ptr(D, C.c_double),
                           _ptr(lo, C.c_int32), _ptr(wn, C.c_int32), _ptr(f, C.c_double))
    return f


def normalisation(P: Params, X):
    X = _f64(X)
    Q = _with_np(P, X.shape[1])
    Z = np.empty(X.shape[1])
    _load().oracle_normalisation(C.byref(Q), _ptr(X, C.c_double), _ptr(Z, C.c_double))
    return Z


def self_disturbance(P: Params, x, Xp, Dp):
    x, Xp, Dp = _f64(x), _f64(Xp), _f64(Dp)
    Q = _with_np(P, x.shape[1])
    vs = np.empty_like(x)
    _load().oracle_self_disturbance(C.byref(Q), _ptr(x, C.c_double), _ptr(Xp, C.c_double),
                                    _ptr(Dp, C.c_double), _ptr(vs, C.c_double))
    return vs


def self_laplacian(P: Params, x, Xp, Dp):
    """Laplacian of the closed-form self-disturbance (Faxen term, self part)."""
    x, Xp, Dp = _f64(x), _f64(Xp), _f64(Dp)
    Q = _with_np(P, x.shape[1])
    ls = np.empty_like(x)
    _load().oracle_self_laplacian(C.byref(Q), _ptr(x, C.c_double), _ptr(Xp, C.c_double),
                                  _ptr(Dp, C.c_double), _ptr(ls, C.c_double))
    return ls


def self_gradient(P: Params, x, Xp, Dp):
    """Gradient of the closed-form self-disturbance, [3 (component)][3 (direction)][np]."""
    x, Xp, Dp = _f64(x), _f64(Xp), _f64(Dp)
    Q = _with_np(P, x.shape[1])
    gs = np.empty((3, 3, x.shape[1]))
    _load().oracle_self_gradient(C.byref(Q), _ptr(x, C.c_double), _ptr(Xp, C.c_double),
                                 _ptr(Dp, C.c_double), _ptr(gs, C.c_double))
    return gs


def grid_gradient(P: Params, u, x):
    """Trilinear interpolation of the central-difference nodal gradient of u (plus the
    mean shear), [3 (component)][3 (direction)][np]."""
    u, x = _f64(u), _f64(x)
    Q = _with_np(P, x.shape[1])
    gu = np.empty((3, 3, x.shape[1]))
    _load().oracle_grid_gradient(C.byref(Q), _ptr(u, C.c_double), _ptr(x, C.c_double),
                                 _ptr(gu, C.c_double))
    return gu


def grid_laplacian(P: Params, u, x):
    """Trilinear interpolation of the 7-point nodal Laplacian of u at x."""
    u, x = _f64(u), _f64(x)
    Q = _with_np(P, x.shape[1])
    lu = np.empty_like(x)
    _load().oracle_grid_laplacian(C.byref(Q), _ptr(u, C.c_double), _ptr(x, C.c_double),
                                  _ptr(lu, C.c_double))
    return lu


def gather(P: Params, u, x):
    u, x = _f64(u), _f64(x)
    Q = _with_np(P, x.shape[1])
    up = np.empty_like(x)
    _load().oracle_gather(C.byref(Q), _ptr(u, C.c_double), _ptr(x, C.c_double),
                          _ptr(up, C.c_double))
    return up


class Run:
    """Multi-step oracle state of one box: x, v, the (M+1)-level history ring."""

    def __init__(self, P: Params, u, x, v, tau):
        self.P = P
        self.u = _f64(u)
        self.x = _f64(x).copy()
        self.v = _f64(v).copy()
        self.tau = np.ascontiguousarray(tau, dtype=np.float32)
        np_ = self.x.shape[1]
        self.P = _with_np(P, np_)
        self.ring_x = np.zeros((P.M + 1, 3, np_))
        self.ring_d = np.zeros((P.M + 1, 3, np_))
        # added-mass history: u~ and u~ + (a^2/10) lap u~ of the previous step
        self.am_hist = np.zeros((6, np_))
        self.am_valid = np.zeros(1, np.int32)
        # Basset history: u~ + (a_b^2/6) lap u~ - v of the previous step
        self.bs_hist = np.zeros((3, np_))
        self.bs_valid = np.zeros(1, np.int32)
        self.n = 0

    def step(self, want_f=True, lo=None, wn=None):
        """Advance one step; returns (f or None, D^n)."""
        P = self.P
        lo_a, wn_a = _window(P, lo, wn)
        f = np.empty((3, wn_a[2], wn_a[1], wn_a[0])) if want_f else None
        D = np.empty_like(self.x)
        fp = _ptr(f, C.c_double) if want_f else C.POINTER(C.c_double)()
        _load().oracle_step(C.byref(P), C.c_int64(self.n), _ptr(self.u, C.c_double),
                            _ptr(self.x, C.c_double), _ptr(self.v, C.c_double),
                            _ptr(self.tau, C.c_float), _ptr(self.ring_x, C.c_double),
                            _ptr(self.ring_d, C.c_double), _ptr(lo_a, C.c_int32),
                            _ptr(wn_a, C.c_int32), fp, _ptr(D, C.c_double),
                            _ptr(self.am_hist, C.c_double), _ptr(self.am_valid, C.c_int32),
                            _ptr(self.bs_hist, C.c_double), _ptr(self.bs_valid, C.c_int32))
        self.n += 1
        return f, D
