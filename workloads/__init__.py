"""Seeded synthetic inputs for the ERPP particle-to-fluid coupling step.

This module only *draws data*: carrier fields on the grid, particle positions,
initial velocities, Stokes times and the physical parameters of each workload.
It contains none of the coupling step's arithmetic (no binning, no Gaussian
kernel, no interpolation, no drag) so that the FP64 oracle and the HIP path can
both consume its arrays without sharing any of the computation they are checked
on.

Workloads (sizes and parameters of the paper's validation and shear-flow runs,
Sec. 3 and Sec. 4, restated as five synthetic configurations):

1. 32^3, L=2pi, frozen Taylor-Green carrier, 1000 uniform particles.
2. 128^3, L=2pi, divergence-free random-phase k^-5/3 carrier (2<=|k|<=40,
   urms=1), 1e5 uniform particles.
3. 256x128x128, 4pi x 2pi x 2pi, mean shear S=1 plus a k^-5/3 fluctuation
   (urms=0.5), 4e5 particles: 70% in 2000 Gaussian blobs of radius 4 dx, 30%
   uniform; three equal Stokes-time populations 0.02 / 0.1 / 0.5.
   (Shaped after the homogeneous-shear run of Sec. 4: 4pi x 2pi x 2pi box,
   ~1e6 particles, mean shear along y.)
4. 512^3, L=2pi, k^-5/3 carrier, 4e6 clustered particles, sigma = 2 dx, M=12.
5. Ensemble of 64 independent boxes with N in {32,64,96,128}^3 and particle
   counts log-uniform in [1e3, 2e5].

Seeds: numpy ``Generator(PCG64(14056969 + 1000*config + box))``.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 14056969


@dataclass
class BoxSpec:
    """Recipe of one periodic box (no arrays)."""

    n: Tuple[int, int, int]                 # nodes (Nx, Ny, Nz), x fastest in memory
    L: Tuple[float, float, float]           # box lengths
    np_: int                                # number of particles
    carrier: str = "k53"                    # "taylor_green" | "k53"
    urms: float = 1.0                       # per-component rms of the k^-5/3 field
    kmin: float = 2.0
    kmax: float = 40.0
    shear: float = 0.0                      # mean shear rate S (U_x = S (y - Ly/2))
    placement: str = "uniform"              # "uniform" | "clustered"
    cluster_frac: float = 0.7
    n_blobs: int = 2000
    blob_radius_dx: float = 4.0
    tau: Tuple[float, ...] = (0.1,)         # Stokes-time populations (equal shares)
    sigma_dx: float = 1.5                   # Gaussian width in grid spacings
    cutoff: float = 3.0                     # stencil radius in units of sigma
    nu: float = 0.005
    rho_f: float = 1.0
    mass_loading: float = 0.1               # Phi = N_p m_p / (rho_f V)
    slip_noise: float = 0.1                 # std of the initial slip velocity
    seed: int = SEED_BASE


@dataclass
class Workload:
    name: str
    boxes: List[BoxSpec]
    M: int
    dt: float
    steps: int
    self_correction: int = 1
    precision: str = "f32"                  # arithmetic of the GPU path under test


@dataclass
class Box:
    """Arrays of one box, ready to upload.  Layouts:

    u   : float64 [3][Nz][Ny][Nx]  carrier velocity fluctuation on the nodes x_i = i*dx
    x,v : float64 [3][np]          positions in [0, L) and velocities (SoA)
    tau : float32 [np]             Stokes times
    """

    spec: BoxSpec
    u: np.ndarray
    x: np.ndarray
    v: np.ndarray
    tau: np.ndarray
    m_p: float

    @property
    def n(self):
        return self.spec.n

    @property
    def L(self):
        return self.spec.L

    @property
    def np_(self):
        return self.spec.np_

    @property
    def dx(self):
        return tuple(self.spec.L[d] / self.spec.n[d] for d in range(3))

    @property
    def sigma(self):
        return self.spec.sigma_dx * self.dx[0]

    def params(self) -> dict:
        s = self.spec
        return dict(n=tuple(s.n), L=tuple(s.L), np=s.np_, m_p=self.m_p,
                    rho_f=s.rho_f, nu=s.nu, sigma=self.sigma, cutoff=s.cutoff,
                    shear=s.shear)


# --------------------------------------------------------------------------
# carriers
# --------------------------------------------------------------------------

def taylor_green(n, L):
    """u = (sin x cos y cos z, -cos x sin y cos z, 0) sampled on x_i = i L/N."""
    Nx, Ny, Nz = n
    x = np.arange(Nx) * (L[0] / Nx)
    y = np.arange(Ny) * (L[1] / Ny)
    z = np.arange(Nz) * (L[2] / Nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u = np.empty((3, Nz, Ny, Nx))
    u[0] = np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    return u


def taylor_green_at(x, L):
    return np.stack([np.sin(x[0]) * np.cos(x[1]) * np.cos(x[2]),
                     -np.cos(x[0]) * np.sin(x[1]) * np.cos(x[2]),
                     np.zeros_like(x[0])])


def k53_field(n, L, urms, kmin, kmax, rng):
    """Real, divergence-free random-phase field with shell spectrum E(k) ~ k^-5/3.

    Modes k = 2 pi m / L with kmin <= |k| <= kmax; amplitude |k|^(-11/6);
    uniform random phase; random direction in the plane normal to k.  The
    spectrum is Hermitian by construction (the m_x = 0 plane is symmetrised
    explicitly), the field is the inverse real FFT, rescaled so that the
    per-component rms equals urms (<|u|^2> = 3 urms^2).
    """
    Nx, Ny, Nz = n
    kmax = min(kmax, min(n) / 2 - 1)
    mxmax = min(int(math.floor(kmax * L[0] / (2 * math.pi))), Nx // 2 - 1)
    mymax = min(int(math.floor(kmax * L[1] / (2 * math.pi))), Ny // 2 - 1)
    mzmax = min(int(math.floor(kmax * L[2] / (2 * math.pi))), Nz // 2 - 1)
    mx = np.arange(0, mxmax + 1)
    my = np.arange(-mymax, mymax + 1)
    mz = np.arange(-mzmax, mzmax + 1)
    MZ, MY, MX = np.meshgrid(mz, my, mx, indexing="ij")
    KX = 2 * np.pi * MX / L[0]
    KY = 2 * np.pi * MY / L[1]
    KZ = 2 * np.pi * MZ / L[2]
    K = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    sel = (K >= kmin) & (K <= kmax)
    mx_s, my_s, mz_s = MX[sel], MY[sel], MZ[sel]
    k = np.stack([KX[sel], KY[sel], KZ[sel]], axis=1)
    kn = K[sel]
    nm = kn.size
    theta = rng.uniform(0.0, 2 * np.pi, nm)
    psi = rng.uniform(0.0, 2 * np.pi, nm)
    khat = k / kn[:, None]
    a = np.zeros_like(khat)
    a[:, 0] = 1.0
    par = np.abs(khat[:, 0]) > 0.9
    a[par] = [0.0, 1.0, 0.0]
    e1 = np.cross(a, khat)
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(khat, e1)
    e = np.cos(psi)[:, None] * e1 + np.sin(psi)[:, None] * e2
    amp = kn ** (-11.0 / 6.0) * np.exp(1j * theta)
    spec = np.zeros((3, Nz, Ny, Nx // 2 + 1), dtype=np.complex128)
    iz = np.mod(mz_s, Nz)
    iy = np.mod(my_s, Ny)
    for c in range(3):
        spec[c, iz, iy, mx_s] = amp * e[:, c]
    # Hermitian symmetry inside the m_x = 0 plane
    p0 = spec[:, :, :, 0]
    mirror = np.conj(p0[:, (-np.arange(Nz)) % Nz][:, :, (-np.arange(Ny)) % Ny])
    spec[:, :, :, 0] = 0.5 * (p0 + mirror)
    u = np.empty((3, Nz, Ny, Nx))
    for c in range(3):
        u[c] = np.fft.irfftn(spec[c], s=(Nz, Ny, Nx), axes=(0, 1, 2))
    del spec
    scale = urms * math.sqrt(3.0) / math.sqrt(float(np.mean(np.sum(u * u, axis=0))))
    u *= scale
    return u


# --------------------------------------------------------------------------
# particles
# --------------------------------------------------------------------------

def _wrap_into(x, L):
    x = np.mod(x, L)
    x[x >= L] = 0.0
    return x


def particle_positions(spec: BoxSpec, rng) -> np.ndarray:
    n, L, npart = spec.n, spec.L, spec.np_
    if spec.placement == "uniform":
        x = np.stack([rng.uniform(0.0, L[d], npart) for d in range(3)])
    elif spec.placement == "clustered":
        dx = L[0] / n[0]
        ncl = int(round(spec.cluster_frac * npart))
        nun = npart - ncl
        centres = np.stack([rng.uniform(0.0, L[d], spec.n_blobs) for d in range(3)])
        pick = rng.integers(0, spec.n_blobs, ncl)
        off = rng.normal(0.0, spec.blob_radius_dx * dx, (3, ncl))
        xc = centres[:, pick] + off
        xu = np.stack([rng.uniform(0.0, L[d], nun) for d in range(3)])
        x = np.concatenate([xc, xu], axis=1)
        x = x[:, rng.permutation(npart)]
    else:
        raise ValueError(spec.placement)
    for d in range(3):
        x[d] = _wrap_into(x[d], L[d])
    return np.ascontiguousarray(x)


def nearest_node_sample(u, x, L):
    """Carrier value at the node nearest to each particle (input drawing only)."""
    Nz, Ny, Nx = u.shape[1:]
    i = np.mod(np.rint(x[0] / (L[0] / Nx)).astype(np.int64), Nx)
    j = np.mod(np.rint(x[1] / (L[1] / Ny)).astype(np.int64), Ny)
    k = np.mod(np.rint(x[2] / (L[2] / Nz)).astype(np.int64), Nz)
    return np.stack([u[c, k, j, i] for c in range(3)])


def make_box(spec: BoxSpec) -> Box:
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    if spec.carrier == "taylor_green":
        u = taylor_green(spec.n, spec.L)
    elif spec.carrier == "k53":
        u = k53_field(spec.n, spec.L, spec.urms, spec.kmin, spec.kmax, rng)
    elif spec.carrier == "zero":
        u = np.zeros((3, spec.n[2], spec.n[1], spec.n[0]))
    else:
        raise ValueError(spec.carrier)
    x = particle_positions(spec, rng)
    if spec.carrier == "taylor_green":
        ufl = taylor_green_at(x, spec.L)
    else:
        ufl = nearest_node_sample(u, x, spec.L)
    v = ufl + rng.normal(0.0, spec.slip_noise, (3, spec.np_))
    if spec.shear != 0.0:
        v[0] += spec.shear * (x[1] - 0.5 * spec.L[1])
    pops = np.asarray(spec.tau, dtype=np.float64)
    tau = pops[np.arange(spec.np_) % pops.size].astype(np.float32)
    vol = spec.L[0] * spec.L[1] * spec.L[2]
    m_p = spec.mass_loading * spec.rho_f * vol / max(spec.np_, 1)
    return Box(spec=spec, u=np.ascontiguousarray(u), x=x, v=np.ascontiguousarray(v),
               tau=tau, m_p=m_p)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

TWO_PI = 2.0 * math.pi


def _seed(cfg, box):
    return SEED_BASE + 1000 * cfg + box


def config(i: int, **overrides) -> Workload:
    """Workload i (1..5).  Keyword overrides patch the BoxSpec of every box
    (e.g. ``np_=2000``) or the run parameters (``steps``, ``M``, ``dt``)."""
    run_keys = {"M", "dt", "steps", "self_correction", "precision", "nbox"}
    run_over = {k: v for k, v in overrides.items() if k in run_keys}
    box_over = {k: v for k, v in overrides.items() if k not in run_keys}
    if i == 1:
        b = BoxSpec(n=(32, 32, 32), L=(TWO_PI,) * 3, np_=1000, carrier="taylor_green",
                    tau=(0.05,), nu=0.01, seed=_seed(1, 0))
        w = Workload("c1_tg32_np1e3", [b], M=4, dt=1e-3, steps=10, precision="f64")
    elif i == 2:
        b = BoxSpec(n=(128, 128, 128), L=(TWO_PI,) * 3, np_=100_000, urms=1.0,
                    tau=(0.1,), nu=0.005, seed=_seed(2, 0))
        w = Workload("c2_k53_128_np1e5", [b], M=8, dt=5e-4, steps=50)
    elif i == 3:
        b = BoxSpec(n=(256, 128, 128), L=(2 * TWO_PI, TWO_PI, TWO_PI), np_=400_000,
                    urms=0.5, shear=1.0, placement="clustered", tau=(0.02, 0.1, 0.5),
                    nu=0.005, seed=_seed(3, 0))
        w = Workload("c3_shear_256x128x128_np4e5", [b], M=8, dt=2e-4, steps=116)
    elif i == 4:
        b = BoxSpec(n=(512, 512, 512), L=(TWO_PI,) * 3, np_=4_000_000, urms=1.0,
                    placement="clustered", tau=(0.02, 0.1, 0.5), sigma_dx=2.0,
                    nu=0.005, seed=_seed(4, 0))
        w = Workload("c4_k53_512_np4e6", [b], M=12, dt=5e-4, steps=46)
    elif i == 5:
        nbox = int(run_over.pop("nbox", 64))
        lay = np.random.Generator(np.random.PCG64(_seed(5, 999)))
        sizes = lay.choice(np.array([32, 64, 96, 128]), nbox)
        nps = np.exp(lay.uniform(math.log(1e3), math.log(2e5), nbox)).astype(np.int64)
        taus = lay.uniform(0.02, 0.5, nbox)
        boxes = [BoxSpec(n=(int(s),) * 3, L=(TWO_PI,) * 3, np_=int(npb), urms=1.0,
                         tau=(float(t),), nu=0.005, seed=_seed(5, b))
                 for b, (s, npb, t) in enumerate(zip(sizes, nps, taus))]
        w = Workload("c5_ensemble64", boxes, M=8, dt=5e-4, steps=116)
    elif i == 33:
        # the 256^3 variant of workload 3 (same particle mix, cubic 2pi box)
        b = BoxSpec(n=(256, 256, 256), L=(TWO_PI,) * 3, np_=400_000, urms=0.5,
                    shear=1.0, placement="clustered", tau=(0.02, 0.1, 0.5), nu=0.005,
                    seed=_seed(3, 1))
        w = Workload("c3cube_shear_256_np4e5", [b], M=8, dt=2e-4, steps=116)
    else:
        raise ValueError(f"no workload {i}")
    for k, val in run_over.items():
        setattr(w, k, val)
    if box_over:
        w.boxes = [dataclasses.replace(b, **box_over) for b in w.boxes]
    return w


def make_boxes(w: Workload) -> List[Box]:
    return [make_box(s) for s in w.boxes]


def tiny_box(seed: int, n=(12, 13, 14), np_=17, sigma_dx=1.5, shear=0.0,
             carrier="k53", L=None, tau=(0.05, 0.2), placement="uniform",
             nu=0.01) -> Box:
    """Small random box for brute-force cross-checks."""
    if L is None:
        L = tuple(1.0 * n[d] / n[0] * 2.0 for d in range(3))
        L = (2.0, 2.0 * n[1] / n[0], 2.0 * n[2] / n[0])
    spec = BoxSpec(n=tuple(n), L=tuple(L), np_=np_, carrier=carrier, urms=1.0,
                   kmin=1.0, kmax=4.0, shear=shear, placement=placement,
                   blob_radius_dx=1.5, n_blobs=3, tau=tau, sigma_dx=sigma_dx,
                   nu=nu, seed=seed)
    return make_box(spec)
