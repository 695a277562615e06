"""MI355X (gfx950) ERPP particle/fluid momentum-coupling step.

Thin Python binding of ``liberpp.so`` (C ABI in ``include/erpp.h``): argument
marshalling only.  Every stage of the step runs in the library's HIP kernels;
PyTorch provides device memory and the current stream.  If the library is not
built this module raises on first use -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liberpp.so")

ERPP_OK, ERPP_EINVAL, ERPP_ENOMEM, ERPP_EHIP, ERPP_EGEOM, ERPP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
F64_PLAIN, F32_FAST = 0, 1
EULER, EXPONENTIAL, HEUN = 0, 1, 2

EXPORTS = ["erpp_plan_create", "erpp_plan_set_tile", "erpp_plan_get_tile", "erpp_plan_tune",
           "erpp_plan_bins", "erpp_bin", "erpp_scatter", "erpp_gather", "erpp_step", "erpp_run",
           "erpp_stage_times", "erpp_plan_destroy", "erpp_status_string", "erpp_last_error",
           "erpp_fluid_create", "erpp_fluid_step", "erpp_fluid_destroy", "erpp_run_coupled",
           "erpp_plan_set_body_force", "erpp_plan_set_integrator", "erpp_plan_set_faxen",
           "erpp_plan_set_added_mass", "erpp_bin_static", "erpp_plan_set_basset",
           "erpp_plan_set_rows_per_item", "erpp_plan_get_rows_per_item"]


class ErppError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class CBox(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3), ("np", C.c_int64),
                ("x", C.c_void_p), ("v", C.c_void_p), ("ring_x", C.c_void_p),
                ("ring_d", C.c_void_p), ("tau", C.c_void_p), ("u", C.c_void_p),
                ("f", C.c_void_p), ("m_p", C.c_double), ("rho_f", C.c_double),
                ("nu", C.c_double), ("sigma", C.c_double), ("cutoff", C.c_double),
                ("shear", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load liberpp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP extension {path} is missing: build it with "
                          f"`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(path)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.erpp_plan_create.argtypes = [C.POINTER(vp), C.POINTER(CBox), i32, i32, d, C.c_int,
                                     i32, vp]
    lib.erpp_plan_set_tile.argtypes = [vp, C.POINTER(i32)]
    lib.erpp_plan_get_tile.argtypes = [vp, C.POINTER(i32)]
    lib.erpp_plan_tune.argtypes = [vp, C.c_char_p, vp]
    lib.erpp_plan_bins.argtypes = [vp, i32, C.POINTER(i32)]
    lib.erpp_bin.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.erpp_scatter.argtypes = [vp, i64, vp]
    lib.erpp_gather.argtypes = [vp, vp, vp]
    lib.erpp_step.argtypes = [vp, i64, vp]
    lib.erpp_run.argtypes = [vp, i64, i64, i32, vp]
    lib.erpp_stage_times.argtypes = [vp, i64, i64, C.POINTER(C.c_double), vp]
    lib.erpp_plan_destroy.argtypes = [vp]
    lib.erpp_plan_destroy.restype = None
    lib.erpp_status_string.argtypes = [C.c_int]
    lib.erpp_status_string.restype = C.c_char_p
    lib.erpp_last_error.argtypes = []
    lib.erpp_last_error.restype = C.c_char_p
    lib.erpp_fluid_create.argtypes = [C.POINTER(vp), C.POINTER(i32), C.POINTER(d), d, d, C.c_int,
                                      vp]
    lib.erpp_fluid_step.argtypes = [vp, vp, vp, vp]
    lib.erpp_fluid_destroy.argtypes = [vp]
    lib.erpp_fluid_destroy.restype = None
    lib.erpp_run_coupled.argtypes = [vp, C.POINTER(vp), i64, i64, i32, vp]
    lib.erpp_plan_set_body_force.argtypes = [vp, i32, C.POINTER(d)]
    lib.erpp_plan_set_integrator.argtypes = [vp, C.c_int]
    lib.erpp_plan_set_faxen.argtypes = [vp, i32, d]
    lib.erpp_plan_set_added_mass.argtypes = [vp, i32, d, vp]
    lib.erpp_bin_static.argtypes = [C.POINTER(i32), C.POINTER(d), i64, vp, vp, vp, vp, vp]
    lib.erpp_plan_set_basset.argtypes = [vp, i32, d, vp]
    lib.erpp_plan_set_rows_per_item.argtypes = [vp, i32]
    lib.erpp_plan_get_rows_per_item.argtypes = [vp, C.POINTER(i32)]
    for name in ["erpp_plan_create", "erpp_plan_set_tile", "erpp_plan_get_tile",
                 "erpp_plan_tune", "erpp_plan_bins", "erpp_bin", "erpp_scatter", "erpp_gather",
                 "erpp_step", "erpp_run", "erpp_stage_times", "erpp_fluid_create",
                 "erpp_fluid_step", "erpp_run_coupled", "erpp_plan_set_body_force",
                 "erpp_plan_set_integrator", "erpp_plan_set_faxen", "erpp_plan_set_added_mass",
                 "erpp_bin_static", "erpp_plan_set_basset", "erpp_plan_set_rows_per_item",
                 "erpp_plan_get_rows_per_item"]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != ERPP_OK:
        lib = load()
        raise ErppError(status, where, lib.erpp_last_error().decode())


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


@dataclass
class DeviceBox:
    """Device arrays and parameters of one box (torch tensors on the GPU)."""
    n: Sequence[int]
    L: Sequence[float]
    x: "object"            # float64 [3][np]
    v: "object"            # float64 [3][np]
    ring_x: "object"       # float64 [M+1][3][np]
    ring_d: "object"       # float32 or float64 [M+1][3][np]
    tau: "object"          # float32 [np]
    u: "object"            # float32 or float64 [3][Nz][Ny][Nx]
    f: "object"            # float32 or float64 [3][Nz][Ny][Nx]
    m_p: float
    rho_f: float
    nu: float
    sigma: float
    cutoff: float = 3.0
    shear: float = 0.0

    @property
    def np_(self) -> int:
        return int(self.x.shape[1])

    def cbox(self) -> CBox:
        b = CBox()
        b.n = (C.c_int32 * 3)(*[int(v) for v in self.n])
        b.L = (C.c_double * 3)(*[float(v) for v in self.L])
        b.np = self.np_
        b.x, b.v, b.ring_x, b.ring_d = _ptr(self.x), _ptr(self.v), _ptr(self.ring_x), _ptr(self.ring_d)
        b.tau, b.u, b.f = _ptr(self.tau), _ptr(self.u), _ptr(self.f)
        b.m_p, b.rho_f, b.nu, b.sigma = self.m_p, self.rho_f, self.nu, self.sigma
        b.cutoff, b.shear = self.cutoff, self.shear
        return b


def device_box(n, L, x, v, tau, u, M, m_p, rho_f, nu, sigma, cutoff=3.0, shear=0.0,
               precision=F32_FAST, device="cuda") -> DeviceBox:
    """Upload host arrays (NumPy) of one box and allocate its ring and forcing."""
    import torch
    fdt = torch.float32 if precision == F32_FAST else torch.float64
    np_ = x.shape[1]
    xt = torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
    vt = torch.as_tensor(v, dtype=torch.float64).to(device).contiguous()
    taut = torch.as_tensor(tau, dtype=torch.float32).to(device).contiguous()
    ut = torch.as_tensor(u).to(device=device, dtype=fdt).contiguous()
    ring_x = torch.zeros((M + 1, 3, np_), dtype=torch.float64, device=device)
    ring_d = torch.zeros((M + 1, 3, np_), dtype=fdt, device=device)
    f = torch.empty_like(ut)
    return DeviceBox(n=tuple(int(a) for a in n), L=tuple(float(a) for a in L), x=xt, v=vt,
                     ring_x=ring_x, ring_d=ring_d, tau=taut, u=ut, f=f, m_p=float(m_p),
                     rho_f=float(rho_f), nu=float(nu), sigma=float(sigma),
                     cutoff=float(cutoff), shear=float(shear))


def bin_static(n, L, pos, stream=None):
    """erpp_bin_static: exact cell binning of the [3][np] FP64 device positions
    `pos` of one box of n cells and lengths L, with no plan and no device
    allocation inside the library.  Returns (key, perm, bin_start) (int32 device
    tensors allocated here by the caller side)."""
    import torch
    lib = load()
    np_ = pos.shape[1]
    dev = pos.device
    ncell = int(n[0]) * int(n[1]) * int(n[2])
    key = torch.empty(np_, dtype=torch.int32, device=dev)
    perm = torch.empty(np_, dtype=torch.int32, device=dev)
    start = torch.empty(ncell + 1, dtype=torch.int32, device=dev)
    nn = (C.c_int32 * 3)(*[int(a) for a in n])
    LL = (C.c_double * 3)(*[float(a) for a in L])
    _check(lib.erpp_bin_static(nn, LL, int(np_), C.c_void_p(pos.data_ptr()),
                               C.c_void_p(key.data_ptr()), C.c_void_p(perm.data_ptr()),
                               C.c_void_p(start.data_ptr()), _stream(stream)),
           "erpp_bin_static")
    return key, perm, start


class Plan:
    """An erpp_plan over a list of DeviceBox (kept alive by the plan)."""

    def __init__(self, boxes: List[DeviceBox], M: int, dt: float, precision: int = F32_FAST,
                 self_correction: int = 1, stream=None):
        self.lib = load()
        self.boxes = list(boxes)
        self.M, self.dt, self.precision = int(M), float(dt), int(precision)
        arr = (CBox * len(self.boxes))(*[b.cbox() for b in self.boxes])
        self._arr = arr
        h = C.c_void_p()
        _check(self.lib.erpp_plan_create(C.byref(h), arr, len(self.boxes), self.M, self.dt,
                                         self.precision, int(self_correction), _stream(stream)),
               "erpp_plan_create")
        self.h = h

    # -- lifecycle
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.erpp_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- configuration
    def set_tile(self, tile):
        t = (C.c_int32 * 3)(*tile)
        _check(self.lib.erpp_plan_set_tile(self.h, t), "erpp_plan_set_tile")

    def set_body_force(self, ibox: int, g):
        """Body acceleration (m_p - m_f) g / m_p of the particles of box ibox."""
        _check(self.lib.erpp_plan_set_body_force(self.h, int(ibox),
                                                 (C.c_double * 3)(*[float(a) for a in g])),
               "erpp_plan_set_body_force")

    def set_faxen(self, ibox: int, a_p: float):
        """Particle radius of the Faxen term (a_p^2/6) lap u~ in the drag of box ibox."""
        _check(self.lib.erpp_plan_set_faxen(self.h, int(ibox), float(a_p)), "erpp_plan_set_faxen")

    def set_added_mass(self, ibox: int, a: float, hist=None):
        """Added-mass terms of box ibox for particles of radius a (0 turns them off).
        hist: FP64 device tensor [6, np] (allocated here when None), kept by the
        plan while the terms are on; it holds u~ and u~ + (a^2/10) lap u~ of the
        last step."""
        import torch
        if a > 0.0 and hist is None:
            np_ = self.boxes[ibox].x.shape[1]
            hist = torch.zeros((6, np_), dtype=torch.float64, device=self.boxes[ibox].x.device)
        if hist is not None and (hist.dtype != torch.float64 or not hist.is_contiguous()):
            raise ValueError("hist must be a contiguous float64 tensor")
        _check(self.lib.erpp_plan_set_added_mass(self.h, int(ibox), float(a), _ptr(hist)),
               "erpp_plan_set_added_mass")
        self._am_hist = getattr(self, "_am_hist", {})
        self._am_hist[int(ibox)] = hist if a > 0.0 else None

    def set_basset(self, ibox: int, a: float, hist=None):
        """Basset term of box ibox for particles of radius a (0 turns it off), its
        memory integral over the last step.  hist: FP64 device tensor [3, np]
        (allocated here when None), kept by the plan while the term is on; it
        holds u~ + (a^2/6) lap u~ - v of the last step."""
        import torch
        if a > 0.0 and hist is None:
            np_ = self.boxes[ibox].x.shape[1]
            hist = torch.zeros((3, np_), dtype=torch.float64, device=self.boxes[ibox].x.device)
        if hist is not None and (hist.dtype != torch.float64 or not hist.is_contiguous()):
            raise ValueError("hist must be a contiguous float64 tensor")
        _check(self.lib.erpp_plan_set_basset(self.h, int(ibox), float(a), _ptr(hist)),
               "erpp_plan_set_basset")
        self._bs_hist = getattr(self, "_bs_hist", {})
        self._bs_hist[int(ibox)] = hist if a > 0.0 else None
        return hist

    def set_integrator(self, kind: int):
        """EULER (explicit Euler), EXPONENTIAL (exact linear drag over the step) or
        HEUN (two stages, self term removed at each)."""
        _check(self.lib.erpp_plan_set_integrator(self.h, int(kind)), "erpp_plan_set_integrator")

    def get_tile(self):
        t = (C.c_int32 * 3)()
        _check(self.lib.erpp_plan_get_tile(self.h, t), "erpp_plan_get_tile")
        return tuple(t)

    def set_rows_per_item(self, rows: int):
        _check(self.lib.erpp_plan_set_rows_per_item(self.h, int(rows)),
               "erpp_plan_set_rows_per_item")

    def get_rows_per_item(self) -> int:
        r = C.c_int32()
        _check(self.lib.erpp_plan_get_rows_per_item(self.h, C.byref(r)),
               "erpp_plan_get_rows_per_item")
        return int(r.value)

    def tune(self, cache_path: Optional[str] = None, stream=None):
        cp = cache_path.encode() if cache_path else None
        _check(self.lib.erpp_plan_tune(self.h, cp, _stream(stream)), "erpp_plan_tune")

    def nbins(self, ibox: int) -> int:
        n = C.c_int32()
        _check(self.lib.erpp_plan_bins(self.h, ibox, C.byref(n)), "erpp_plan_bins")
        return n.value

    # -- stages
    def bin(self, ibox: int, pos, stream=None):
        import torch
        np_ = pos.shape[1]
        dev = pos.device
        key = torch.empty(np_, dtype=torch.int32, device=dev)
        perm = torch.empty(np_, dtype=torch.int32, device=dev)
        start = torch.empty(self.nbins(ibox) + 1, dtype=torch.int32, device=dev)
        _check(self.lib.erpp_bin(self.h, ibox, C.c_void_p(pos.data_ptr()), C.c_void_p(key.data_ptr()),
                                 C.c_void_p(perm.data_ptr()), C.c_void_p(start.data_ptr()),
                                 _stream(stream)), "erpp_bin")
        return key, perm, start

    def scatter(self, step: int, stream=None):
        _check(self.lib.erpp_scatter(self.h, int(step), _stream(stream)), "erpp_scatter")

    def gather(self, stream=None):
        import torch
        tot = sum(b.np_ for b in self.boxes)
        dev = self.boxes[0].x.device
        out = torch.empty(3 * max(tot, 1), dtype=torch.float64, device=dev)
        _check(self.lib.erpp_gather(self.h, C.c_void_p(out.data_ptr()), _stream(stream)),
               "erpp_gather")
        res, off = [], 0
        for b in self.boxes:
            res.append(out[off:off + 3 * b.np_].view(3, b.np_))
            off += 3 * b.np_
        return res

    def step(self, step: int, stream=None):
        _check(self.lib.erpp_step(self.h, int(step), _stream(stream)), "erpp_step")

    def stage_times(self, step0: int, nsteps: int, stream=None):
        """Average per-stage milliseconds over nsteps real steps (see erpp.h)."""
        ms = (C.c_double * 5)()
        _check(self.lib.erpp_stage_times(self.h, int(step0), int(nsteps), ms, _stream(stream)),
               "erpp_stage_times")
        return list(ms)

    def run(self, step0: int, nsteps: int, graph: bool = True, stream=None):
        _check(self.lib.erpp_run(self.h, int(step0), int(nsteps), int(bool(graph)),
                                 _stream(stream)), "erpp_run")

    def run_coupled(self, fluids, step0: int, nsteps: int, graph: bool = True, stream=None):
        """Two-way coupled steps: coupling step, then fluids[b] advances box b's u."""
        arr = (C.c_void_p * len(fluids))(*[f.h.value for f in fluids])
        _check(self.lib.erpp_run_coupled(self.h, arr, int(step0), int(nsteps), int(bool(graph)),
                                         _stream(stream)), "erpp_run_coupled")


class Fluid:
    """An erpp_fluid: the App. E unsteady-Stokes step u <- P exp(nu dt lap)(u + dt f)
    on one periodic grid (see erpp.h)."""

    def __init__(self, n, L, nu: float, dt: float, precision: int = F32_FAST, stream=None):
        self.lib = load()
        self.n = tuple(int(a) for a in n)
        self.L = tuple(float(a) for a in L)
        self.nu, self.dt, self.precision = float(nu), float(dt), int(precision)
        h = C.c_void_p()
        _check(self.lib.erpp_fluid_create(C.byref(h), (C.c_int32 * 3)(*self.n),
                                          (C.c_double * 3)(*self.L), self.nu, self.dt,
                                          self.precision, _stream(stream)), "erpp_fluid_create")
        self.h = h

    def step(self, u, f, stream=None):
        """Advance u ([3][Nz][Ny][Nx] device tensor, updated in place) by one step
        with forcing f (same shape and dtype)."""
        import torch
        want = torch.float32 if self.precision == F32_FAST else torch.float64
        shape = (3, self.n[2], self.n[1], self.n[0])
        for name, t in (("u", u), ("f", f)):
            if t.dtype != want or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {want} tensor of shape {shape}")
        _check(self.lib.erpp_fluid_step(self.h, C.c_void_p(u.data_ptr()),
                                        C.c_void_p(f.data_ptr()), _stream(stream)),
               "erpp_fluid_step")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.erpp_fluid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
