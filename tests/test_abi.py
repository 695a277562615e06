"""C-ABI contract on the CPU: the library loads, exports every function the
header declares, and rejects invalid arguments with a status (validation runs
before any device call, so no GPU is needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1405_6969_amd as erpp
    if not os.path.exists(erpp.LIB_PATH):
        pytest.skip("liberpp.so not built")
    return erpp, erpp.load()


def test_header_declares_exports():
    erpp, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "erpp.h")).read()
    declared = set(re.findall(r"^\s*(?:erpp_status|void|const char \*)\s*(erpp_\w+)\s*\(", hdr,
                              re.M))
    assert declared == set(erpp.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    erpp, lib = _lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.erpp_status_string(s).startswith(b"ERPP_")


def _box(erpp, n=(32, 32, 32), L=(6.283185307179586,) * 3, np_=10, sigma=None):
    b = erpp.CBox()
    b.n = (C.c_int32 * 3)(*n)
    b.L = (C.c_double * 3)(*L)
    b.np = np_
    fake = 0x1000
    b.x = b.v = b.ring_x = b.ring_d = b.tau = b.u = b.f = fake
    b.m_p, b.rho_f, b.nu = 1e-3, 1.0, 0.01
    b.sigma = 1.5 * L[0] / n[0] if sigma is None else sigma
    b.cutoff, b.shear = 3.0, 0.0
    return b


def _create(lib, boxes, nbox=None, M=4, dt=1e-3, prec=1, s=1):
    arr = (type(boxes[0]) * len(boxes))(*boxes)
    h = C.c_void_p()
    st = lib.erpp_plan_create(C.byref(h), arr, len(boxes) if nbox is None else nbox, M, dt,
                              prec, s, None)
    return st, h


@pytest.mark.parametrize("case,expect", [
    ("nbox0", -1), ("M0", -1), ("dt0", -1), ("prec", -1), ("selfc", -1), ("np_neg", -1),
    ("null_x", -1), ("grid_small", -4), ("L0", -4), ("sigma0", -4), ("grid_huge", -5),
    ("stencil_wide", -5), ("mass0", -1), ("sigma_tiny", -4),
])
def test_invalid_arguments_return_status(case, expect):
    erpp, lib = _lib()
    b = _box(erpp)
    kw = {}
    if case == "nbox0":
        kw["nbox"] = 0
    elif case == "M0":
        kw["M"] = 0
    elif case == "dt0":
        kw["dt"] = 0.0
    elif case == "prec":
        kw["prec"] = 7
    elif case == "selfc":
        kw["s"] = 2
    elif case == "np_neg":
        b.np = -1
    elif case == "null_x":
        b.x = None
    elif case == "grid_small":
        b = _box(erpp, n=(11, 32, 32), L=(11 * 0.19634954084936207, 6.283185307179586,
                                          6.283185307179586), sigma=1.5 * 0.19634954084936207)
    elif case == "L0":
        b.L = (C.c_double * 3)(0.0, 1.0, 1.0)
    elif case == "sigma0":
        b.sigma = 0.0
    elif case == "sigma_tiny":
        b.sigma = 0.28 * 6.283185307179586 / 32     # 3 sigma < half the cell diagonal
    elif case == "grid_huge":
        b = _box(erpp, n=(4096, 32, 32), L=(4096 * 0.19634954084936207, 6.283185307179586,
                                            6.283185307179586), sigma=1.5 * 0.19634954084936207)
    elif case == "stencil_wide":
        b = _box(erpp, n=(64, 64, 64), sigma=3.0 * 6.283185307179586 / 64)
    elif case == "mass0":
        b.m_p = 0.0
    st, h = _create(lib, [b], **kw)
    assert st == expect, (case, st, lib.erpp_last_error())
    assert not h.value
    assert len(lib.erpp_last_error()) > 0


def test_null_plan_calls():
    erpp, lib = _lib()
    assert lib.erpp_step(None, 0, None) == -1
    assert lib.erpp_scatter(None, 0, None) == -1
    assert lib.erpp_gather(None, None, None) == -1
    assert lib.erpp_run(None, 0, 1, 1, None) == -1
    assert lib.erpp_plan_tune(None, None, None) == -1
    lib.erpp_plan_destroy(None)   # NULL-safe


@pytest.mark.parametrize("case,expect", [
    ("null_out", -1), ("n0", -4), ("L0", -4), ("nu_neg", -1), ("dt0", -1), ("prec", -1),
    ("n_huge", -5), ("too_many", -5),
])
def test_fluid_create_invalid_arguments(case, expect):
    erpp, lib = _lib()
    n, L, nu, dt, prec = [16, 16, 16], [1.0, 1.0, 1.0], 0.01, 1e-3, 1
    h = C.c_void_p()
    out = C.byref(h)
    if case == "null_out":
        out = None
    elif case == "n0":
        n[1] = 0
    elif case == "L0":
        L[2] = 0.0
    elif case == "nu_neg":
        nu = -1.0
    elif case == "dt0":
        dt = 0.0
    elif case == "prec":
        prec = 5
    elif case == "n_huge":
        n[0] = 5000
    elif case == "too_many":
        n = [1024, 1024, 1024]
    st = lib.erpp_fluid_create(out, (C.c_int32 * 3)(*n), (C.c_double * 3)(*L), nu, dt, prec, None)
    assert st == expect
    assert not h.value
    assert lib.erpp_last_error()


def test_fluid_step_null_arguments():
    erpp, lib = _lib()
    assert lib.erpp_fluid_step(None, None, None, None) == -1
    lib.erpp_fluid_destroy(None)


def test_setters_reject_a_null_plan():
    """Every per-plan setter validates its plan before touching the device."""
    erpp, lib = _lib()
    g = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert lib.erpp_plan_set_body_force(None, 0, g) == erpp.ERPP_EINVAL
    assert lib.erpp_plan_set_faxen(None, 0, C.c_double(0.1)) == erpp.ERPP_EINVAL
    assert lib.erpp_plan_set_integrator(None, 0) == erpp.ERPP_EINVAL
    assert lib.erpp_plan_set_added_mass(None, 0, C.c_double(0.1), None) == erpp.ERPP_EINVAL
    assert lib.erpp_plan_set_rows_per_item(None, 3) == erpp.ERPP_EINVAL
    rows = C.c_int32(0)
    assert lib.erpp_plan_get_rows_per_item(None, C.byref(rows)) == erpp.ERPP_EINVAL
    assert lib.erpp_last_error()


def test_bin_static_rejects_sizes_beyond_its_scratch():
    """erpp_bin_static validates before touching the device: more cells or
    particles than its static scratch holds, bad geometry and NULL outputs give
    ERPP_EINVAL with a message."""
    erpp, lib = _lib()
    n = (C.c_int32 * 3)
    L = (C.c_double * 3)(1.0, 1.0, 1.0)
    fake = C.c_void_p(0x1000)
    st = lib.erpp_bin_static(n(256, 128, 128), L, 10, fake, fake, fake, fake, None)
    assert st == -1 and b"static scratch" in lib.erpp_last_error()
    st = lib.erpp_bin_static(n(8, 8, 8), L, (1 << 21) + 1, fake, fake, fake, fake, None)
    assert st == -1 and b"static scratch" in lib.erpp_last_error()
    st = lib.erpp_bin_static(n(8, 0, 8), L, 10, fake, fake, fake, fake, None)
    assert st == -1
    st = lib.erpp_bin_static(n(8, 8, 8), (C.c_double * 3)(1.0, -1.0, 1.0), 10, fake, fake,
                             fake, fake, None)
    assert st == -1
    st = lib.erpp_bin_static(n(8, 8, 8), L, 10, fake, fake, fake, None, None)
    assert st == -1
    st = lib.erpp_bin_static(n(8, 8, 8), L, 10, None, fake, fake, fake, None)
    assert st == -1
