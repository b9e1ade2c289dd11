"""The C-ABI library loads and exports every function include/pz.h declares;
argument validation runs on the host before any device work (no GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pz.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def pz():
    import paper_2607_24141_amd as pz
    return pz


def test_exports_every_declared_symbol(pz):
    declared = _declared()
    assert {"synth_forward", "synth_backward", "synth_batch", "pz_plan_create"} <= set(declared)
    for name in declared:
        assert hasattr(pz.lib, name), name
    assert set(declared) == set(pz.EXPORTS)


def test_version(pz):
    assert pz.pz_version() == pz.ABI_VERSION == 6


def _lines(pz, L=3, **over):
    import numpy as np
    d = dict(lam0=np.array([500.1, 500.2, 500.3])[:L], loggf=np.zeros(L), E=np.ones(L),
             sp=np.zeros(L, np.int32), ion=np.zeros(L, np.int32), gr=np.full(L, 8.0), gs=np.full(L, -5.0),
             gw=np.full(L, -8.0))
    d.update(over)
    keep = [np.ascontiguousarray(d[k], np.float64 if k not in ("sp", "ion") else np.int32) for k in
            ("lam0", "loggf", "E", "sp", "ion", "gr", "gs", "gw")]
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    ln = pz.pz_lines(L, dp(keep[0]), dp(keep[1]), dp(keep[2]), ip(keep[3]), ip(keep[4]), dp(keep[5]),
                     dp(keep[6]), dp(keep[7]))
    return ln, keep


def _create(pz, grid=None, lines=None, S=2, D=8, opts=None):
    g = grid or pz.pz_grid(500.0, 3e5, 100)
    ln, keep = lines if lines is not None else _lines(pz)
    o = opts or pz.pz_options(0.3, 0, 0, 0, 0)
    h = C.c_void_p()
    rc = pz.lib.pz_plan_create(C.byref(g), C.byref(ln), S, D, C.byref(o), C.byref(h))
    return rc, pz.lib.pz_last_error().decode()


@pytest.mark.parametrize("case,code", [
    ("N", -2), ("R", -1), ("lam", -1), ("D", -2), ("Dbig", -2), ("S", -2), ("W", -1), ("quad", -1),
    ("tile", -1), ("flags", -1), ("species", -1), ("ion", -1), ("nan", -5), ("eta", -1), ("eta_nan", -1),
    ("scat_iter", -1), ("scat_tol", -1), ("scat_e2", -6), ("LD", -2), ("tileLD", -2)])
def test_plan_validation(pz, case, code):
    import numpy as np
    kw = {}
    if case == "N":
        kw["grid"] = pz.pz_grid(500.0, 3e5, 1)
    elif case == "R":
        kw["grid"] = pz.pz_grid(500.0, -1.0, 100)
    elif case == "lam":
        kw["grid"] = pz.pz_grid(float("nan"), 3e5, 100)
    elif case == "D":
        kw["D"] = 1
    elif case == "Dbig":
        kw["D"] = pz.PZ_MAX_DEPTH + 1
    elif case == "S":
        kw["S"] = 0
    elif case == "W":
        kw["opts"] = pz.pz_options(0.0, 0, 0, 0, 0)
    elif case == "quad":
        kw["opts"] = pz.pz_options(0.3, 7, 0, 0, 0)
    elif case == "tile":
        kw["opts"] = pz.pz_options(0.3, 0, 48, 0, 0)
    elif case == "flags":
        kw["opts"] = pz.pz_options(0.3, 0, 0, 0, 4)
    elif case == "eta":
        kw["opts"] = pz.pz_options(0.3, 0, 0, 0, 0, -1e-3)
    elif case == "eta_nan":
        kw["opts"] = pz.pz_options(0.3, 0, 0, 0, 0, float("nan"))
    elif case == "scat_iter":
        kw["opts"] = pz.pz_options(0.3, 0, 0, 0, pz.PZ_FLAG_SCATTERING, 0.0, -3)
    elif case == "scat_tol":
        kw["opts"] = pz.pz_options(0.3, 0, 0, 0, pz.PZ_FLAG_SCATTERING, 0.0, 0, float("inf"))
    elif case == "scat_e2":
        kw["opts"] = pz.pz_options(0.3, pz.PZ_QUAD_E2, 0, 0, pz.PZ_FLAG_SCATTERING)
    elif case == "species":
        kw["lines"] = _lines(pz, sp=np.array([0, 5, 0], np.int32))
    elif case == "ion":
        kw["lines"] = _lines(pz, ion=np.array([0, 2, 0], np.int32))
    elif case == "nan":
        kw["lines"] = _lines(pz, loggf=np.array([0.0, np.nan, 0.0]))
    elif case == "LD":                       # L D >= 2^31: rejected before any line is read
        ln, keep = _lines(pz)
        ln.L = 27_000_000
        kw["lines"] = (ln, keep)
        kw["D"] = pz.PZ_MAX_DEPTH
    elif case == "tileLD":                   # 3.4e6 lines over one pixel tile: 2.7e8 rows >= 2^28
        L = 3_400_000
        kw["lines"] = _lines(pz, L, lam0=np.full(L, 500.1))
        kw["D"] = pz.PZ_MAX_DEPTH
    rc, msg = _create(pz, **kw)
    assert rc == code, (rc, msg)
    assert msg


def test_entry_points_reject_null_before_device_work(pz):
    assert pz.lib.synth_forward(None, None, None, None, None, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.synth_backward(None, None, None, None, None, None, None, None, None, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.pz_line_opacity(None, None, None, None, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.pz_debug_formal_solve(1, 4, None, None, 0, None, None) == pz.PZ_E_SHAPE
    assert pz.lib.pz_debug_formal_solve(8, 4, None, None, 0, None, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.synth_batch(None, 1, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.pz_select_lines(None, None, None, 1e-3, 1e-3, None, None, None, None, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.pz_scatter_iterations(None, None) == pz.PZ_E_INVALID_ARG
    assert pz.lib.pz_plan_info(None, None, None, None, None, None, None) == pz.PZ_E_INVALID_ARG


@pytest.mark.parametrize("case", ["support_low", "support_high", "order", "sigma", "vbmax", "J", "P", "vrot", "JR",
                                  "eps"])
def test_instrument_validation(pz, case):
    """pz_inst_create validates on the host before any device call."""
    import numpy as np
    g = pz.pz_grid(1550.0, 3e5, 1200)
    h = np.log1p(1.0 / 3e5)
    lam = 1550.0 * np.exp(h * np.linspace(300, 900, 40))
    sig = np.full(40, 2e-5)
    vb, P, vrot, eps = 10.0, 40, 0.0, 0.6
    if case == "support_low":
        lam[0] = 1550.0 * np.exp(h * 3)
    elif case == "support_high":
        lam[-1] = 1550.0 * np.exp(h * 1198)
    elif case == "order":
        lam[5] = lam[4]
    elif case == "sigma":
        sig[3] = 0.0
    elif case == "vbmax":
        vb = 0.0
    elif case == "J":
        vb = 1e5
    elif case == "P":
        P = 0
    elif case == "vrot":
        vrot = -1.0
    elif case == "JR":
        vrot = 2e3
    elif case == "eps":
        vrot, eps = 10.0, 1.5
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    d = pz.pz_inst_desc(P, dp(lam), dp(sig), 0.0, vb, vrot, eps)
    out = C.c_void_p()
    rc = pz.lib.pz_inst_create(C.byref(g), C.byref(d), C.byref(out))
    assert rc in (-1, -2) and out.value is None, (rc, pz.lib.pz_last_error())
