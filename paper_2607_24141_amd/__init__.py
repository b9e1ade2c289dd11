"""Python binding of libpz (MI355X / gfx950 LTE spectral synthesis).

Argument marshalling only: every step of the synthesis runs in the HIP
kernels behind the C ABI declared in include/pz.h.  PyTorch supplies device
memory and the stream.  Importing this package fails loudly if the library has
not been built (there is no CPU fallback).

Names follow the C ABI: pz_plan_create, synth_forward, synth_backward,
synth_batch, pz_line_opacity, pz_debug_formal_solve, ...
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpz.so")

PZ_OK = 0
PZ_E_INVALID_ARG = -1
PZ_E_SHAPE = -2
PZ_E_NOMEM = -3
PZ_E_HIP = -4
PZ_E_NONFINITE = -5
PZ_E_UNSUPPORTED = -6
PZ_QUAD_GAUSS3 = 0
PZ_QUAD_E2 = 1
PZ_FLAG_DAMPING_FAMILIES = 1
PZ_FLAG_SCATTERING = 2
PZ_MODE_FWD = 1
PZ_MODE_FWD_BWD = 2
PZ_MAX_DEPTH = 80
PZ_NOALLOC_SCRATCH_BYTES = 64 << 20
PZ_N_STAGES = 7
STAGES = ("populations", "line_params", "opacity", "flux", "reverse_scan", "gather", "reduce")

_c_double_p = C.POINTER(C.c_double)
_c_int_p = C.POINTER(C.c_int32)
_c_float_p = C.POINTER(C.c_float)


class pz_grid(C.Structure):
    _fields_ = [("lam_first_nm", C.c_double), ("R", C.c_double), ("N", C.c_int32)]


class pz_lines(C.Structure):
    _fields_ = [("L", C.c_int32), ("lam0_nm", _c_double_p), ("loggf", _c_double_p), ("E_eV", _c_double_p),
                ("species", _c_int_p), ("ion", _c_int_p), ("log_grad", _c_double_p),
                ("log_gstark", _c_double_p), ("log_gvdw", _c_double_p)]


ABI_VERSION = 6   # PZ_VERSION of include/pz.h the structures below follow


class pz_options(C.Structure):
    _fields_ = [("window_nm", C.c_double), ("quadrature", C.c_int32), ("tile_px", C.c_int32),
                ("lines_per_chunk", C.c_int32), ("flags", C.c_int32), ("center_eta", C.c_double),
                ("scatter_max_iter", C.c_int32), ("scatter_tol", C.c_double)]


class pz_inst_desc(C.Structure):
    _fields_ = [("P", C.c_int32), ("lam_obs_nm", _c_double_p), ("lsf_sigma_ln", _c_double_p),
                ("lsf_trunc", C.c_double), ("vb_max_kms", C.c_double), ("vrot_max_kms", C.c_double),
                ("limb_eps", C.c_double)]


class pz_atmos(C.Structure):
    _fields_ = [("D", C.c_int32), ("S", C.c_int32), ("T", C.c_void_p), ("m", C.c_void_p), ("ne", C.c_void_p),
                ("npert", C.c_void_p), ("rho", C.c_void_p), ("n_species", C.c_void_p),
                ("chi_ion_eV", C.c_void_p), ("U", C.c_void_p), ("mass_amu", C.c_void_p),
                ("kappa0", C.c_double), ("lam_ref_nm", C.c_double), ("alpha", C.c_double),
                ("sigma_c", C.c_void_p), ("sigma_alpha", C.c_double)]


class pz_params(C.Structure):
    _fields_ = [("dgf", C.c_void_p), ("ddamp", C.c_void_p), ("dA", C.c_void_p), ("xi_kms", C.c_void_p),
                ("ddamp_family", C.c_void_p)]


class pz_star(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("atm", pz_atmos), ("par", pz_params), ("F", C.c_void_p),
                ("Fc", C.c_void_p), ("dL_dF", C.c_void_p), ("y", C.c_void_p), ("sigma", C.c_float),
                ("loss", C.c_void_p), ("g_loggf", C.c_void_p), ("g_damp", C.c_void_p),
                ("g_abund", C.c_void_p), ("g_xi", C.c_void_p)]


class PzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libpz error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpz.so is not built (%s); run paper_2607_24141_amd/build.py" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    lib.pz_version.restype = C.c_int
    if lib.pz_version() != ABI_VERSION:
        raise ImportError("libpz.so reports ABI version %d, this binding needs %d; rebuild with "
                          "paper_2607_24141_amd/build.py" % (lib.pz_version(), ABI_VERSION))
    lib.pz_last_error.restype = C.c_char_p
    lib.pz_plan_create.argtypes = [C.POINTER(pz_grid), C.POINTER(pz_lines), C.c_int32, C.c_int32,
                                   C.POINTER(pz_options), C.POINTER(C.c_void_p)]
    lib.pz_plan_destroy.argtypes = [C.c_void_p]
    lib.pz_plan_destroy.restype = None
    lib.pz_plan_info.argtypes = [C.c_void_p] + [_c_int_p] * 5 + [C.POINTER(C.c_int64)]
    lib.synth_forward.argtypes = [C.c_void_p, C.POINTER(pz_atmos), C.POINTER(pz_params), C.c_void_p,
                                  C.c_void_p, C.c_void_p]
    lib.synth_forward_noalloc.argtypes = lib.synth_forward.argtypes
    lib.synth_backward.argtypes = [C.c_void_p, C.POINTER(pz_atmos), C.POINTER(pz_params), C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pz_line_opacity.argtypes = [C.c_void_p, C.POINTER(pz_atmos), C.POINTER(pz_params), C.c_void_p,
                                    C.c_void_p]
    lib.pz_debug_opacity_adjoint.argtypes = [C.c_void_p, C.POINTER(pz_atmos), C.POINTER(pz_params), C.c_void_p,
                                             C.c_void_p, C.c_void_p]
    lib.pz_debug_formal_solve.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                          C.c_void_p, C.c_void_p]
    lib.pz_chi2_seed.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pz_plan_invalidate.argtypes = [C.c_void_p]
    lib.pz_plan_profile.argtypes = [C.c_void_p, C.c_int32]
    lib.pz_plan_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), _c_int_p]
    lib.pz_batch_create.argtypes = [C.c_int32, C.POINTER(pz_star), C.POINTER(C.c_void_p)]
    lib.pz_batch_destroy.argtypes = [C.c_void_p]
    lib.pz_batch_destroy.restype = None
    lib.synth_batch.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.pz_autotune.argtypes = [C.POINTER(pz_grid), C.POINTER(pz_lines), C.c_int32, C.c_int32,
                                C.POINTER(pz_options), C.POINTER(pz_atmos), C.POINTER(pz_params), C.c_int32,
                                C.POINTER(pz_options), C.POINTER(C.c_float)]
    lib.pz_inst_create.argtypes = [C.POINTER(pz_grid), C.POINTER(pz_inst_desc), C.POINTER(C.c_void_p)]
    lib.pz_inst_destroy.argtypes = [C.c_void_p]
    lib.pz_inst_destroy.restype = None
    lib.pz_inst_forward.argtypes = [C.c_void_p] + [C.c_void_p] * 6 + [C.c_void_p]
    lib.pz_inst_backward.argtypes = [C.c_void_p] + [C.c_void_p] * 7 + [C.c_void_p]
    lib.pz_scatter_iterations.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
    lib.pz_select_lines.argtypes = [C.c_void_p, C.POINTER(pz_atmos), C.POINTER(pz_params), C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pz_correction_groups.argtypes = [C.c_int32] + [C.c_void_p] * 7 + [C.c_double, C.c_double, C.c_void_p,
                                                                          _c_int_p]
    lib.pz_groups_create.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.pz_groups_destroy.argtypes = [C.c_void_p]
    lib.pz_groups_destroy.restype = None
    lib.pz_groups_info.argtypes = [C.c_void_p, _c_int_p, _c_int_p]
    lib.pz_groups_expand.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.pz_groups_reduce.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.pz_wmse_seed.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                 C.c_void_p, C.c_int32, C.c_void_p]
    for name in ("pz_plan_create", "pz_plan_info", "pz_plan_invalidate", "pz_plan_profile", "pz_plan_profile_read", "pz_chi2_seed", "synth_forward", "synth_forward_noalloc", "synth_backward", "pz_line_opacity",
                 "pz_debug_opacity_adjoint", "pz_debug_formal_solve", "pz_batch_create", "synth_batch", "pz_autotune",
                 "pz_inst_create", "pz_inst_forward", "pz_inst_backward", "pz_correction_groups",
                 "pz_select_lines", "pz_scatter_iterations", "pz_groups_create", "pz_groups_info", "pz_groups_expand", "pz_groups_reduce", "pz_wmse_seed"):
        getattr(lib, name).restype = C.c_int
    return lib


lib = _load()

EXPORTS = ("pz_version", "pz_last_error", "pz_plan_create", "pz_plan_destroy", "pz_plan_info", "pz_plan_invalidate",
           "pz_plan_profile", "pz_plan_profile_read",
           "synth_forward", "synth_forward_noalloc", "synth_backward", "pz_chi2_seed", "pz_line_opacity", "pz_debug_opacity_adjoint",
           "pz_debug_formal_solve",
           "pz_batch_create", "pz_batch_destroy", "synth_batch", "pz_autotune",
           "pz_inst_create", "pz_inst_destroy", "pz_inst_forward", "pz_inst_backward",
           "pz_select_lines", "pz_scatter_iterations", "pz_correction_groups", "pz_groups_create", "pz_groups_destroy", "pz_groups_info", "pz_groups_expand",
           "pz_groups_reduce", "pz_wmse_seed")


def _check(rc):
    if rc != PZ_OK:
        raise PzError(rc, lib.pz_last_error().decode())
    return rc


def pz_version():
    return lib.pz_version()


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------- plan
def c_grid_lines(grid, lines):
    """pz_grid and pz_lines descriptors over contiguous host copies (kept alive by the caller)."""
    keep = []

    def d(arr, dt):
        a = np.ascontiguousarray(arr, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(_c_double_p if dt == np.float64 else _c_int_p)

    g = pz_grid(float(grid.lam_first_nm), float(grid.R), int(grid.N))
    ln = pz_lines(int(len(lines.lam0_nm)), d(lines.lam0_nm, np.float64), d(lines.loggf, np.float64),
                  d(lines.E_eV, np.float64), d(lines.species, np.int32), d(lines.ion, np.int32),
                  d(lines.log_grad, np.float64), d(lines.log_gstark, np.float64), d(lines.log_gvdw, np.float64))
    return g, ln, keep


def pz_autotune(grid, lines, n_species, n_depth, atm, par, window_nm=0.3, reps=3):
    """Fastest (tile_px, lines_per_chunk) for these inputs -> (tile_px, lines_per_chunk, ms)."""
    g, ln, keep = c_grid_lines(grid, lines)
    base = pz_options(float(window_nm), PZ_QUAD_GAUSS3, 0, 0, 0)
    best = pz_options()
    ms = C.c_float()
    _check(lib.pz_autotune(C.byref(g), C.byref(ln), int(n_species), int(n_depth), C.byref(base), C.byref(atm.c),
                           C.byref(par.c), int(reps), C.byref(best), C.byref(ms)))
    del keep
    return best.tile_px, best.lines_per_chunk, ms.value


class Plan:
    """pz_plan_create / pz_plan_destroy around host line arrays (float64)."""

    def __init__(self, grid, lines, n_species, n_depth, window_nm=0.3, quadrature=PZ_QUAD_GAUSS3,
                 tile_px=0, lines_per_chunk=0, flags=0, center_eta=0.0, scatter_max_iter=0, scatter_tol=0.0):
        g, ln, keep = c_grid_lines(grid, lines)
        opts = pz_options(float(window_nm), int(quadrature), int(tile_px), int(lines_per_chunk), int(flags),
                          float(center_eta), int(scatter_max_iter), float(scatter_tol))
        h = C.c_void_p()
        _check(lib.pz_plan_create(C.byref(g), C.byref(ln), int(n_species), int(n_depth), C.byref(opts),
                                  C.byref(h)))
        del keep
        self.handle = h
        self.N, self.L, self.S, self.D, self.tile_px, self.voigt_evals = self.info()

    def info(self):
        v = [C.c_int32() for _ in range(5)]
        ev = C.c_int64()
        _check(lib.pz_plan_info(self.handle, *[C.byref(x) for x in v], C.byref(ev)))
        return tuple(x.value for x in v) + (ev.value,)

    def scatter_iterations(self):
        """pz_scatter_iterations: the largest iteration counts of the last scattering
        forward (total, continuum) and adjoint solve."""
        it = (C.c_int32 * 3)()
        _check(lib.pz_scatter_iterations(self.handle, it))
        return tuple(it)

    def invalidate(self):
        """pz_plan_invalidate: the next synth_backward recomputes the forward opacity."""
        _check(lib.pz_plan_invalidate(self.handle))

    def profile(self, enable=True):
        """pz_plan_profile: record hipEvents around this plan's kernel launches."""
        _check(lib.pz_plan_profile(self.handle, 1 if enable else 0))

    def profile_read(self):
        """pz_plan_profile_read -> {stage: (total_ms, launches)}."""
        ms = (C.c_double * PZ_N_STAGES)()
        n = (C.c_int32 * PZ_N_STAGES)()
        _check(lib.pz_plan_profile_read(self.handle, ms, n))
        return {STAGES[k]: (ms[k], n[k]) for k in range(PZ_N_STAGES)}

    def destroy(self):
        if getattr(self, "handle", None):
            lib.pz_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def plan_for(workload, **kw):
    kw.setdefault("center_eta", getattr(workload, "center_eta", 0.0))
    if getattr(workload.atm, "sigma_c", None) is not None:
        kw["flags"] = kw.get("flags", 0) | PZ_FLAG_SCATTERING
    return Plan(workload.grid, workload.lines, workload.atm.S, workload.atm.D,
                window_nm=workload.window_nm,
                quadrature=PZ_QUAD_GAUSS3 if workload.quadrature == "gauss3" else PZ_QUAD_E2, **kw)


# --------------------------------------------------------------- autotuning
TUNE_CACHE = os.path.join(_HERE, "autotune_cache.json")


def tune_key(workload):
    """Size bucket of a workload: GPU arch, log2 of pixels, log2 of lines per pixel window, depths."""
    import math
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    N, L = workload.grid.N, workload.lines.L
    win_px = 2.0 * workload.window_nm / (workload.grid.lam_first_nm / workload.grid.R)
    overlap = max(L * win_px / N, 1.0)
    return "%s|N%d|ov%d|D%d" % (arch, int(math.log2(N)), int(math.log2(overlap)), workload.atm.D)


def tuned_options(workload, atm=None, par=None, reps=3, cache_path=TUNE_CACHE):
    """(tile_px, lines_per_chunk) for a workload: from the cache, else pz_autotune (then cached)."""
    import json
    key = tune_key(workload)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    if key in cache:
        return tuple(cache[key][:2])
    atm = atm or Atmos(workload.atm)
    par = par or Params.from_host(workload.params)
    tile, chunk, ms = pz_autotune(workload.grid, workload.lines, workload.atm.S, workload.atm.D, atm, par,
                                  window_nm=workload.window_nm, reps=reps)
    cache[key] = [tile, chunk, ms]
    if cache_path:
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return tile, chunk


def plan_tuned(workload, atm=None, par=None, **kw):
    tile, chunk = tuned_options(workload, atm, par, **kw)
    return plan_for(workload, tile_px=tile, lines_per_chunk=chunk)


# ----------------------------------------------------------------- atmosphere
class Atmos:
    """Device copy (float64) of an atmosphere and its pz_atmos descriptor."""

    def __init__(self, atm, device="cuda"):
        import torch
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=device)
        self.t = dict(T=f(atm.T), m=f(atm.m), ne=f(atm.ne), npert=f(atm.npert), rho=f(atm.rho),
                      n_species=f(atm.n_species), chi=f(atm.chi_ion_eV), U=f(atm.U), mass=f(atm.mass_amu))
        t = self.t
        self.c = pz_atmos(int(atm.T.shape[0]), int(atm.mass_amu.shape[0]), t["T"].data_ptr(), t["m"].data_ptr(),
                          t["ne"].data_ptr(), t["npert"].data_ptr(), t["rho"].data_ptr(),
                          t["n_species"].data_ptr(), t["chi"].data_ptr(), t["U"].data_ptr(),
                          t["mass"].data_ptr(), float(atm.kappa0), float(atm.lam_ref_nm), float(atm.alpha),
                          None, float(getattr(atm, "sigma_alpha", 0.0)))
        sig = getattr(atm, "sigma_c", None)
        if sig is not None:
            t["sigma_c"] = f(sig)
            self.c.sigma_c = t["sigma_c"].data_ptr()


class Params:
    """Device float32 corrections (dgf[L], ddamp[L], dA[S], xi[1], optional
    ddamp_family[3][L]) and pz_params."""

    def __init__(self, dgf, ddamp, dA, xi, ddamp_family=None):
        self.dgf, self.ddamp, self.dA, self.xi, self.ddamp_family = dgf, ddamp, dA, xi, ddamp_family
        ptr = lambda t: None if t is None else t.data_ptr()
        self.c = pz_params(ptr(dgf), ptr(ddamp), ptr(dA), xi.data_ptr(), ptr(ddamp_family))

    @classmethod
    def from_host(cls, p, device="cuda"):
        import torch
        f = lambda a: torch.as_tensor(np.asarray(a, np.float32), device=device).contiguous()
        fam = getattr(p, "ddamp_family", None)
        return cls(f(p.dgf), f(p.ddamp), f(p.dA), f([p.xi_kms]), None if fam is None else f(fam))


# ------------------------------------------------------------- entry points
def synth_forward(plan, atm, par, F, Fc, stream=None):
    _check(lib.synth_forward(plan.handle, C.byref(atm.c), C.byref(par.c), _ptr(F), _ptr(Fc), _stream(stream)))


def synth_forward_noalloc(plan, atm, par, F, Fc, stream=None):
    _check(lib.synth_forward_noalloc(plan.handle, C.byref(atm.c), C.byref(par.c), _ptr(F), _ptr(Fc),
                                     _stream(stream)))


def synth_backward(plan, atm, par, dL_dF, g_loggf, g_damp, g_abund, g_xi, dL_dFc=None, stream=None):
    _check(lib.synth_backward(plan.handle, C.byref(atm.c), C.byref(par.c), _ptr(dL_dF), _ptr(dL_dFc),
                              _ptr(g_loggf), _ptr(g_damp), _ptr(g_abund), _ptr(g_xi), _stream(stream)))


def pz_line_opacity(plan, atm, par, kappa, stream=None):
    _check(lib.pz_line_opacity(plan.handle, C.byref(atm.c), C.byref(par.c), _ptr(kappa), _stream(stream)))


def pz_debug_opacity_adjoint(plan, atm, par, dL_dF, g_kappa, stream=None):
    _check(lib.pz_debug_opacity_adjoint(plan.handle, C.byref(atm.c), C.byref(par.c), _ptr(dL_dF), _ptr(g_kappa),
                                        _stream(stream)))


def pz_chi2_seed(F, Fc, y, sigma, dL_dF, dL_dFc=None, loss=None, stream=None):
    _check(lib.pz_chi2_seed(int(F.numel()), _ptr(F), _ptr(Fc), _ptr(y), float(sigma), _ptr(dL_dF), _ptr(dL_dFc),
                            _ptr(loss), _stream(stream)))


def pz_debug_formal_solve(S, tau, F, quadrature=PZ_QUAD_GAUSS3, stream=None):
    D, n = S.shape
    _check(lib.pz_debug_formal_solve(int(D), int(n), _ptr(S), _ptr(tau), int(quadrature), _ptr(F),
                                     _stream(stream)))


class Batch:
    """pz_batch_create / synth_batch over a list of pz_star descriptors."""

    def __init__(self, stars):
        arr = (pz_star * len(stars))(*stars)
        h = C.c_void_p()
        _check(lib.pz_batch_create(len(stars), arr, C.byref(h)))
        self.handle = h
        self._stars = arr

    def destroy(self):
        if getattr(self, "handle", None):
            lib.pz_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def synth_batch(batch, mode, stream=None):
    _check(lib.synth_batch(batch.handle, int(mode), _stream(stream)))


# ---------------------------------------------------------------- autograd
def _autograd_function():
    import torch

    class PzSynth(torch.autograd.Function):
        """F, Fc = PzSynth.apply(plan, atm, dgf, ddamp, dA, xi): gradients for the four corrections."""

        @staticmethod
        def forward(ctx, plan, atm, dgf, ddamp, dA, xi):
            dev = xi.device
            F = torch.empty(plan.N, dtype=torch.float32, device=dev)
            Fc = torch.empty(plan.N, dtype=torch.float32, device=dev)
            par = Params(dgf.detach().contiguous(), ddamp.detach().contiguous(), dA.detach().contiguous(),
                         xi.detach().contiguous())
            synth_forward(plan, atm, par, F, Fc)
            # torch's version counters then reject a backward after an in-place
            # edit of the corrections (the plan's workspace holds this forward)
            ctx.save_for_backward(dgf, ddamp, dA, xi)
            token = object()
            plan._autograd_token = token
            ctx.plan, ctx.atm, ctx.par, ctx.token = plan, atm, par, token
            ctx.mark_non_differentiable(Fc)
            return F, Fc

        @staticmethod
        def backward(ctx, gF, gFc):
            ctx.saved_tensors                       # raises if an input was modified in place
            plan, par = ctx.plan, ctx.par
            if getattr(plan, "_autograd_token", None) is not ctx.token:
                plan.invalidate()                   # another forward ran on this plan since: recompute
            dev = par.xi.device
            g = [torch.empty(plan.L, dtype=torch.float32, device=dev),
                 torch.empty(plan.L, dtype=torch.float32, device=dev),
                 torch.empty(plan.S, dtype=torch.float32, device=dev),
                 torch.empty(1, dtype=torch.float32, device=dev)]
            gF = torch.zeros(plan.N, dtype=torch.float32, device=dev) if gF is None else gF.contiguous()
            synth_backward(plan, ctx.atm, par, gF, *g)
            return None, None, g[0], g[1], g[2], g[3]

    return PzSynth


_PzSynth = None


def PzSynth():
    global _PzSynth
    if _PzSynth is None:
        _PzSynth = _autograd_function()
    return _PzSynth


# ------------------------------------------------------------- line selection
def pz_select_lines(plan, atm, par, eta_sel=1e-3, bin_ln=1e-3, keep=None, R=None, R_deep=None, n_keep=None,
                    stream=None):
    """The keep test of Eqs. 17-19 on the device: keep [L] uint8, R and R_deep [L]
    float64, n_keep [1] int32 (device tensors, caller line order; any may be None)."""
    for t, n, sz in ((keep, "keep", 1), (R, "R", 8), (R_deep, "R_deep", 8)):
        if t is not None and (t.numel() != plan.L or t.element_size() != sz or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous device tensor of L = %d elements of %d bytes" % (n, plan.L, sz))
    if n_keep is not None and (n_keep.numel() != 1 or n_keep.element_size() != 4):
        raise ValueError("n_keep must be one int32")
    _check(lib.pz_select_lines(plan.handle, C.byref(atm.c), C.byref(par.c), float(eta_sel), float(bin_ln),
                               _ptr(keep), _ptr(R), _ptr(R_deep), _ptr(n_keep), _stream(stream)))


def select_lines(plan, atm, par, eta_sel=1e-3, bin_ln=1e-3):
    """Host keep mask ([L] bool, caller order) of pz_select_lines."""
    import torch
    keep = torch.empty(plan.L, dtype=torch.uint8, device="cuda")
    pz_select_lines(plan, atm, par, eta_sel, bin_ln, keep=keep)
    return keep.cpu().numpy().astype(bool)


# ------------------------------------------------------------ line calibration
CM1_EV = 1.239841984e-4      # one wavenumber (cm^-1) in eV


def correction_groups(lines, dE_cm=2.0, dlam_nm=0.035, active=None, anchor=None):
    """pz_correction_groups on a line list: (group_of_line [L] int32 numpy, G).
    dE_cm in cm^-1; active: [L] bool or None (all); anchor: [L] int or None."""
    L = int(lines.L)
    keep = [np.ascontiguousarray(lines.lam0_nm, np.float64), np.ascontiguousarray(lines.E_eV, np.float64),
            np.ascontiguousarray(lines.species, np.int32), np.ascontiguousarray(lines.ion, np.int32),
            np.ascontiguousarray(lines.loggf, np.float64)]
    act = None if active is None else np.ascontiguousarray(active, np.uint8)
    anc = None if anchor is None else np.ascontiguousarray(anchor, np.int32)
    q = np.empty(L, np.int32)
    G = C.c_int32()
    p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    _check(lib.pz_correction_groups(L, *[p(a) for a in keep], p(act), p(anc), float(dE_cm) * CM1_EV,
                                    float(dlam_nm), p(q), C.byref(G)))
    return q, G.value


class Groups:
    """pz_groups_create / pz_groups_destroy: a group map on the device, with
    expand (group values -> lines) and reduce (line values -> group sums)."""

    def __init__(self, group_of_line, G):
        self._q = np.ascontiguousarray(group_of_line, np.int32)
        h = C.c_void_p()
        _check(lib.pz_groups_create(int(self._q.size), int(G), self._q.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.handle = h
        self.L, self.G = int(self._q.size), int(G)

    def _rows(self, x_group, x_line):
        R = x_group.numel() // self.G
        for t in (x_group, x_line):
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4 and t.is_contiguous()):
                raise ValueError("group and line arrays must be contiguous float32 device tensors")
        if x_group.numel() != R * self.G or x_line.numel() != R * self.L:
            raise ValueError("shapes: x_group needs R*G = %d*%d and x_line R*L = %d*%d elements (got %d, %d)"
                             % (R, self.G, R, self.L, x_group.numel(), x_line.numel()))
        return R

    def expand(self, x_group, x_line, stream=None):
        """x_line [R][L] from x_group [R][G] (device float32)."""
        R = self._rows(x_group, x_line)
        _check(lib.pz_groups_expand(self.handle, int(R), _ptr(x_group), _ptr(x_line), _stream(stream)))

    def reduce(self, x_line, x_group, accumulate=False, stream=None):
        """x_group [R][G] (+)= fixed-order group sums of x_line [R][L] (device float32)."""
        R = self._rows(x_group, x_line)
        _check(lib.pz_groups_reduce(self.handle, int(R), _ptr(x_line), _ptr(x_group), 1 if accumulate else 0,
                                    _stream(stream)))

    def destroy(self):
        if getattr(self, "handle", None):
            lib.pz_groups_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def pz_wmse_seed(f, y, w, c, dL_df=None, loss=None, accumulate=False, stream=None):
    """dL_df = 2 c w (f - y) and loss (+)= c sum w (f - y)^2 (device float32; w may be None)."""
    P = f.numel()
    if y.numel() != P or (w is not None and w.numel() != P) or (dL_df is not None and dL_df.numel() != P):
        raise ValueError("f, y, w and dL_df must all have P = %d elements" % P)
    _check(lib.pz_wmse_seed(int(f.numel()), _ptr(f), _ptr(y), _ptr(w), float(c), _ptr(dL_df), _ptr(loss),
                            1 if accumulate else 0, _stream(stream)))


# ----------------------------------------------------------------- instrument
class Instrument:
    """pz_inst_create / pz_inst_destroy: the instrument operator of Eq. 31 for a
    synthesis grid, observed pixel centres (nm), LSF widths (ln lambda) and the
    largest broadening velocity (km/s); with vrot_max_kms > 0 also a rotation
    stage (largest v sin i, linear limb-darkening coefficient limb_eps), whose
    velocity vectors then hold (v_r, v_b, v sin i)."""

    def __init__(self, grid, lam_obs_nm, lsf_sigma_ln, vb_max_kms, lsf_trunc=0.0, vrot_max_kms=0.0, limb_eps=0.6):
        import numpy as np
        self._lam = np.ascontiguousarray(lam_obs_nm, dtype=np.float64)
        self._sig = np.ascontiguousarray(lsf_sigma_ln, dtype=np.float64)
        g = pz_grid(float(grid.lam_first_nm), float(grid.R), int(grid.N))
        d = pz_inst_desc(int(self._lam.size), self._lam.ctypes.data_as(_c_double_p),
                         self._sig.ctypes.data_as(_c_double_p), float(lsf_trunc), float(vb_max_kms),
                         float(vrot_max_kms), float(limb_eps))
        h = C.c_void_p()
        _check(lib.pz_inst_create(C.byref(g), C.byref(d), C.byref(h)))
        self.handle = h
        self.N, self.P = int(grid.N), int(self._lam.size)
        self.n_vel = 3 if vrot_max_kms > 0 else 2

    def destroy(self):
        if getattr(self, "handle", None):
            lib.pz_inst_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def pz_inst_forward(inst, F, Fc, vel, KF=None, KFc=None, f=None, stream=None):
    """f = K S R B F / K S R B Fc on torch's current stream (device float32
    tensors; vel holds inst.n_vel velocities)."""
    if vel.numel() < inst.n_vel:
        raise ValueError("vel needs %d entries for this instrument" % inst.n_vel)
    _check(lib.pz_inst_forward(inst.handle, _ptr(F), _ptr(Fc), _ptr(vel), _ptr(KF), _ptr(KFc), _ptr(f),
                               _stream(stream)))


def pz_inst_backward(inst, F, Fc, vel, dL_df, dL_dF=None, dL_dFc=None, g_vel=None, stream=None):
    """VJP of pz_inst_forward's f for the seed dL_df (g_vel holds inst.n_vel entries)."""
    if vel.numel() < inst.n_vel or (g_vel is not None and g_vel.numel() < inst.n_vel):
        raise ValueError("vel and g_vel need %d entries for this instrument" % inst.n_vel)
    _check(lib.pz_inst_backward(inst.handle, _ptr(F), _ptr(Fc), _ptr(vel), _ptr(dL_df), _ptr(dL_dF),
                                _ptr(dL_dFc), _ptr(g_vel), _stream(stream)))
