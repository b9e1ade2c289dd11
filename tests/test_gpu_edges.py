"""Edge cases of the synthesis path on the GPU through the C ABI, against the
FP64 oracle: the smallest grid and atmosphere the ABI accepts (N = 2, D = 2,
one line), the largest depth count (D = 80), strongly damped lines (a from
0.01 to several thousand: the float64 core and the large-a wings), a jump of
the perturber density between adjacent layers (a from ~1 to ~3e4 inside one
wavefront), damping ratios from ~3 to ~900 over the depths of every line (one
wing tier for all of a wavefront's depth groups), 200 identical lines in one
tile (many LDS chunks), every LDS chunk count of a tile from 1 to 59, and
the backward of an empty catalogue (zero abundance and microturbulence
gradients)."""
import copy

import numpy as np
import pytest
import torch

import workloads as W
from oracle import synth as O
from test_gpu_adjoint import grad_close_cond, gpu_vjp
from test_gpu_forward import FLUX_RTOL, _flux_close, _run_forward

pytestmark = pytest.mark.gpu


def _kappa(pz, wl):
    plan = pz.plan_for(wl)
    kap = torch.empty((wl.atm.D, wl.grid.N), dtype=torch.float32, device="cuda")
    print("pz_line_opacity", wl.name, flush=True)
    pz.pz_line_opacity(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params), kap)
    torch.cuda.synchronize()
    return kap.cpu().numpy().astype(np.float64)


def _check_vjp(pz, wl, seed):
    s = np.random.default_rng(seed).normal(size=wl.grid.N).astype(np.float32)
    g = gpu_vjp(pz, wl, s)
    ref = O.adjoint(wl, wl.params, s.astype(np.float64), conditions=True)
    grad_close_cond(g[0], ref["g_loggf"], ref["abs_loggf"], name="loggf")
    grad_close_cond(g[1], ref["g_damp"], ref["abs_damp"], name="damp")
    grad_close_cond(g[2], ref["g_abund"], ref["abs_abund"], name="abund")
    grad_close_cond(g[3], ref["g_xi"], ref["abs_xi"], name="xi")


def test_smallest_problem(gpu_lib):
    wl = W.tiny(seed=72, L=1, N=2, D=2, S=2)
    wl.lines.lam0_nm[0] = O.wavelengths_nm(wl.grid)[1]
    wl.params = W.random_params(np.random.default_rng(72), 1, 2, 1.0)
    F, Fc = _run_forward(gpu_lib, wl)
    _flux_close(F, Fc, *O.synthesize(wl))
    assert np.all(F < Fc)
    _check_vjp(gpu_lib, wl, 72)


def test_largest_depth_count(gpu_lib):
    wl = W.tiny(seed=73, L=50, N=900, D=gpu_lib.PZ_MAX_DEPTH, S=4, n_molecular=1)
    wl.params = W.random_params(np.random.default_rng(73), 50, 4, 1.1)
    F, Fc = _run_forward(gpu_lib, wl)
    _flux_close(F, Fc, *O.synthesize(wl))
    _check_vjp(gpu_lib, wl, 73)


def test_strongly_damped_lines(gpu_lib):
    wl = W.tiny(seed=71, L=40, N=600, D=40, S=4, n_molecular=1)
    wl.lines.log_gvdw = wl.lines.log_gvdw + 4.0
    wl.lines.log_gstark = wl.lines.log_gstark + 3.0
    wl.params = W.random_params(np.random.default_rng(71), 40, 4, 1.0)
    got = _kappa(gpu_lib, wl)
    ref = O.line_opacity(wl, wl.params)
    kc = O.continuum_opacity(wl)[None, :]
    err = np.abs(got - ref) / (ref + 1e-6 * kc)
    print("strong damping: max kappa err %.3e" % err.max(), flush=True)
    assert np.all(np.isfinite(got)) and err.max() <= 2e-5
    F, Fc = _run_forward(gpu_lib, wl)
    _flux_close(F, Fc, *O.synthesize(wl))
    _check_vjp(gpu_lib, wl, 71)


def test_damping_jump_between_layers(gpu_lib):
    """n_pert x 100 from layer 8 down: the damping ratio runs from ~1 to ~3e4
    within one 16-depth group of the opacity kernel, so near and far lanes
    share a wavefront; each must use a Voigt tier valid for it."""
    wl = W.tiny(seed=76, L=6, N=300, D=24, S=3)
    wl.atm = copy.deepcopy(wl.atm)
    wl.atm.npert[8:] *= 1e2
    wl.lines.log_gvdw[:] = -3.0
    wl.lines.log_gstark[:] = -12.0
    wl.lines.log_grad[:] = 5.0
    got = _kappa(gpu_lib, wl)
    ref = O.line_opacity(wl, wl.params)
    kc = O.continuum_opacity(wl)[None, :]
    err = np.abs(got - ref) / (ref + 1e-6 * kc)
    print("damping jump: max kappa err %.3e" % err.max(), flush=True)
    assert np.all(np.isfinite(got)) and err.max() <= 2e-5


def test_wing_tiers_across_depths(gpu_lib):
    """Damping ratio from ~3 at the top to ~900 at the bottom of 72 depths
    for every line (not flagged for the wide pass, a < 1000): away from the
    line centres a wavefront's lanes span |z| from ~5.5 to ~900 over its depth
    groups, so the opacity kernel sums all of them with one wing tier (the
    6-node tier up to |z| ~ 900, the 4-node and 2-node tiers farther out)."""
    import math
    wl = W.tiny(seed=78, L=30, N=900, D=72, S=3)
    wl.lines.log_gstark[:] = -14.0
    p = wl.params
    dnu = O.line_depth_params(wl.atm, wl.lines, p.dgf, p.ddamp, p.dA, p.xi_kms)["dnu"]
    wl.lines.log_grad[:] = np.log10(3.0 * 4 * math.pi * dnu[:, 0])
    wl.lines.log_gvdw[:] = np.log10(900.0 * 4 * math.pi * dnu[:, -1] / wl.atm.npert[-1])
    a = O.line_depth_params(wl.atm, wl.lines, p.dgf, p.ddamp, p.dA, p.xi_kms)["a"]
    assert 2.5 < a.min() and a.max() < 1000.0
    got = _kappa(gpu_lib, wl)
    ref = O.line_opacity(wl, wl.params)
    kc = O.continuum_opacity(wl)[None, :]
    err = np.abs(got - ref) / (ref + 1e-6 * kc)
    print("wing tiers: max kappa err %.3e" % err.max(), flush=True)
    assert np.all(np.isfinite(got)) and err.max() <= 2e-5
    F, Fc = _run_forward(gpu_lib, wl)
    _flux_close(F, Fc, *O.synthesize(wl))


def test_identical_lines_pile_up(gpu_lib):
    wl = W.tiny(seed=74, L=200, N=400, D=24, S=3)
    one = wl.lines.take(np.zeros(200, int))                 # 200 copies of line 0
    one.lam0_nm[:] = O.wavelengths_nm(wl.grid)[200] + 1e-4
    wl.lines = one
    wl.params = W.zero_params(200, 3, 1.0)
    got = _kappa(gpu_lib, wl)
    ref = O.line_opacity(wl, wl.params)
    kc = O.continuum_opacity(wl)[None, :]
    assert np.max(np.abs(got - ref) / (ref + 1e-6 * kc)) <= 2e-5
    single = W.Workload("single", wl.grid, wl.atm, wl.lines.take([0]), W.zero_params(1, 3, 1.0))
    np.testing.assert_allclose(got, 200.0 * _kappa(gpu_lib, single), rtol=2e-5, atol=1e-30)


def _kappa_opts(pz, wl, **kw):
    plan = pz.plan_for(wl, **kw)
    kap = torch.empty((wl.atm.D, wl.grid.N), dtype=torch.float32, device="cuda")
    print("pz_line_opacity", wl.name, kw, flush=True)
    pz.pz_line_opacity(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params), kap)
    torch.cuda.synchronize()
    return kap.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("L,chunk", [(61, 1), (61, 2), (61, 3), (61, 5), (20, 7), (20, 16), (9, 16), (9, 3)])
def test_lds_chunk_counts(gpu_lib, L, chunk):
    """The tiles of these cases hold 4 to 59 lines, so LDS chunks of 1 to 16
    lines give every chunk count from 1 to 59, odd and even: the paired
    double buffer (first and second of a pair, the last chunk alone, the
    window fields staged two chunks ahead) and the centre test's single
    buffer.  Plain opacity against the oracle at two tile widths; with the
    centre test, the same opacity as with 16-line chunks up to the rounding
    of a different line order."""
    pz = gpu_lib
    wl = W.tiny(seed=76, L=L, N=400, D=72, S=4, n_molecular=1)
    wl.params = W.random_params(np.random.default_rng(76), L, 4, 1.2)
    ref = O.line_opacity(wl, wl.params)
    kc = O.continuum_opacity(wl)[None, :]
    for tile in (32, 64):
        got = _kappa_opts(pz, wl, tile_px=tile, lines_per_chunk=chunk)
        err = np.abs(got - ref) / (ref + 1e-6 * kc)
        print("L %d chunk %d tile %d: max kappa err %.3e" % (L, chunk, tile, err.max()), flush=True)
        assert err.max() <= 2e-5
    wl.center_eta = 1e-3
    a = _kappa_opts(pz, wl, lines_per_chunk=chunk)
    b = _kappa_opts(pz, wl, lines_per_chunk=16)
    assert np.all(np.abs(a - b) <= 2e-6 * np.abs(b) + 1e-9 * kc)


def test_backward_of_empty_catalogue(gpu_lib):
    pz = gpu_lib
    wl = W.tiny(seed=75, L=0, N=300, D=16, S=3)
    plan = pz.plan_for(wl)
    atm, par = pz.Atmos(wl.atm), pz.Params.from_host(wl.params)
    F, Fc = torch.empty(plan.N, device="cuda"), torch.empty(plan.N, device="cuda")
    pz.synth_forward(plan, atm, par, F, Fc)
    ga = torch.full((plan.S,), float("nan"), device="cuda")
    gx = torch.full((1,), float("nan"), device="cuda")
    s = torch.ones(plan.N, device="cuda")
    pz.synth_backward(plan, atm, par, s, None, None, ga, gx)
    torch.cuda.synchronize()
    assert np.all(ga.cpu().numpy() == 0.0) and float(gx[0]) == 0.0
