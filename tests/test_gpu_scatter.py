"""Transfer with continuum scattering (Sec. 2.1, Eqs. 3 and 6-8) on the GPU
through the C ABI, against the FP64 oracle (oracle/scatter.py), which solves
each pixel's fixed point S = eps B + (1 - eps) Lambda S as a linear system and
differentiates by complex step.  The GPU iterates to the same fixed point
(accelerated Lambda iteration, float64) and solves the adjoint fixed point.

Tolerances: F and F_c to 1e-5 relative (the float32 line opacity is the only
float32 input); dL/dkappa_line elementwise to 2e-5 of each pixel's largest
magnitude; line gradients with the conditioning-aware bound of the plain
path."""
import copy

import numpy as np
import pytest
import torch

import workloads as W
from oracle import scatter as SC
from oracle import synth as O

pytestmark = pytest.mark.gpu


def _wl(seed, L, N, D, sigma0, salpha=0.0):
    wl = W.tiny(seed=seed, L=L, N=N, D=D, S=4, n_molecular=1, xi=1.2)
    wl.params = W.random_params(np.random.default_rng(seed), L, 4, 1.2)
    wl.atm = copy.deepcopy(wl.atm)
    j = np.arange(D)
    wl.atm.sigma_c = sigma0 * (1.0 + 0.5 * np.sin(0.7 * j))
    wl.atm.sigma_alpha = salpha
    return wl


def _forward(pz, wl, **kw):
    plan = pz.plan_for(wl, **kw)
    F = torch.empty(wl.grid.N, device="cuda")
    Fc = torch.empty(wl.grid.N, device="cuda")
    pz.synth_forward(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params), F, Fc)
    torch.cuda.synchronize()
    return plan, F.cpu().numpy().astype(np.float64), Fc.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("seed,L,N,D,sigma0,salpha", [(61, 40, 800, 72, 0.5, 0.0), (62, 30, 600, 30, 3.0, -4.0),
                                                      (63, 20, 500, 8, 10.0, 0.0)])
def test_forward_vs_oracle(gpu_lib, seed, L, N, D, sigma0, salpha):
    wl = _wl(seed, L, N, D, sigma0, salpha)
    print("scatter forward seed=%d D=%d sigma0=%g" % (seed, D, sigma0), flush=True)
    plan, F, Fc = _forward(gpu_lib, wl)
    Fo, Fco = SC.synthesize(wl)
    err = max(np.max(np.abs(F / Fo - 1)), np.max(np.abs(Fc / Fco - 1)))
    it = plan.scatter_iterations()
    print("max rel err %.3e, iterations %s" % (err, it), flush=True)
    assert err <= 1e-5
    assert 1 < it[0] < 500 and 1 < it[1] < 500
    # scattering changes the flux at this strength
    Fp, Fcp = O.synthesize(wl)
    assert np.max(np.abs(Fco / Fcp - 1)) > 1e-3


def test_zero_scattering_equals_plain_transfer(gpu_lib):
    wl = _wl(64, 30, 700, 72, 0.0)
    _, F, Fc = _forward(gpu_lib, wl)
    plain = copy.deepcopy(wl)
    plain.atm.sigma_c = None
    _, Fp, Fcp = _forward(gpu_lib, plain)
    np.testing.assert_allclose(F, Fp, rtol=1e-5)
    np.testing.assert_allclose(Fc, Fcp, rtol=1e-5)


@pytest.mark.parametrize("seed,L,N,D,sigma0", [(65, 30, 400, 72, 0.8), (66, 12, 300, 20, 5.0)])
def test_opacity_adjoint_vs_oracle(gpu_lib, seed, L, N, D, sigma0):
    pz = gpu_lib
    wl = _wl(seed, L, N, D, sigma0)
    s = np.random.default_rng(seed).normal(size=N).astype(np.float32)
    plan = pz.plan_for(wl)
    g = torch.empty((D, N), device="cuda")
    print("scatter adjoint seed=%d D=%d" % (seed, D), flush=True)
    pz.pz_debug_opacity_adjoint(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params),
                                torch.as_tensor(s, device="cuda"), g)
    torch.cuda.synchronize()
    ref = SC.opacity_adjoint(wl, O.line_opacity(wl), s.astype(np.float64))
    err = np.abs(g.cpu().numpy() - ref) / np.max(np.abs(ref), axis=0, keepdims=True)
    print("max rel err of dL/dkappa %.3e, iterations %s" % (err.max(), plan.scatter_iterations()), flush=True)
    assert err.max() <= 2e-5


def test_vjp_vs_oracle(gpu_lib):
    from test_gpu_adjoint import grad_close_cond, gpu_vjp
    wl = _wl(67, 25, 400, 40, 1.5)
    s = np.random.default_rng(67).normal(size=wl.grid.N).astype(np.float32)
    g = gpu_vjp(gpu_lib, wl, s)
    ref = SC.adjoint(wl, wl.params, s.astype(np.float64), conditions=True)
    grad_close_cond(g[0], ref["g_loggf"], ref["abs_loggf"], name="loggf")
    grad_close_cond(g[1], ref["g_damp"], ref["abs_damp"], name="damp")
    grad_close_cond(g[2], ref["g_abund"], ref["abs_abund"], name="abund")
    grad_close_cond(g[3], ref["g_xi"], ref["abs_xi"], name="xi")


def test_backward_without_forward_recomputes(gpu_lib):
    """synth_backward on a plan whose last forward was another atmosphere solves
    the scattering forward again: bitwise the same gradients."""
    pz = gpu_lib
    wl = _wl(68, 20, 500, 72, 1.0)
    other = _wl(68, 20, 500, 72, 2.0)
    plan = pz.plan_for(wl)
    atm, atm2, par = pz.Atmos(wl.atm), pz.Atmos(other.atm), pz.Params.from_host(wl.params)
    s = torch.as_tensor(np.random.default_rng(5).normal(size=wl.grid.N).astype(np.float32), device="cuda")
    F, Fc = torch.empty(wl.grid.N, device="cuda"), torch.empty(wl.grid.N, device="cuda")
    outs = []
    for prior in (atm, atm2):
        pz.synth_forward(plan, prior, par, F, Fc)
        g = [torch.empty(plan.L, device="cuda"), torch.empty(plan.L, device="cuda"),
             torch.empty(plan.S, device="cuda"), torch.empty(1, device="cuda")]
        pz.synth_backward(plan, atm, par, s, *g)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in g])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_scattering_rejected_where_unsupported(gpu_lib):
    pz = gpu_lib
    wl = _wl(69, 5, 200, 10, 1.0)
    plan = pz.Plan(wl.grid, wl.lines, wl.atm.S, wl.atm.D)      # built without the scattering workspace
    F = torch.empty(wl.grid.N, device="cuda")
    with pytest.raises(pz.PzError):
        pz.synth_forward(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params), F, torch.empty_like(F))


def test_full_size_sampled(gpu_lib):
    """The 1500-1700 nm workload (37,550 pixels, 2e5 lines, 72 depths) with grey
    scattering sigma_c = 0.5 kappa_0, as the bench times it: F, F_c and
    dL/dkappa_line at sampled pixels against the oracle's per-pixel fixed
    point and complex-step derivative."""
    pz = gpu_lib
    wl = W.giant_1500_1700nm()
    wl.atm = copy.deepcopy(wl.atm)
    wl.atm.sigma_c = np.full(wl.atm.D, 0.5 * wl.atm.kappa0)
    wl.atm.sigma_alpha = 0.0
    print("scatter full size", flush=True)
    plan, F, Fc = _forward(pz, wl)
    rng = np.random.default_rng(11)
    pix = np.unique(rng.integers(0, wl.grid.N, 24))
    Fo, Fco = SC.synthesize(wl, None, pix)
    err = max(np.max(np.abs(F[pix] / Fo - 1)), np.max(np.abs(Fc[pix] / Fco - 1)))
    print("full size: max rel err %.3e at %d pixels, iterations %s" % (err, pix.size, plan.scatter_iterations()),
          flush=True)
    assert err <= 1e-5
    s = rng.normal(size=wl.grid.N).astype(np.float32)
    g = torch.empty((wl.atm.D, wl.grid.N), device="cuda")
    pz.pz_debug_opacity_adjoint(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params),
                                torch.as_tensor(s, device="cuda"), g)
    torch.cuda.synchronize()
    ref = SC.opacity_adjoint(wl, O.line_opacity(wl, None, pix), s[pix].astype(np.float64), pix)
    got = g.cpu().numpy()[:, pix]
    e = np.abs(got - ref) / np.max(np.abs(ref), axis=0, keepdims=True)
    print("full size: max rel err of dL/dkappa %.3e" % e.max(), flush=True)
    assert e.max() <= 2e-5
