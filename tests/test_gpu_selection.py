"""The line-selection keep test of Sec. 3 (Eqs. 17-19) on the GPU through the C
ABI, against the FP64 oracle (oracle/selection.py).

Both sides decide in float64 from the same formulas; their exp/log/pow
roundings differ by ulps (the oracle takes the corrections rounded to the
float32 the GPU receives), so R and R_deep agree to 1e-12 relative and the keep
masks agree exactly except for a line whose proxy lies within 1e-12 of the
threshold (none in these cases; the test checks it).  Also: the count output,
edge bins, corrections, the 2e5- and 5e6-line catalogues, and a synthesis of
the selected subset against the oracle's synthesis of its own subset."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import selection as OS
from oracle import synth as O

pytestmark = pytest.mark.gpu


def _f32_params(p):
    """The corrections as the GPU receives them (float32), in float64 for the oracle."""
    r = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return W.Params(r(p.dgf), r(p.ddamp), r(p.dA), float(np.float32(p.xi_kms)))


def _run(pz, wl, eta, bin_ln):
    plan = pz.plan_for(wl)
    atm, par = pz.Atmos(wl.atm), pz.Params.from_host(wl.params)
    L = wl.lines.L
    keep = torch.empty(L, dtype=torch.uint8, device="cuda")
    R = torch.empty(L, dtype=torch.float64, device="cuda")
    Rd = torch.empty(L, dtype=torch.float64, device="cuda")
    n = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    print("pz_select_lines %s L=%d eta=%g bin=%g" % (wl.name, L, eta, bin_ln), flush=True)
    pz.pz_select_lines(plan, atm, par, eta, bin_ln, keep, R, Rd, n)
    torch.cuda.synchronize()
    out = keep.cpu().numpy().astype(bool), R.cpu().numpy(), Rd.cpu().numpy(), int(n.cpu()[0])
    plan.destroy()
    return out


def _compare(wl, got, ref, bin_ln):
    keep, R, Rd, n = got
    b_frac = np.log(wl.lines.lam0_nm / wl.grid.lam_first_nm) / bin_ln
    edge = np.abs(b_frac - np.round(b_frac)) < 1e-9
    assert not edge.any()                              # no line on a bin boundary in these cases
    np.testing.assert_allclose(R, ref["R"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(Rd, ref["R_deep"], rtol=1e-12, atol=0)
    near = (np.abs(ref["R"] - 1.0) < 1e-12) | (np.abs(ref["R_deep"] - 1.0) < 1e-12)
    assert not near.any()
    np.testing.assert_array_equal(keep, ref["keep"])
    assert n == int(keep.sum())


@pytest.mark.parametrize("seed,eta,bin_ln", [(11, 1e-3, 1e-3), (12, 1e-2, 3e-4), (13, 1e-4, 2e-3)])
def test_keep_test_vs_oracle_small(gpu_lib, seed, eta, bin_ln):
    wl = W.tiny(seed=seed, L=400, N=3000, D=40, S=6, n_molecular=1, lam_lo=1500.0)
    wl.params = _f32_params(W.random_params(np.random.default_rng(seed), wl.lines.L, 6, 1.1))
    wl.lines.lam0_nm[:2] = [1499.5, 1520.0]            # outside the grid: edge bins
    ref = OS.select_lines(wl, wl.params, eta, bin_ln)
    assert 0 < ref["keep"].sum() < wl.lines.L
    _compare(wl, _run(gpu_lib, wl, eta, bin_ln), ref, bin_ln)


@pytest.mark.parametrize("make", [W.giant_1500_1700nm, W.solar_300_1000nm])
def test_keep_test_vs_oracle_full_catalogues(gpu_lib, make):
    wl = make()
    wl.params = _f32_params(wl.params)
    ref = OS.select_lines(wl, wl.params, 1e-3, 1e-3)
    _compare(wl, _run(gpu_lib, wl, 1e-3, 1e-3), ref, 1e-3)


def test_selected_synthesis_vs_oracle(gpu_lib):
    """Synthesis of the kept subset: GPU (its own mask) vs the oracle (its own
    mask) to the forward tolerance, and the change from the full catalogue."""
    pz = gpu_lib
    wl = W.tiny(seed=21, L=500, N=2500, D=72, S=6, n_molecular=1, lam_lo=1500.0)
    wl.params = _f32_params(W.random_params(np.random.default_rng(21), wl.lines.L, 6, 1.0))
    eta = 3e-2
    ref = OS.select_lines(wl, wl.params, eta, 1e-3)
    keep = _run(pz, wl, eta, 1e-3)[0]
    np.testing.assert_array_equal(keep, ref["keep"])
    idx = np.flatnonzero(keep)
    sub = W.Workload(wl.name + "_sel", wl.grid, wl.atm, wl.lines.take(idx),
                     W.Params(wl.params.dgf[idx], wl.params.ddamp[idx], wl.params.dA, wl.params.xi_kms),
                     window_nm=wl.window_nm)
    Fo, Fco = O.synthesize(sub)
    plan = pz.plan_for(sub)
    F = torch.empty(wl.grid.N, device="cuda")
    Fc = torch.empty(wl.grid.N, device="cuda")
    pz.synth_forward(plan, pz.Atmos(sub.atm), pz.Params.from_host(sub.params), F, Fc)
    torch.cuda.synchronize()
    np.testing.assert_allclose(F.cpu().numpy(), Fo, rtol=1e-4)
    Ff, Fcf = O.synthesize(wl)
    dmax = np.max(np.abs(Fo / Fco - Ff / Fcf))
    print("kept %d of %d lines; max |f_selected - f_full| = %.3e" % (idx.size, wl.lines.L, dmax), flush=True)
    assert 0 < idx.size < wl.lines.L and dmax < 0.05
