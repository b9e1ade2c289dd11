"""synth_forward_noalloc (the forward synthesis with its workspace in the
library's static device array) against synth_forward, through the C ABI.

Both run the same kernels on the same inputs, so F and F_c must agree
bitwise.  Two calls in a row, the second with a smaller plan, show that what
the first call left in the shared array does not leak into the second; a
plan too large for the array is rejected before any launch.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _forward(pz, fn, plan, wl):
    atm = pz.Atmos(wl.atm)
    par = pz.Params.from_host(wl.params)
    F = torch.full((plan.N,), np.nan, dtype=torch.float32, device="cuda")
    Fc = torch.full_like(F, np.nan)
    print(fn.__name__, wl.name, "N", plan.N, "L", plan.L, flush=True)
    fn(plan, atm, par, F, Fc)
    torch.cuda.synchronize()
    return F.cpu().numpy(), Fc.cpu().numpy()


@pytest.mark.parametrize("center_eta", [0.0, 1e-3])
def test_noalloc_equals_synth_forward(gpu_lib, center_eta):
    pz = gpu_lib
    big = W.tiny(seed=71, L=400, N=3000, D=72, S=4, n_molecular=1)
    big.params = W.random_params(np.random.default_rng(71), big.lines.L, big.atm.S, 1.3)
    small = W.tiny(seed=72, L=60, N=700, D=40, S=3)
    small.params = W.random_params(np.random.default_rng(72), small.lines.L, small.atm.S, 0.8)
    for wl in (big, small):
        plan = pz.plan_for(wl, center_eta=center_eta)
        ref = _forward(pz, pz.synth_forward, plan, wl)
        got = _forward(pz, pz.synth_forward_noalloc, plan, wl)
        assert np.all(np.isfinite(got[0])) and np.all(np.isfinite(got[1]))
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        plan.destroy()


def test_noalloc_full_size_forward(gpu_lib):
    """The 500-503 nm workload (1,795 pixels, 1,000 lines, 72 depths), twice in a row."""
    pz = gpu_lib
    wl = W.solar_500_503nm()
    plan = pz.plan_for(wl)
    ref = _forward(pz, pz.synth_forward, plan, wl)
    for _ in range(2):
        got = _forward(pz, pz.synth_forward_noalloc, plan, wl)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
    plan.destroy()


def test_noalloc_rejects_plans_beyond_the_array(gpu_lib):
    pz = gpu_lib
    wl = W.tiny(seed=73, L=60_000, N=4000, D=72, S=3)   # 60,000 x 72 x 16 B of line parameters > 64 MiB
    plan = pz.plan_for(wl)
    F = torch.zeros(plan.N, device="cuda")
    Fc = torch.zeros_like(F)
    with pytest.raises(pz.PzError) as e:
        pz.synth_forward_noalloc(plan, pz.Atmos(wl.atm), pz.Params.from_host(wl.params), F, Fc)
    assert e.value.code == pz.PZ_E_SHAPE
    torch.cuda.synchronize()
    assert float(F.abs().sum()) == 0.0                  # nothing was launched
    plan.destroy()
