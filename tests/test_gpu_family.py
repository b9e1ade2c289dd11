"""Per-family damping corrections of Eq. 30 on the GPU, through the C ABI:
forward with radiative, Stark and van der Waals corrections, and the
[3][L] damping gradients (PZ_FLAG_DAMPING_FAMILIES) against the oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import synth as O
from test_gpu_adjoint import grad_close_cond
from test_gpu_forward import _flux_close, _run_forward

pytestmark = pytest.mark.gpu


def _wl(seed, L, N, D):
    wl = W.tiny(seed=seed, L=L, N=N, D=D, S=4, n_molecular=1, xi=1.2)
    rng = np.random.default_rng(seed)
    wl.params = W.random_params(rng, L, 4, 1.2)
    wl.params.ddamp_family = rng.normal(0.0, 0.3, (3, L))
    return wl


@pytest.mark.parametrize("seed,L,N,D", [(111, 40, 900, 72), (112, 25, 500, 8)])
def test_family_forward_vs_oracle(gpu_lib, seed, L, N, D):
    wl = _wl(seed, L, N, D)
    F, Fc = _run_forward(gpu_lib, wl)
    Fo, Fco = O.synthesize(wl)
    _flux_close(F, Fc, Fo, Fco)


@pytest.mark.parametrize("seed,L,N,D,eta", [(113, 40, 900, 72, 0.0), (114, 30, 700, 72, 1e-3)])
def test_family_gradients_vs_oracle(gpu_lib, seed, L, N, D, eta):
    pz = gpu_lib
    wl = _wl(seed, L, N, D)
    wl.center_eta = eta
    s = np.random.default_rng(seed).normal(size=N).astype(np.float32)
    plan = pz.plan_for(wl, flags=pz.PZ_FLAG_DAMPING_FAMILIES)
    atm, par = pz.Atmos(wl.atm), pz.Params.from_host(wl.params)
    g = [torch.full((L,), np.nan, device="cuda"), torch.full((3 * L,), np.nan, device="cuda"),
         torch.full((4,), np.nan, device="cuda"), torch.full((1,), np.nan, device="cuda")]
    print("synth_backward with damping families", flush=True)
    pz.synth_backward(plan, atm, par, torch.as_tensor(s, device="cuda"), *g)
    torch.cuda.synchronize()
    g = [x.cpu().numpy().astype(np.float64) for x in g]
    ref = O.adjoint(wl, wl.params, s.astype(np.float64), conditions=True)
    fam = g[1].reshape(3, L)
    for f, name in enumerate(("rad", "stark", "vdw")):
        grad_close_cond(fam[f], ref["g_damp_family"][f], ref["abs_damp_family"][f], name=name)
    grad_close_cond(g[0], ref["g_loggf"], ref["abs_loggf"], name="loggf")
    grad_close_cond(g[2], ref["g_abund"], ref["abs_abund"], name="abund")
    grad_close_cond(g[3], ref["g_xi"], ref["abs_xi"], name="xi")
    # the families sum to the total-width gradient of a plan without the flag
    plan2 = pz.plan_for(wl)
    gt = torch.empty(L, device="cuda")
    pz.synth_backward(plan2, atm, par, torch.as_tensor(s, device="cuda"), None, gt, None, None)
    torch.cuda.synchronize()
    grad_close_cond(fam.sum(axis=0), gt.cpu().numpy(), ref["abs_damp"], name="sum")
