"""Full-size gradient parity on the differentiation workload (1500-1700 nm,
37,550 pixels, 2e5 lines, 20 species), through the C ABI, against FP64 oracle
values stored in tests/golden/fit_1500_1700nm_golden.npz (written by
tests/golden/make_fit_1500_1700nm_golden.py, which calls only the oracle).

The chi^2 objective (Sec. 5, Eq. 9 flux ratio) is evaluated at the base
corrections against a target made from the truth corrections plus noise at
S/N = 100; the stored seed dL/dF is fed to synth_backward, so the GPU
gradients are compared with the oracle adjoint for the same seed."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from test_gpu_adjoint import grad_close_s17

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fit_1500_1700nm_golden.npz")


@pytest.fixture(scope="module")
def run(gpu_lib):
    pz = gpu_lib
    z = np.load(GOLDEN)
    wl = W.giant_1500_1700nm_fit()
    plan = pz.plan_for(wl)
    atm, par = pz.Atmos(wl.atm), pz.Params.from_host(wl.params)
    N, L, S = plan.N, plan.L, plan.S
    d = "cuda"
    F, Fc = torch.empty(N, device=d), torch.empty(N, device=d)
    print("golden: synth_forward N", N, "L", L, flush=True)
    pz.synth_forward(plan, atm, par, F, Fc)
    y = torch.as_tensor(z["y"], device=d)
    gF, loss = torch.empty(N, device=d), torch.empty(1, device=d)
    pz.pz_chi2_seed(F, Fc, y, wl.extra["sigma"], gF, None, loss)
    g = [torch.full((L,), np.nan, device=d), torch.full((L,), np.nan, device=d),
         torch.full((S,), np.nan, device=d), torch.full((1,), np.nan, device=d)]
    print("golden: synth_backward with the stored seed", flush=True)
    pz.synth_backward(plan, atm, par, torch.as_tensor(z["seed"], device=d), *g)
    torch.cuda.synchronize()
    out = dict(z=z, gF=gF.cpu().numpy().astype(np.float64), loss=float(loss.item()),
               g=[x.cpu().numpy().astype(np.float64) for x in g])
    plan.destroy()
    return out


def test_loss_and_seed(run):
    z = run["z"]
    assert abs(run["loss"] - float(z["loss"])) <= 1e-4 * float(z["loss"])
    seed = z["seed"].astype(np.float64)
    # the seed 2 (f - y)/(sigma^2 Fc) carries the flux error amplified by 1/|f - y|
    assert np.max(np.abs(run["gF"] - seed)) <= 2e-3 * np.max(np.abs(seed))


def _conditioning(got, ref, abs_sum, name):
    big = np.abs(ref) >= 1e-2 * np.max(np.abs(ref))
    cond = abs_sum[big] / np.abs(ref[big])
    err = np.abs(got - ref)[big] / np.abs(ref[big])
    print("%s: %d large of %d, max sum|t|/|g| %.1f, worst rel err %.2e, share within 1e-3 %.3f"
          % (name, int(big.sum()), ref.size, cond.max(initial=0), err.max(initial=0),
             float(np.mean(np.abs(got - ref)[np.abs(ref) > 0] <= 1e-3 * np.abs(ref[np.abs(ref) > 0])))))


def test_line_gradients(run):
    """288 sampled lines (256 random, the 32 largest |dL/d loggf|): dL/d loggf and
    dL/d ddamp within 1e-3 relative where |g_ref| >= 1e-2 of the largest of its
    kind, and within 1e-5 of the largest below that."""
    z = run["z"]
    lines = z["lines"]
    for k, name in ((0, "loggf"), (1, "damp")):
        got, ref = run["g"][k][lines], z["g_" + name]
        _conditioning(got, ref, z["abs_" + name], name)
        grad_close_s17(got, ref, name=name)


def test_species_and_xi_gradients(run):
    """The 20 abundance gradients (same rule) and the microturbulence gradient
    (1e-3 relative)."""
    z = run["z"]
    _conditioning(run["g"][2], z["g_abund"], z["abs_abund"], "abund")
    grad_close_s17(run["g"][2], z["g_abund"], name="abund")
    g_xi, ref_xi = run["g"][3][0], float(z["g_xi"])
    print("xi: got %.6e ref %.6e sum|t|/|g| %.1f" % (g_xi, ref_xi, float(z["abs_xi"]) / abs(ref_xi)))
    assert abs(g_xi - ref_xi) <= 1e-3 * abs(ref_xi), (g_xi, ref_xi)


def test_fd_parameters(run):
    """The 50 finite-difference parameters (20 log gf, 20 damping, 9 abundances,
    xi): GPU gradient within 1e-3 of the FP64 central difference where that
    is at least 1e-2 of the largest, else within 1e-5 of the largest."""
    z = run["z"]
    rich = (4.0 * z["fd_value_half"] - z["fd_value"]) / 3.0
    g = np.array([run["g"][0][i] if k == "loggf" else run["g"][1][i] if k == "damp" else
                  run["g"][2][i] if k == "abund" else run["g"][3][0] for k, i in zip(z["fd_kind"], z["fd_index"])])
    gmax = np.max(np.abs(rich))
    big = np.abs(rich) >= 1e-2 * gmax
    err = np.abs(g - rich)
    ok = np.where(big, err <= 1e-3 * np.abs(rich), err <= 1e-5 * gmax)
    assert ok.all(), [(z["fd_kind"][i], int(z["fd_index"][i]), g[i], rich[i]) for i in np.flatnonzero(~ok)[:5]]
