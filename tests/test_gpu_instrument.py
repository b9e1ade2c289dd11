"""The instrument operator of Eq. 31 on the GPU, through the C ABI, against the
FP64 oracle (oracle/instrument.py) on the APOGEE-like pixels of the
1500-1700 nm grid (7,902 observed pixels, 37,550 native).

Inputs are float32; the oracle takes the same float32 values in float64.
Forward: K S B F, K S B Fc and f to 1e-5 relative.  Backward: dL/dF and
dL/dFc to 1e-4 of their largest magnitude, the velocity gradients to 1e-3
relative (the seed is a chi^2 residual against a model at other velocities,
so their sums are not cancellation-dominated)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import instrument as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(gpu_lib):
    pz = gpu_lib
    grid = W.grid_for(1500.0, 1700.0, 3.0e5)
    lam, sig, vbmax = W.apogee_instrument(grid)
    inst = pz.Instrument(grid, lam, sig, vbmax)
    oinst = I.Instrument(grid, lam, sig, vbmax)
    rng = np.random.default_rng(3)
    x = np.arange(grid.N)
    Fc = (1.0 + 0.1 * np.sin(x / 5000.0)).astype(np.float32)
    depth = np.zeros(grid.N)
    for c in rng.uniform(0, grid.N, 400):
        w = rng.uniform(2.0, 12.0)
        depth += rng.uniform(0.05, 0.6) * np.exp(-0.5 * ((x - c) / w) ** 2)
    F = (Fc * np.exp(-depth)).astype(np.float32)
    return pz, grid, inst, oinst, F, Fc


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("vr,vb", [(0.0, 5.0), (23.7, 11.2), (-61.3, 2.4), (7.0, 0.0)])
def test_instrument_forward_vs_oracle(setup, vr, vb):
    pz, grid, inst, oinst, F, Fc = setup
    P = inst.P
    KF, KFc, f = (torch.empty(P, device="cuda") for _ in range(3))
    print("pz_inst_forward", vr, vb, flush=True)
    pz.pz_inst_forward(inst, _dev(F), _dev(Fc), _dev([vr, vb]), KF, KFc, f)
    torch.cuda.synchronize()
    rKF, rKFc, rf = I.forward(oinst, F.astype(np.float64), Fc.astype(np.float64), vr, max(vb, 1e-3 * I.C_KMS * oinst.h))
    for got, ref in ((KF, rKF), (KFc, rKFc), (f, rf)):
        np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-5)


@pytest.mark.parametrize("vr,vb", [(12.0, 6.0), (-30.0, 15.0)])
def test_instrument_backward_vs_oracle(setup, vr, vb):
    pz, grid, inst, oinst, F, Fc = setup
    F64, Fc64 = F.astype(np.float64), Fc.astype(np.float64)
    _, _, ymodel = I.forward(oinst, F64, Fc64, vr + 1.5, vb + 0.8)
    _, _, f = I.forward(oinst, F64, Fc64, vr, vb)
    seed = (2.0 * (f - ymodel) / 1e-4).astype(np.float32)       # chi^2 with sigma = 0.01
    dF, dFc = torch.empty(grid.N, device="cuda"), torch.empty(grid.N, device="cuda")
    gv = torch.full((2,), np.nan, device="cuda")
    print("pz_inst_backward", vr, vb, flush=True)
    pz.pz_inst_backward(inst, _dev(F), _dev(Fc), _dev([vr, vb]), _dev(seed), dF, dFc, gv)
    torch.cuda.synchronize()
    rdF, rdFc, rvr, rvb = I.adjoint(oinst, F64, Fc64, vr, vb, seed.astype(np.float64))
    for got, ref in ((dF, rdF), (dFc, rdFc)):
        got = got.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref))
    g = gv.cpu().numpy()
    np.testing.assert_allclose(g, [rvr, rvb], rtol=1e-3)


def test_instrument_backward_deterministic(setup):
    pz, grid, inst, oinst, F, Fc = setup
    seed = _dev(np.random.default_rng(4).normal(size=inst.P))
    outs = []
    for _ in range(2):
        dF, dFc, gv = torch.empty(grid.N, device="cuda"), torch.empty(grid.N, device="cuda"), torch.empty(2, device="cuda")
        pz.pz_inst_backward(inst, _dev(F), _dev(Fc), _dev([5.0, 4.0]), seed, dF, dFc, gv)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (dF, dFc, gv)])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def test_fit_step_through_the_instrument(gpu_lib):
    """One fitting step of Eq. 31: synthesis, instrument, chi^2 on the observed
    pixels, the instrument VJP and the synthesis VJP, against the oracle's
    chain: gradients of the four corrections and of v_r, v_b."""
    from oracle import synth as O
    from test_gpu_adjoint import grad_close_cond
    pz = gpu_lib
    wl = W.tiny(seed=91, L=60, N=2500, D=72, S=4, n_molecular=1, xi=1.4)
    wl.params = W.random_params(np.random.default_rng(91), 60, 4, 1.4)
    grid = wl.grid
    import math
    x0, h = math.log(grid.lam_first_nm), math.log1p(1.0 / grid.R)
    xp = np.arange(x0 + 150 * h, x0 + (grid.N - 150) * h, 4.2 * h)
    sig = np.full(xp.size, 5.5 * h)
    vel = (9.0, 4.0)
    inst = pz.Instrument(grid, np.exp(xp), sig, 10.0)
    oinst = I.Instrument(grid, np.exp(xp), sig, 10.0)
    # oracle chain
    Fo, Fco = O.synthesize(wl)
    _, _, fo = I.forward(oinst, Fo, Fco, *vel)
    y = fo + np.random.default_rng(2).normal(0.0, 0.01, fo.size) + 0.02 * np.sin(np.arange(fo.size) / 7.0)
    seed_o = 2.0 * (fo - y) / 1e-4
    dF_o, _, gvr_o, gvb_o = I.adjoint(oinst, Fo, Fco, *vel, seed_o)
    ref = O.adjoint(wl, wl.params, dF_o, conditions=True)
    # GPU chain
    plan = pz.plan_for(wl)
    atm, par = pz.Atmos(wl.atm), pz.Params.from_host(wl.params)
    F, Fc = torch.empty(grid.N, device="cuda"), torch.empty(grid.N, device="cuda")
    pz.synth_forward(plan, atm, par, F, Fc)
    v = _dev(vel)
    f = torch.empty(inst.P, device="cuda")
    pz.pz_inst_forward(inst, F, Fc, v, None, None, f)
    seed = (2.0 * (f - _dev(y)) / 1e-4).contiguous()
    dF, gv = torch.empty(grid.N, device="cuda"), torch.empty(2, device="cuda")
    pz.pz_inst_backward(inst, F, Fc, v, seed, dF, None, gv)
    g = [torch.empty(plan.L, device="cuda"), torch.empty(plan.L, device="cuda"), torch.empty(plan.S, device="cuda"),
         torch.empty(1, device="cuda")]
    print("fit step: synth_backward", flush=True)
    pz.synth_backward(plan, atm, par, dF, *g)
    torch.cuda.synchronize()
    g = [x.cpu().numpy().astype(np.float64) for x in g]
    grad_close_cond(g[0], ref["g_loggf"], ref["abs_loggf"], name="loggf")
    grad_close_cond(g[1], ref["g_damp"], ref["abs_damp"], name="damp")
    grad_close_cond(g[2], ref["g_abund"], ref["abs_abund"], name="abund")
    grad_close_cond(g[3], ref["g_xi"], ref["abs_xi"], name="xi")
    np.testing.assert_allclose(gv.cpu().numpy(), [gvr_o, gvb_o], rtol=2e-3)


# ------------------------------------------------- rotational broadening R
VROT_MAX = 40.0


@pytest.fixture(scope="module")
def rot_setup(setup):
    pz, grid, _, _, F, Fc = setup
    lam, sig, vbmax = W.apogee_instrument(grid)
    inst = pz.Instrument(grid, lam, sig, vbmax, vrot_max_kms=VROT_MAX, limb_eps=0.6)
    oinst = I.Instrument(grid, lam, sig, vbmax, vrot_max_kms=VROT_MAX, limb_eps=0.6)
    assert inst.n_vel == 3 and oinst.JR == 41
    return pz, grid, inst, oinst, F, Fc


@pytest.mark.parametrize("vr,vb,vs", [(0.0, 5.0, 12.5), (23.7, 3.2, 39.0), (-8.0, 2.4, 0.3), (4.0, 1.0, 46.0)])
def test_rotation_forward_vs_oracle(rot_setup, vr, vb, vs):
    """K S R B on the GPU against the oracle: a broad and a near-maximal v sin i,
    one narrower than a pixel (the identity), and one above the support (cut
    and renormalised, as the oracle does)."""
    pz, grid, inst, oinst, F, Fc = rot_setup
    P = inst.P
    KF, KFc, f = (torch.empty(P, device="cuda") for _ in range(3))
    print("pz_inst_forward rotation", vr, vb, vs, flush=True)
    pz.pz_inst_forward(inst, _dev(F), _dev(Fc), _dev([vr, vb, vs]), KF, KFc, f)
    torch.cuda.synchronize()
    rKF, rKFc, rf = I.forward(oinst, F.astype(np.float64), Fc.astype(np.float64), vr, vb, vsini=vs)
    for got, ref in ((KF, rKF), (KFc, rKFc), (f, rf)):
        np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-5)


def test_rotation_zero_is_the_plain_operator(rot_setup, setup):
    """v sin i = 0 gives r_0 = 1 and nothing else: bit-for-bit the instrument
    without a rotation stage, forward and backward (v sin i gradient zero)."""
    pz, grid, inst, _, F, Fc = rot_setup
    plain = setup[2]
    seed = _dev(np.random.default_rng(8).normal(size=inst.P))
    outs = []
    for ins, vel in ((plain, [6.0, 3.0]), (inst, [6.0, 3.0, 0.0])):
        f = torch.empty(ins.P, device="cuda")
        dF, dFc = torch.empty(grid.N, device="cuda"), torch.empty(grid.N, device="cuda")
        gv = torch.full((3,), np.nan, device="cuda")
        pz.pz_inst_forward(ins, _dev(F), _dev(Fc), _dev(vel), None, None, f)
        pz.pz_inst_backward(ins, _dev(F), _dev(Fc), _dev(vel), seed, dF, dFc, gv)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (f, dF, dFc, gv)])
    for a, b in zip(outs[0][:3], outs[1][:3]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(outs[0][3][:2], outs[1][3][:2])
    assert outs[1][3][2] == 0.0


@pytest.mark.parametrize("vr,vb,vs", [(12.0, 6.0, 18.0), (-30.0, 3.0, 33.0)])
def test_rotation_backward_vs_oracle(rot_setup, vr, vb, vs):
    """The VJP through R: dL/dF, dL/dFc to 1e-4 of their largest magnitude and
    (dL/dv_r, dL/dv_b, dL/d v sin i) to 1e-3 relative, for a chi^2 seed
    against a model at other velocities and another v sin i."""
    pz, grid, inst, oinst, F, Fc = rot_setup
    F64, Fc64 = F.astype(np.float64), Fc.astype(np.float64)
    _, _, ymodel = I.forward(oinst, F64, Fc64, vr + 1.5, vb + 0.8, vsini=vs + 2.5)
    _, _, f = I.forward(oinst, F64, Fc64, vr, vb, vsini=vs)
    seed = (2.0 * (f - ymodel) / 1e-4).astype(np.float32)
    dF, dFc = torch.empty(grid.N, device="cuda"), torch.empty(grid.N, device="cuda")
    gv = torch.full((3,), np.nan, device="cuda")
    print("pz_inst_backward rotation", vr, vb, vs, flush=True)
    pz.pz_inst_backward(inst, _dev(F), _dev(Fc), _dev([vr, vb, vs]), _dev(seed), dF, dFc, gv)
    torch.cuda.synchronize()
    rdF, rdFc, rvr, rvb, rvs = I.adjoint(oinst, F64, Fc64, vr, vb, seed.astype(np.float64), vsini=vs)
    for got, ref in ((dF, rdF), (dFc, rdFc)):
        got = got.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref))
    g = gv.cpu().numpy()
    print("g_vel", g, "oracle", [rvr, rvb, rvs], flush=True)
    np.testing.assert_allclose(g, [rvr, rvb, rvs], rtol=1e-3)


def test_rotation_backward_deterministic(rot_setup):
    pz, grid, inst, oinst, F, Fc = rot_setup
    seed = _dev(np.random.default_rng(5).normal(size=inst.P))
    outs = []
    for _ in range(2):
        dF, dFc, gv = torch.empty(grid.N, device="cuda"), torch.empty(grid.N, device="cuda"), torch.empty(3, device="cuda")
        pz.pz_inst_backward(inst, _dev(F), _dev(Fc), _dev([5.0, 4.0, 21.0]), seed, dF, dFc, gv)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (dF, dFc, gv)])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("vrot_max,eps,vs", [(0.4, 0.0, 0.35), (12.0, 1.0, 11.5), (12.0, 0.0, -3.0)])
def test_rotation_edge_cases(setup, vrot_max, eps, vs):
    """A support of one cell (v sin i below a pixel), the two limb-darkening
    extremes (a uniform and a fully darkened disc) and a negative v sin i (the
    identity), forward and backward against the oracle."""
    pz, grid, _, _, F, Fc = setup
    lam, sig, vbmax = W.apogee_instrument(grid)
    inst = pz.Instrument(grid, lam, sig, vbmax, vrot_max_kms=vrot_max, limb_eps=eps)
    oinst = I.Instrument(grid, lam, sig, vbmax, vrot_max_kms=vrot_max, limb_eps=eps)
    F64, Fc64 = F.astype(np.float64), Fc.astype(np.float64)
    vr, vb = 3.0, 4.0
    f = torch.empty(inst.P, device="cuda")
    print("rotation edge case", vrot_max, eps, vs, "JR", oinst.JR, flush=True)
    pz.pz_inst_forward(inst, _dev(F), _dev(Fc), _dev([vr, vb, vs]), None, None, f)
    _, _, rf = I.forward(oinst, F64, Fc64, vr, vb, vsini=vs)
    np.testing.assert_allclose(f.cpu().numpy(), rf, rtol=1e-5)
    _, _, ym = I.forward(oinst, F64, Fc64, vr + 1.0, vb + 0.5, vsini=abs(vs) + 1.0)
    seed = (2.0 * (rf - ym) / 1e-4).astype(np.float32)
    dF = torch.empty(grid.N, device="cuda")
    gv = torch.full((3,), np.nan, device="cuda")
    pz.pz_inst_backward(inst, _dev(F), _dev(Fc), _dev([vr, vb, vs]), _dev(seed), dF, None, gv)
    torch.cuda.synchronize()
    rdF, _, rvr, rvb, rvs = I.adjoint(oinst, F64, Fc64, vr, vb, seed.astype(np.float64), vsini=vs)
    assert np.max(np.abs(dF.cpu().numpy() - rdF)) <= 1e-4 * np.max(np.abs(rdF))
    g = gv.cpu().numpy()
    np.testing.assert_allclose(g[:2], [rvr, rvb], rtol=1e-3)
    if vs <= 0.5 * I.C_KMS * oinst.h:              # the identity: no dependence on v sin i
        assert g[2] == 0.0 and rvs == 0.0
    else:
        assert abs(g[2] - rvs) <= 1e-3 * abs(rvs)
