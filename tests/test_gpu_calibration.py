"""Line calibration (Sec. 6, Eq. 30) on the GPU through the C ABI.

* pz_groups_expand / pz_groups_reduce: bit-exact against a gather and a
  sequential float32 sum in ascending line order (the documented order).
* pz_wmse_seed: loss and seed against the oracle's weighted mean square.
* The multi-standard objective (two stars, three spectra sharing one line
  list; group expansion, synthesis with damping-family corrections, the
  instrument operator, the weighted mean square and the whole reverse chain)
  against the oracle's objective and group gradient on a small catalogue.
* At the full 1500-1700 nm calibration size: the group gradient is the
  fixed-order sum of the line gradients, and it predicts the change of the
  objective along a descent direction.
* L-BFGS with the strong-Wolfe search recovers planted group corrections on a
  mock problem."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import calibration as OC
from oracle import instrument as I

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _seq_sums(q, G, x):
    out = np.zeros((x.shape[0], G), np.float32)
    for r in range(x.shape[0]):
        for l in range(q.size):                       # ascending line order, float32 adds
            if q[l] >= 0:
                out[r, q[l]] = np.float32(out[r, q[l]] + x[r, l])
    return out


@pytest.mark.parametrize("R", [1, 4])
def test_groups_expand_reduce_bitwise(gpu_lib, R):
    pz = gpu_lib
    rng = np.random.default_rng(R)
    L, G = 3001, 701
    q = rng.integers(-1, G, L).astype(np.int32)
    q[:G] = np.arange(G)                              # every group non-empty but the tail ragged
    q[G:G + 40] = -1
    groups = pz.Groups(q, G)
    xg = rng.normal(size=(R, G)).astype(np.float32)
    xl = torch.empty(R, L, device="cuda")
    print("pz_groups_expand R=%d" % R, flush=True)
    groups.expand(_dev(xg), xl)
    ref = np.where(q[None, :] >= 0, xg[:, np.maximum(q, 0)], 0.0).astype(np.float32)
    np.testing.assert_array_equal(xl.cpu().numpy(), ref)
    x = rng.normal(size=(R, L)).astype(np.float32)
    out = torch.empty(R, G, device="cuda")
    groups.reduce(_dev(x), out)
    s = _seq_sums(q, G, x)
    np.testing.assert_array_equal(out.cpu().numpy(), s)
    groups.reduce(_dev(x), out, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), (s + s).astype(np.float32))
    groups.destroy()


def test_groups_single_line_and_empty_group(gpu_lib):
    pz = gpu_lib
    groups = pz.Groups(np.array([1], np.int32), 3)     # groups 0 and 2 empty
    out = torch.full((1, 3), 7.0, device="cuda")
    groups.reduce(_dev([[2.5]]), out)
    xl = torch.empty(1, 1, device="cuda")
    groups.expand(_dev([[1.0, 2.0, 3.0]]), xl)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), [[0.0, 2.5, 0.0]])
    assert float(xl[0, 0]) == 2.0


def test_wmse_seed_vs_oracle(gpu_lib):
    pz = gpu_lib
    rng = np.random.default_rng(5)
    for P in (1, 1000, 26735):
        f = rng.normal(1.0, 0.1, P).astype(np.float32)
        y = (f + rng.normal(0.0, 0.01, P)).astype(np.float32)
        w = rng.uniform(0.0, 1.0, P).astype(np.float32)
        c = 1.0 / P
        ref_l, ref_g = OC.weighted_mse(f, y, w, c)
        g = torch.empty(P, device="cuda")
        loss = torch.full((1,), 0.25, device="cuda")
        print("pz_wmse_seed P=%d" % P, flush=True)
        pz.pz_wmse_seed(_dev(f), _dev(y), _dev(w), c, g, loss)
        torch.cuda.synchronize()
        np.testing.assert_allclose(g.cpu().numpy(), ref_g, rtol=1e-6, atol=1e-12 * np.max(np.abs(ref_g)))
        np.testing.assert_allclose(float(loss[0]), ref_l, rtol=1e-5)
        pz.pz_wmse_seed(_dev(f), _dev(y), None, c, None, loss, accumulate=True)
        torch.cuda.synchronize()
        np.testing.assert_allclose(float(loss[0]), ref_l + OC.weighted_mse(f, y, np.ones(P), c)[0], rtol=1e-5)


def _unit_residual_scale(stds, q, G, theta):
    """Group sums of the absolute gradient terms for a unit model error on every
    observed pixel (seed |2 c w| through the instrument adjoint): a model error
    eps_f in f moves each group gradient by at most eps_f times this."""
    from oracle import synth as O
    tot = np.zeros((4, G))
    for st in stds:
        par = OC._params(st, q, theta)
        F, Fc = O.synthesize(st.wl, par)
        dF = I.adjoint(st.inst, F, Fc, *st.vel, 2.0 * st.c * st.w)[0]
        r = O.adjoint(st.wl, par, np.abs(dF), conditions=True)
        tot += OC.group_sums(q, G, np.vstack([r["abs_loggf"], r["abs_damp_family"]]))
    return tot


EPS_F = 1e-5     # float32 model error in f, the bound of the forward and instrument parity tests


def test_objective_and_gradient_vs_oracle(gpu_lib):
    """Two stars (a dwarf and a giant observed at two epochs) share 46 lines;
    loss to 1e-4 relative; group gradients to the 1e-3 rule (1e-3 relative
    where |g| >= 1e-2 max, else 1e-5 max) or, for ill-conditioned groups only,
    1e-3 relative plus 1e-5 of the sum of absolute contributions plus the
    propagated float32 model error
    EPS_F (the seed 2 c w (f - y) carries it where f - y is small, and a weak
    group's gradient is a sum of noise residuals of either sign)."""
    from paper_2607_24141_amd import calibrate as CAL
    from test_gpu_adjoint import grad_close_cond
    cal = W.calibration_tiny(seed=31, n_records=40, N=2500, D=24)
    q, G = OC.correction_groups(cal.lines.lam0_nm, cal.lines.E_eV, cal.lines.species, cal.lines.ion,
                                cal.lines.loggf, 2.0 * OC.CM1_EV, 0.035, active=cal.active)
    truth = W.calibration_truth(np.random.default_rng(3), G)
    theta = 0.5 * W.calibration_truth(np.random.default_rng(4), G)
    rng = np.random.default_rng(5)
    stds = []
    for s in cal.standards:
        inst = I.Instrument(s.wl.grid, s.lam_obs_nm, s.lsf_sigma_ln, s.vb_max_kms)
        st = OC.Standard(s.wl, inst, s.vel, np.zeros(s.lam_obs_nm.size), s.w, s.c)
        st.y = (OC.model(st, q, truth) + rng.normal(0.0, 0.002, s.lam_obs_nm.size)).astype(np.float32)
        stds.append(st)
    theta32 = theta.astype(np.float32)
    ref_loss, ref_g, ref_abs = OC.objective(stds, q, G, theta32.astype(np.float64))
    print("calibration objective G=%d" % G, flush=True)
    gc = CAL.Calibration(cal, y=[s.y for s in stds], groups=(q.astype(np.int32), G))
    assert len(gc.stars) == 2 and len(gc.epochs) == 3
    loss, grad = gc.evaluate(_dev(theta32))
    torch.cuda.synchronize()
    np.testing.assert_allclose(float(loss[0]), ref_loss, rtol=1e-4)
    g = grad.cpu().numpy().astype(np.float64)
    unit = _unit_residual_scale(stds, q, G, theta32.astype(np.float64))
    from test_gpu_adjoint import TERM_TOL
    for r, kind in enumerate(CAL.KINDS):
        grad_close_cond(g[r], ref_g[r], ref_abs[r] + EPS_F / TERM_TOL * unit[r], rtol=1e-3, name=kind,
                        cond_fallback=True)
    # strong groups (the 25 % largest gradients) hold to 1e-3 relative alone
    big = np.abs(ref_g) >= np.quantile(np.abs(ref_g), 0.75)
    assert np.all(np.abs(g - ref_g)[big] <= 1e-3 * np.abs(ref_g)[big])
    # the autograd wrapper returns the same value and gradient
    t = _dev(theta32).requires_grad_(True)
    val = CAL.loss_fn(gc, t)
    val.backward()
    np.testing.assert_array_equal(t.grad.cpu().numpy(), g.astype(np.float32))


@pytest.fixture(scope="module")
def full_calibration(gpu_lib):
    from paper_2607_24141_amd import calibrate as CAL
    cal = W.calibration()
    print("full calibration: grouping + plans", flush=True)
    gc = CAL.Calibration(cal)
    return cal, gc


def test_full_size_group_gradient_is_fixed_order_line_sum(full_calibration):
    cal, gc = full_calibration
    assert gc.L == 60_886 and gc.G == 25_147
    theta = _dev(0.3 * W.calibration_truth(np.random.default_rng(1), gc.G))
    ys = gc.model(_dev(W.calibration_truth(np.random.default_rng(2), gc.G)))
    gc.set_observed(ys)
    print("full calibration: evaluate", flush=True)
    loss, grad = gc.evaluate(theta)
    torch.cuda.synchronize()
    assert np.isfinite(float(loss[0])) and float(loss[0]) > 0.0
    # the last star's line gradients, reduced alone, in the documented order
    last = torch.empty(4, gc.G, device="cuda")
    gc.groups.reduce(gc.GL, last)
    torch.cuda.synchronize()
    sample = np.random.default_rng(3).choice(gc.G, 400, replace=False)
    GL = gc.GL.cpu().numpy()
    members = {g: np.flatnonzero(gc.q == g) for g in sample}
    lg = last.cpu().numpy()
    for g in sample:
        for r in range(4):
            a = np.float32(0.0)
            for l in members[g]:
                a = np.float32(a + GL[r, l])
            assert lg[r, g] == a
    # band lines have no group: their expanded corrections are zero
    assert np.all(gc.X[:, ~torch.as_tensor(cal.active, device="cuda")].cpu().numpy() == 0.0)


def test_full_size_gradient_predicts_descent(full_calibration):
    cal, gc = full_calibration
    theta = _dev(0.3 * W.calibration_truth(np.random.default_rng(1), gc.G))
    gc.set_observed(gc.model(_dev(W.calibration_truth(np.random.default_rng(2), gc.G))))
    loss, grad = gc.evaluate(theta)
    l0, g = float(loss[0]), grad.clone()
    d = -g / torch.linalg.vector_norm(g)
    slope = float((g * d).sum())
    for eps in (3e-3, 1e-2):
        lp = float(gc.evaluate(theta + eps * d)[0][0])
        lm = float(gc.evaluate(theta - eps * d)[0][0])
        fd = (lp - lm) / (2 * eps)
        print("directional derivative eps=%g fd=%.6e adjoint=%.6e" % (eps, fd, slope), flush=True)
        assert abs(fd - slope) <= 0.03 * abs(slope)
    assert lp < l0 < lm


def test_lbfgs_recovers_planted_corrections(gpu_lib):
    """Mock data at planted corrections plus noise sigma: L-BFGS from zero
    reaches the noise floor (E L(truth) = sigma^2: each spectrum's c w sum to
    its share of 1) and recovers log gf where the data constrain it: groups
    whose Fisher information (from finite differences of the model) gives a
    standard error below 0.01 dex."""
    from paper_2607_24141_amd import calibrate as CAL
    sigma = 1e-3
    cal = W.calibration_tiny(seed=41, n_records=300, N=12000, D=72)
    gc = CAL.Calibration(cal)
    truth = W.calibration_truth(np.random.default_rng(6), gc.G)
    gc.set_observed(CAL.mock_observed(gc, truth, sigma, seed=7))
    print("L-BFGS G=%d" % gc.G, flush=True)
    r = CAL.fit(gc, max_iter=40)
    print("loss %.4e -> %.4e in %d iterations, %d evaluations, %.2f s" % (r["loss0"], r["loss"], r["iters"],
                                                                          r["evals"], r["seconds"]), flush=True)
    assert r["loss0"] > 20 * sigma ** 2 and r["loss"] < 1.2 * sigma ** 2
    # Fisher information of each group's log gf correction
    h = 0.02
    tt = _dev(truth)
    base = [f.clone() for f in gc.model(tt)]
    fisher = np.zeros(gc.G)
    for g in range(gc.G):
        tp = tt.clone()
        tp[0, g] += h
        for e, f0, f1 in zip(gc.epochs, base, gc.model(tp)):
            fisher[g] += float((e.w * ((f1 - f0) / h) ** 2).sum()) / sigma ** 2
    good = fisher > 1.0 / 0.01 ** 2
    th = r["theta"].cpu().numpy()
    err = np.abs(th[0] - truth[0])
    c = CAL.correlation(th[0][good], truth[0][good])
    print("constrained groups %d of %d: log gf correlation %.4f, median |error| %.4f dex, all groups %.3f"
          % (good.sum(), gc.G, c, np.median(err[good]), CAL.correlation(th[0], truth[0])), flush=True)
    assert good.sum() >= 30
    assert c > 0.8 and np.median(err[good]) < 0.02
