"""Pins of the scattering-transfer oracle (Sec. 2.1, Eqs. 3 and 6-8): without
scattering it is the plain transfer; its mean-intensity operator is exact on a
constant and on a linear source function (closed forms of the formal
solution); the matrix and the sweeps agree; the fixed point satisfies its
equation; an isothermal atmosphere with constant eps approaches the sqrt(eps)
law S(0) = sqrt(eps) B at second order in the depth spacing; the
complex-step gradient agrees with real central differences."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import scatter as SC
from oracle import synth as O


def _tau(D=40, n=3):
    return np.logspace(-4, 2, D)[:, None] * np.linspace(0.7, 1.3, n)[None, :]


def test_no_scattering_is_the_plain_transfer():
    wl = W.tiny(seed=3, L=20, N=300, D=30, S=4, n_molecular=1)
    F0, Fc0 = O.synthesize(wl)
    F1, Fc1 = SC.synthesize(wl)
    np.testing.assert_allclose(F1, F0, rtol=1e-13)
    np.testing.assert_allclose(Fc1, Fc0, rtol=1e-13)


def test_mean_intensity_constant_and_linear_source():
    tau = _tau()
    J = SC.mean_intensity(2.0 * np.ones_like(tau), tau)
    ref = 2.0 * (1.0 - 0.5 * sum(w * np.exp(-tau / mu) for mu, w in zip(O.GAUSS3_MU, O.GAUSS3_W)))
    np.testing.assert_allclose(J, ref, rtol=1e-13)
    a, b = 1.3, 0.7
    J = SC.mean_intensity(a + b * tau, tau)
    # I+ = a + b (tau + mu), I- = a + b tau - b mu + (b mu - a) exp(-tau/mu)
    ref = a + b * tau + 0.5 * sum(w * (b * mu - a) * np.exp(-tau / mu) for mu, w in zip(O.GAUSS3_MU, O.GAUSS3_W))
    np.testing.assert_allclose(J, ref, rtol=1e-13)


def test_lambda_matrix_equals_sweeps_and_emergent_flux():
    tau = _tau()
    S = np.random.default_rng(1).uniform(1.0, 2.0, tau.shape)
    Lam = SC.lambda_matrix(tau)
    np.testing.assert_allclose(np.einsum("nij,jn->in", Lam, S), SC.mean_intensity(S, tau), rtol=1e-13)
    np.testing.assert_allclose(SC.emergent_flux(S, tau), O.flux_gauss3(S, tau), rtol=1e-13)


def test_fixed_point_equation():
    tau = _tau()
    rng = np.random.default_rng(2)
    eps = rng.uniform(0.05, 1.0, tau.shape)
    B = rng.uniform(1.0, 3.0, tau.shape)
    S = SC.source_function(eps, B, tau)
    np.testing.assert_allclose(S, eps * B + (1.0 - eps) * SC.mean_intensity(S, tau), rtol=1e-12)


def test_sqrt_eps_law():
    errs = []
    for D in (200, 400, 800):
        tau = np.logspace(-6, 4, D)[:, None]
        S = SC.source_function(np.full_like(tau, 0.01), np.ones_like(tau), tau)
        errs.append(abs(S[0, 0] / 0.1 - 1.0))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0     # second order in the spacing


def test_complex_step_matches_central_differences():
    wl = W.tiny(seed=4, L=12, N=120, D=16, S=4, n_molecular=1)
    wl.atm = copy.deepcopy(wl.atm)
    wl.atm.sigma_c = np.full(wl.atm.D, 0.8)
    wl.atm.sigma_alpha = -1.0
    kl = O.line_opacity(wl)
    seed = np.random.default_rng(3).normal(size=wl.grid.N)
    g = SC.opacity_adjoint(wl, kl, seed)
    h = 1e-4                                         # relative step: truncation ~1e-8, rounding below
    for j, i in ((0, 10), (5, 60), (15, 100)):
        kp, km = kl.copy(), kl.copy()
        d = h * max(kl[j, i], 1e-3)
        kp[j, i] += d
        km[j, i] -= d
        fd = seed @ (SC.flux_from_opacity(wl, kp)[0] - SC.flux_from_opacity(wl, km)[0]) / (2 * d)
        assert abs(fd - g[j, i]) <= 1e-6 * abs(g[j, i]) + 1e-9 * np.max(np.abs(g))


def test_more_scattering_lowers_the_continuum():
    """More scattering at fixed absorption lowers the surface source function
    (photons escape), so the emergent continuum flux drops."""
    wl = W.tiny(seed=5, L=1, N=50, D=40, S=3)
    wl.atm = copy.deepcopy(wl.atm)
    fluxes = []
    for s in (0.0, 0.5, 2.0):
        wl.atm.sigma_c = np.full(wl.atm.D, s)
        fluxes.append(SC.synthesize(wl)[1])
    assert np.all(fluxes[1] < fluxes[0]) and np.all(fluxes[2] < fluxes[1])
