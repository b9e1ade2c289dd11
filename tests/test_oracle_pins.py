"""Pins of the FP64 oracle against closed forms, limits, brute force and
independent physical constants (no GPU).  Each test names the passage it pins.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc
from scipy import integrate
from numpy.polynomial.legendre import leggauss
from scipy.special import expn

import workloads as W
from oracle import synth as O


# --------------------------------------------------------------------- Voigt profile
@pytest.mark.parametrize("a,v", [(1e-4, 0.3), (1e-3, 2.5), (0.05, 4.0), (0.3, 1.0),
                                 (1.0, 6.0), (2.0, 0.0), (0.01, 12.0)])
def test_voigt_is_convolution_integral(a, v):
    """H(a, v) = (a/pi) int exp(-t^2) / ((v - t)^2 + a^2) dt (the Voigt profile, Sec. 2.1)."""
    f = lambda t: math.exp(-t * t) / ((v - t) ** 2 + a * a)
    pts = [v] if abs(v) < 8 else None
    val, _ = integrate.quad(f, -12, 12, points=pts, limit=800, epsabs=0, epsrel=1e-12)
    # Lorentzian tails outside |t| < 12 are below 1e-60 relative and ignored
    ref = a / math.pi * val
    assert abs(O.voigt(a, v) - ref) <= 1e-9 * ref


def test_voigt_gaussian_limit():
    """a = 0 reduces the Voigt profile to the Doppler Gaussian exp(-v^2)."""
    v = np.linspace(-5, 5, 101)
    np.testing.assert_allclose(O.voigt(0.0, v), np.exp(-v * v), rtol=1e-13, atol=1e-300)


def test_voigt_line_center():
    """v = 0: H(a, 0) = exp(a^2) erfc(a) (computed with libm's erfc)."""
    for a in (1e-5, 1e-3, 0.1, 0.5, 1.0, 3.0):
        ref = math.exp(a * a) * math.erfc(a)
        assert abs(O.voigt(a, 0.0) - ref) <= 1e-12 * ref


def test_voigt_lorentz_wings():
    """|v| >> 1: H -> a / (sqrt(pi) v^2) (1 + 3/(2 v^2) + ...); large a: a/(sqrt(pi)(a^2+v^2))."""
    for a in (1e-4, 1e-2, 0.3):
        for v in (50.0, 200.0, 1000.0):
            H = O.voigt(a, v)
            lor = a / (math.sqrt(math.pi) * v * v)
            assert abs(H / lor - 1.0) < 2.0 / v ** 2
    a, v = 200.0, 3.0
    assert abs(O.voigt(a, v) / (a / (math.sqrt(math.pi) * (a * a + v * v))) - 1) < 1e-4


@pytest.mark.parametrize("a", [1e-3, 0.05, 0.5])
def test_voigt_normalisation(a):
    """int_{-V}^{V} H dv = sqrt(pi) (1 - 2a/(pi V) + O(V^-3)): phi integrates to one (Eq. 4)."""
    V = 400.0
    v = np.concatenate([np.linspace(0, 10, 200001), np.linspace(10, V, 400001)[1:]])
    H = O.voigt(a, v)
    integral = 2 * integrate.simpson(H, x=v)
    expect = math.sqrt(math.pi) * (1 - 2 * a / (math.pi * V))
    assert abs(integral - expect) < 1e-7 * expect


def test_voigt_derivative_identities():
    """dH/dv = -2(vH - aL), dH/da = 2(vL + aH) - 2/sqrt(pi) (from w' = -2 z w + 2i/sqrt(pi))."""
    rng = np.random.default_rng(1)
    a = 10 ** rng.uniform(-4, 0.5, 200)
    v = rng.uniform(-20, 20, 200)
    H, L = O.voigt_w(a, v)
    h = 1e-6
    Hv_fd = (O.voigt(a, v + h) - O.voigt(a, v - h)) / (2 * h)
    Ha_fd = (O.voigt(a + h * a, v) - O.voigt(a - h * a, v)) / (2 * h * a)
    np.testing.assert_allclose(-2 * (v * H - a * L), Hv_fd, rtol=2e-6, atol=1e-12)
    np.testing.assert_allclose(2 * (v * L + a * H) - 2 / math.sqrt(math.pi), Ha_fd, rtol=2e-6, atol=1e-11)


# ------------------------------------------------------------------------ populations
def _atm_one(T, ne, chi, U1, U2):
    D = len(T)
    return W.Atmosphere(T=np.asarray(T, float), m=np.linspace(1, 2, D), ne=np.asarray(ne, float),
                        npert=np.ones(D), rho=np.ones(D), n_species=np.ones((1, D)),
                        chi_ion_eV=np.array([chi]), U=np.array([[[U1] * D, [U2] * D]], float),
                        mass_amu=np.array([1.0]))


def test_saha_against_si_constants():
    """Eq. 11 evaluated independently in SI units with scipy.constants (hydrogen-like case)."""
    T, ne_cgs, chi, U1, U2 = 9000.0, 3e13, 13.6, 2.0, 1.0
    f = O.ion_fractions(_atm_one([T], [ne_cgs], chi, U1, U2))[0, :, 0]
    lam_th = sc.h / math.sqrt(2 * math.pi * sc.m_e * sc.k * T)      # thermal de Broglie, m
    ratio = 2 * U2 / U1 / lam_th ** 3 * math.exp(-chi * sc.e / (sc.k * T)) / (ne_cgs * 1e6)
    assert abs(f[1] / f[0] / ratio - 1) < 1e-8
    assert abs(f.sum() - 1) < 1e-15


def test_saha_scalings_and_molecules():
    """Phi proportional to T^{3/2} exp(-chi/kT)/n_e; infinite chi => one stage."""
    f1 = O.ion_fractions(_atm_one([6000.0, 6000.0], [1e12, 2e12], 7.0, 3.0, 5.0))
    phi = f1[0, 1] / f1[0, 0]
    assert abs(phi[0] / phi[1] - 2.0) < 1e-12
    fm = O.ion_fractions(_atm_one([6000.0], [1e12], np.inf, 3.0, 5.0))
    assert fm[0, 0, 0] == 1.0 and fm[0, 1, 0] == 0.0


# ----------------------------------------------------------------- source and transfer
def test_planck_stefan_boltzmann_and_wien():
    """B_lambda per nm: pi int B dlambda = sigma T^4 and the Wien peak (scipy.constants)."""
    T = 5777.0
    lam = np.geomspace(50.0, 2e6, 400001)          # nm
    B = O.planck_lambda_per_nm(lam, [T])[0]          # erg s^-1 cm^-2 sr^-1 nm^-1
    total = math.pi * integrate.simpson(B, x=lam)    # erg s^-1 cm^-2
    sigma_cgs = sc.Stefan_Boltzmann * 1e3
    assert abs(total / (sigma_cgs * T ** 4) - 1) < 1e-6
    lam_peak = sc.Wien / T * 1e9
    fine = np.linspace(lam_peak * 0.99, lam_peak * 1.01, 20001)
    Bf = O.planck_lambda_per_nm(fine, [T])[0]
    assert abs(fine[np.argmax(Bf)] / lam_peak - 1) < 2e-6


def test_tau_scan_exact_cases():
    """d tau = chi dm with the trapezoid rule: exact for chi constant or linear in m."""
    m = np.geomspace(1e-3, 10, 72)
    chi = np.full((72, 3), 2.5)
    np.testing.assert_allclose(O.optical_depth(chi, m), 2.5 * m[:, None] * np.ones((1, 3)), rtol=1e-14)
    c0, c1 = 0.7, 3.0
    chi = (c0 + c1 * m)[:, None]
    tau = O.optical_depth(chi, m)[:, 0]
    # tau(m) = tau_0 + int_{m0}^{m} chi dm with tau_0 = chi_0 m_0
    ref = chi[0, 0] * m[0] + c0 * (m - m[0]) + 0.5 * c1 * (m ** 2 - m[0] ** 2)
    np.testing.assert_allclose(tau, ref, rtol=1e-13)


@pytest.mark.parametrize("quad", ["gauss3", "e2"])
def test_linear_source_flux(quad):
    """S = a + b tau => F = pi (a + 2b/3) exactly (Eqs. 7-8)."""
    tau = np.geomspace(1e-4, 50.0, 72)[:, None] * np.array([1.0, 3.0])[None, :]
    a, b = 2.0, 3.0
    S = a + b * tau
    F = O.emergent_flux(S, tau, quad)
    np.testing.assert_allclose(F, math.pi * (a + 2 * b / 3), rtol=1e-12)


def test_milne_eddington_ratio():
    """Line opacity eta times a grey continuum with S linear in tau_c:
    F/F_c = (a + 2b/(3(1+eta))) / (a + 2b/3)."""
    tc = np.geomspace(1e-4, 60.0, 72)[:, None] * np.ones((1, 4))
    eta = np.array([0.0, 0.3, 5.0, 300.0])[None, :]
    a, b = 1.0, 2.5
    S = a + b * tc
    for quad in ("gauss3", "e2"):
        ratio = O.emergent_flux(S, tc * (1 + eta), quad) / O.emergent_flux(S, tc, quad)
        expect = (a + 2 * b / (3 * (1 + eta[0]))) / (a + 2 * b / 3)
        np.testing.assert_allclose(ratio, expect, rtol=1e-11)


def test_e2_equals_angle_integral():
    """F = 2 pi int_0^1 I(0,mu) mu dmu; Gauss-Legendre with many angles converges to the E2 form."""
    tau = np.geomspace(1e-3, 30.0, 72)[:, None]
    S = np.exp(-1.0 / (0.3 + tau)) + 0.2 * np.sqrt(tau)   # curved source
    x, w = leggauss(64)
    mu, w = 0.5 * (x + 1), 0.5 * w
    F = sum(2 * math.pi * wk * mk * O.intensity_surface(S, tau, mk) for mk, wk in zip(mu, w))
    np.testing.assert_allclose(O.flux_e2(S, tau), F, rtol=1e-9)
    # Gauss-3 is a different (coarser) angular rule: close but not identical
    g3 = O.flux_gauss3(S, tau)
    assert 1e-7 < abs(g3[0] / F[0] - 1) < 1e-2


# Shallow atmospheres: at tau_max of order one the lower boundary carries a
# large share of the flux (the diffusion intensity I = S + mu dS/dtau behind
# the last layer for Gauss-3, the tail S_D E3(tau_D) + s_D E4(tau_D) of the E2
# form), so every closed form below also pins those terms (Eqs. 7-8).
SHALLOW = (0.3, 2.0)


def _shallow_tau(tau_max, cols=1):
    return np.geomspace(1e-4 * tau_max, tau_max, 72)[:, None] * np.linspace(1.0, 0.5, cols)[None, :]


@pytest.mark.parametrize("quad", ["gauss3", "e2"])
@pytest.mark.parametrize("tau_max", SHALLOW)
def test_linear_source_flux_shallow(quad, tau_max):
    """S = a + b tau through a slab of depth tau_max ~ 1: still F = pi (a + 2b/3) exactly.

    The semi-infinite linear atmosphere gives I(0, mu) = a + b mu; the diffusion
    boundary continues S linearly below the last layer, so any depth of slab
    reproduces it.  The boundary term is checked to carry a large share of the
    flux, so a dropped or mis-signed term (or a missing mu) fails the test."""
    tau = _shallow_tau(tau_max, 3)
    a, b = 2.0, 3.0
    S = a + b * tau
    F = O.emergent_flux(S, tau, quad)
    np.testing.assert_allclose(F, math.pi * (a + 2 * b / 3), rtol=1e-12)
    tD = tau[-1]
    bottom = 2 * math.pi * (S[-1] * expn(3, tD) + b * expn(4, tD))
    assert np.all(bottom / F > 0.05), bottom / F


@pytest.mark.parametrize("tau_max", SHALLOW)
def test_milne_eddington_ratio_shallow(tau_max):
    """The Milne-Eddington ratio with the continuum slab only tau_max deep."""
    tc = _shallow_tau(tau_max) * np.ones((1, 4))
    eta = np.array([0.0, 0.3, 5.0, 300.0])[None, :]
    a, b = 1.0, 2.5
    S = a + b * tc
    for quad in ("gauss3", "e2"):
        ratio = O.emergent_flux(S, tc * (1 + eta), quad) / O.emergent_flux(S, tc, quad)
        expect = (a + 2 * b / (3 * (1 + eta[0]))) / (a + 2 * b / 3)
        np.testing.assert_allclose(ratio, expect, rtol=1e-11)


@pytest.mark.parametrize("tau_max", SHALLOW)
def test_e2_equals_angle_integral_shallow(tau_max):
    """A curved source in a shallow slab: the E2 form (with its E3/E4 tail) equals
    the 64-angle integral of I(0, mu), whose rays start from the diffusion
    intensity S_D + mu s_D at the bottom."""
    tau = _shallow_tau(tau_max, 2)
    S = np.exp(-1.0 / (0.3 + tau)) + 0.2 * np.sqrt(tau) + 0.7 * tau ** 2
    x, w = leggauss(64)
    mu, w = 0.5 * (x + 1), 0.5 * w
    F = sum(2 * math.pi * wk * mk * O.intensity_surface(S, tau, mk) for mk, wk in zip(mu, w))
    np.testing.assert_allclose(O.flux_e2(S, tau), F, rtol=1e-9)


@pytest.mark.parametrize("tau_max", SHALLOW)
@pytest.mark.parametrize("mu", [0.05, 0.1127016653792583, 0.5, 0.8872983346207417, 1.0])
def test_intensity_is_the_formal_integral_shallow(tau_max, mu):
    """I(0, mu) from the layer recursion equals the formal solution of Eq. 7
    written as one integral, I = int_0^tau_D S(t) e^{-t/mu} dt/mu +
    (S_D + mu s_D) e^{-tau_D/mu}, with S piecewise linear in tau (extended
    linearly to tau = 0), integrated by adaptive quadrature segment by segment."""
    tau = _shallow_tau(tau_max)[:, 0]
    S = 1.0 + np.sin(3.0 * tau / tau_max) + 0.4 * (tau / tau_max) ** 2
    knots_t = np.concatenate([[0.0], tau])
    S0 = S[0] - tau[0] * (S[1] - S[0]) / (tau[1] - tau[0])
    knots_S = np.concatenate([[S0], S])
    total = 0.0
    for k in range(len(knots_t) - 1):
        ta, tb, Sa, Sb = knots_t[k], knots_t[k + 1], knots_S[k], knots_S[k + 1]
        f = lambda t: (Sa + (Sb - Sa) * (t - ta) / (tb - ta)) * math.exp(-t / mu) / mu
        val, _ = integrate.quad(f, ta, tb, epsabs=0, epsrel=1e-13)
        total += val
    sD = (S[-1] - S[-2]) / (tau[-1] - tau[-2])
    total += (S[-1] + mu * sD) * math.exp(-tau[-1] / mu)
    got = float(O.intensity_surface(S[:, None], tau[:, None], mu)[0])
    assert abs(got / total - 1) < 1e-12, (got, total)


def test_lin_weight_series_matches_direct():
    x = np.geomspace(1e-8, 40, 2001)
    xd = x[x > 0.06]
    direct = (1 - (1 + xd) * np.exp(-xd)) / xd
    np.testing.assert_allclose(O.lin_weight(xd), direct, rtol=1e-14)
    # small x: the direct formula evaluated with 60-digit decimal arithmetic
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    for xx in (1e-8, 3.3e-5, 1e-3, 0.02, 0.0499):
        X = Decimal(xx)
        ref = (1 - (1 + X) * (-X).exp()) / X
        assert abs(O.lin_weight(np.array(xx)) / float(ref) - 1) < 1e-14
    h = 1e-7
    for xx in (1e-3, 0.0499, 0.051, 0.5, 5.0):
        fd = (O.lin_weight(np.array(xx + h)) - O.lin_weight(np.array(xx - h))) / (2 * h)
        assert abs(O._lin_weight_deriv(np.array(xx)) - fd) < 1e-7


# --------------------------------------------------------------------- grid / continuum
def test_grid_and_sizes():
    """Eq. 1 ratio and the Eq. 2 sample counts of the three wavelength windows."""
    g = W.grid_for(500.0, 503.0, 3e5)
    lam = O.wavelengths_nm(g)
    np.testing.assert_allclose(lam[1:] / lam[:-1], 1 + 1 / 3e5, rtol=1e-14)
    assert (g.N, W.grid_for(1500.0, 1700.0, 3e5).N, W.grid_for(300.0, 1000.0, 3e5).N) == (1795, 37550, 361193)
    assert lam[-1] <= 503.0 < lam[-1] * (1 + 1 / 3e5)


def test_continuum_power_law():
    wl = W.tiny()
    wl.atm.lam_ref_nm = O.wavelengths_nm(wl.grid, [10])[0]
    kc = O.continuum_opacity(wl, [10, 20])
    assert abs(kc[0] - wl.atm.kappa0) < 1e-15
    r = O.wavelengths_nm(wl.grid, [20])[0] / wl.atm.lam_ref_nm
    assert abs(kc[1] - r ** wl.atm.alpha) < 1e-15


# ---------------------------------------------------------------------- line opacity
def _brute_opacity(wl, params, window=None):
    """Every (pixel, line, depth) triple with explicit loops over lines (no pair search)."""
    lam = O.wavelengths_nm(wl.grid)
    nu = sc.c * 100 / (lam * 1e-7)
    out = np.zeros((wl.atm.D, wl.grid.N))
    for l in range(wl.lines.L):
        one = wl.lines.take([l])
        lp = O.line_depth_params(wl.atm, one, params.dgf[[l]], params.ddamp[[l]], params.dA, params.xi_kms)
        v = (nu[None, :] - lp["nu_l"][0]) / lp["dnu"][0][:, None]
        k = lp["s"][0][:, None] * O.voigt(lp["a"][0][:, None], v) / (math.sqrt(math.pi) * lp["dnu"][0][:, None])
        if window is not None:
            k = k * (np.abs(lam - wl.lines.lam0_nm[l]) <= window)[None, :]
        out += k
    return out


def test_windowed_equals_brute_force():
    """Windowing: with W covering the grid the windowed sum is the unwindowed sum;
    otherwise it equals the brute-force sum masked to |lambda_i - lambda_l| <= W."""
    wl = W.tiny(seed=3, L=15, N=600, D=6)
    wl.params = W.random_params(np.random.default_rng(0), wl.lines.L, wl.atm.S, 1.3)
    wide = W.tiny(seed=3, L=15, N=600, D=6, window_nm=50.0)
    wide.params = wl.params
    np.testing.assert_allclose(O.line_opacity(wide), _brute_opacity(wide, wide.params), rtol=1e-12)
    np.testing.assert_allclose(O.line_opacity(wl), _brute_opacity(wl, wl.params, wl.window_nm), rtol=1e-12)
    out_of_window = _brute_opacity(wl, wl.params) - O.line_opacity(wl)
    assert np.all(out_of_window >= -1e-30) and out_of_window.max() > 0


def test_line_integrated_strength():
    """Eq. 4: the profile integrates to one, so sum_i kappa_i dnu_i recovers the
    frequency-integrated strength (pi e^2/m_e c) n/(rho U) gf e^{-E/kT}(1-e^{-h nu/kT})."""
    wl = W.tiny(seed=5, L=1, N=40001, D=3, R=3e6, window_nm=5.0)
    wl.lines.lam0_nm[:] = O.wavelengths_nm(wl.grid, [20000])[0] + 1e-6
    wl.lines.log_grad[:] = 7.0
    wl.lines.log_gstark[:] = -9.0
    wl.lines.log_gvdw[:] = -12.0
    k = O.line_opacity(wl)
    lam = O.wavelengths_nm(wl.grid)
    nu = sc.c * 100 / (lam * 1e-7)
    dnu = -np.gradient(nu)
    integral = (k * dnu[None, :]).sum(axis=1)
    # independent strength: SI constants, f from the same species/ion population
    ln = wl.lines
    sp, r = ln.species[0], ln.ion[0]
    f = O.ion_fractions(wl.atm)[sp, r]
    n = wl.atm.n_species[sp] * f
    T = wl.atm.T
    e_cgs = sc.e * sc.c * 10          # esu
    const = math.pi * e_cgs ** 2 / (sc.m_e * 1e3 * sc.c * 100)
    nu0 = sc.c / (ln.lam0_nm[0] * 1e-9)
    strength = const * n / (wl.atm.rho * wl.atm.U[sp, r]) * 10 ** ln.loggf[0] * \
        np.exp(-ln.E_eV[0] * sc.e / (sc.k * T)) * (1 - np.exp(-sc.h * nu0 / (sc.k * T)))
    lp = O.line_depth_params(wl.atm, ln, [0.0], [0.0], wl.params.dA, wl.params.xi_kms)
    V = 5.0 / (ln.lam0_nm[0]) * nu0 / lp["dnu"][0]          # window half-width in Doppler units
    trunc = 1 - 2 * lp["a"][0] / (math.pi * V)               # Lorentz wings beyond the window
    np.testing.assert_allclose(integral, strength * trunc, rtol=2e-6)


def test_doppler_width_second_moment():
    """Pure Doppler profile (negligible damping): <(nu - nu_l)^2> = dnu_D^2 / 2 with
    dnu_D = (nu_l/c) sqrt(2 k T / m + xi^2) (Eq. 5), constants from scipy.constants."""
    wl = W.tiny(seed=9, L=1, N=4001, D=2, R=3e6, window_nm=0.5, xi=1.7)
    wl.lines.lam0_nm[:] = O.wavelengths_nm(wl.grid, [2000])[0]
    wl.lines.log_grad[:] = 1.0
    wl.lines.log_gstark[:] = -20.0
    wl.lines.log_gvdw[:] = -20.0
    k = O.line_opacity(wl)
    lam = O.wavelengths_nm(wl.grid)
    nu = sc.c / (lam * 1e-9)
    dnu = -np.gradient(nu)
    nu0 = sc.c / (wl.lines.lam0_nm[0] * 1e-9)
    m = wl.atm.mass_amu[wl.lines.species[0]] * sc.atomic_mass
    for j in range(2):
        w = k[j] * dnu
        var = np.sum(w * (nu - nu0) ** 2) / np.sum(w)
        dv2 = 2 * sc.k * wl.atm.T[j] / m + (1.7e3) ** 2
        assert abs(var / (0.5 * (nu0 / sc.c) ** 2 * dv2) - 1) < 1e-5


# ------------------------------------------------------------------------- structure
def test_empty_catalog_total_equals_continuum():
    wl = W.tiny(L=0)
    F, Fc = O.synthesize(wl)
    np.testing.assert_array_equal(F, Fc)


def test_linearity_and_permutation():
    wl = W.tiny(seed=11, L=20, N=300)
    k_all = O.line_opacity(wl)
    idx = np.random.default_rng(2).permutation(20)
    wl_p = W.Workload(wl.name, wl.grid, wl.atm, wl.lines.take(idx), wl.params, wl.window_nm)
    wl_p.params = W.zero_params(20, wl.atm.S, wl.params.xi_kms)
    np.testing.assert_allclose(O.line_opacity(wl_p), k_all, rtol=1e-13)
    a = W.Workload(wl.name, wl.grid, wl.atm, wl.lines.take(np.arange(0, 9)), W.zero_params(9, wl.atm.S, 1.0), wl.window_nm)
    b = W.Workload(wl.name, wl.grid, wl.atm, wl.lines.take(np.arange(9, 20)), W.zero_params(11, wl.atm.S, 1.0), wl.window_nm)
    np.testing.assert_allclose(O.line_opacity(a) + O.line_opacity(b), k_all, rtol=1e-13)


def test_weak_line_limit():
    """F_c - F is proportional to gf to first order."""
    wl = W.tiny(seed=4, L=3, N=300)
    base = wl.lines.loggf.copy()
    depth = []
    for shift in (-7.0, -8.0):
        wl.lines.loggf[:] = base + shift
        F, Fc = O.synthesize(wl)
        depth.append(np.max(Fc - F))
    assert abs(depth[0] / depth[1] / 10 - 1) < 5e-5


def test_slice_locality():
    """A pixel's flux depends only on lines within W: any slice reproduces the full run."""
    wl = W.tiny(seed=8, L=25, N=700)
    F, Fc = O.synthesize(wl)
    pix = np.array([0, 5, 333, 334, 699])
    Fs, Fcs = O.synthesize(wl, pix=pix)
    np.testing.assert_allclose(Fs, F[pix], rtol=1e-14)
    np.testing.assert_allclose(Fcs, Fc[pix], rtol=1e-14)


# ------------------------------------------------------------------------- adjoint
def _loss(wl, params, seedF):
    F, _ = O.synthesize(wl, params)
    return float(np.dot(seedF, F))


@pytest.mark.parametrize("quad", ["gauss3", "e2"])
def test_adjoint_matches_central_differences(quad):
    """Reverse pass of Sec. 6 (four corrections of Eq. 30) vs FP64 central differences
    with a Richardson consistency check."""
    wl = W.tiny(seed=21, L=10, N=350, D=10, S=3, n_molecular=1)
    wl.quadrature = quad
    rng = np.random.default_rng(3)
    wl.params = W.random_params(rng, wl.lines.L, wl.atm.S, 1.4)
    seed = rng.normal(size=wl.grid.N)
    g = O.adjoint(wl, wl.params, seed)

    def fd(setter, h):
        import copy
        p1, p2 = copy.deepcopy(wl.params), copy.deepcopy(wl.params)
        setter(p1, +h)
        setter(p2, -h)
        return (_loss(wl, p1, seed) - _loss(wl, p2, seed)) / (2 * h)

    F0, _ = O.synthesize(wl, wl.params)
    loss_mag = float(np.sum(np.abs(seed * F0)))

    def check(val, setter, h):
        d1, d2 = fd(setter, h), fd(setter, h / 2)
        noise = 1e-14 * loss_mag / h          # rounding floor of a central difference
        scale = abs(d2)
        assert abs(d1 - d2) <= 1e-6 * scale + noise
        assert abs(val - d2) <= 1e-6 * scale + noise, (val, d2)

    for l in range(wl.lines.L):
        def sgf(p, h, l=l):
            p.dgf[l] += h
        def sdd(p, h, l=l):
            p.ddamp[l] += h
        check(g["g_loggf"][l], sgf, 1e-4)
        check(g["g_damp"][l], sdd, 1e-4)
    for s in range(wl.atm.S):
        def sA(p, h, s=s):
            p.dA[s] += h
        check(g["g_abund"][s], sA, 1e-4)

    def sxi(p, h):
        p.xi_kms += h
    check(g["g_xi"], sxi, 1e-4)
    # abundance enters exactly like dgf of the species' lines (fixed atmosphere)
    for s in range(wl.atm.S):
        assert abs(g["g_abund"][s] - g["g_loggf"][wl.lines.species == s].sum()) <= 1e-12 * (abs(g["g_abund"][s]) + 1e-300)


def test_damping_width_far_wing():
    """Eq. 5 damping: far from the core the profile is Lorentzian,
    phi -> (Gamma / 4 pi^2) / (nu - nu_l)^2 with Gamma = 10^ddamp (g_rad + g_S n_e + g_vdW n_pert)."""
    wl = W.tiny(seed=13, L=1, N=3001, D=3, R=3e5, window_nm=2.0)
    lam = O.wavelengths_nm(wl.grid)
    wl.lines.lam0_nm[:] = lam[1500]
    wl.params.ddamp[:] = 0.37
    k = O.line_opacity(wl)
    ln, atm = wl.lines, wl.atm
    lp = O.line_depth_params(atm, ln, [0.0], [0.37], wl.params.dA, wl.params.xi_kms)
    gamma = 10 ** 0.37 * (10 ** ln.log_grad[0] + 10 ** ln.log_gstark[0] * atm.ne + 10 ** ln.log_gvdw[0] * atm.npert)
    nu = sc.c * 100 / (lam * 1e-7)
    nu0 = sc.c * 100 / (ln.lam0_nm[0] * 1e-7)
    i = 1500 + 350                     # ~ 1.75 nm from the centre: >> Doppler width
    lor = lp["s"][0] * gamma / (4 * math.pi ** 2) / ((nu[i] - nu0) ** 2 + (gamma / (4 * math.pi)) ** 2)
    dv = (nu[i] - nu0) / lp["dnu"][0]
    corr = 1 + 1.5 / dv ** 2           # next term of the wing expansion
    np.testing.assert_allclose(k[:, i], lor * corr, rtol=1e-6)
