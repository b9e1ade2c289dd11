"""FP64 CPU oracle for LTE synthesis through a fixed 1-D atmosphere.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It shares no code with the
GPU library: it is the plain definition of what the GPU path computes, written
out step by step from the paper, slow and in float64.

Steps and the passages they follow (Sec. 2.1 unless noted):

  grid        Eq. 1: lambda_i = lambda_first (1 + 1/R)^i
  populations Sec. 3, Eq. 11 (Saha, two stages, no ionisation lowering);
              Eq. 30 for the abundance correction 10^dA
  line params Eqs. 4-5 (Doppler width with microturbulence, damping ratio),
              Eq. 30 (gf' = gf 10^dgf, gamma' = gamma 10^ddamp)
  profile     Voigt H(a, v) = Re w(v + i a), phi = H / (sqrt(pi) dnu_D)
              (normalised to unit frequency integral as Eq. 4 requires);
              w is the Faddeeva function (scipy.special.wofz, a library
              special function used as one step)
  window      pixel i receives line l iff |lambda_i - lambda_l| <= W
              (the bounded wing span of Sec. 2.2; W fixed by the workload)
  centre test optional (Sec. 2.2, Table 2): a (line, depth) pair is kept only
              if its centre opacity reaches eta times the continuum, and a kept
              pair deposits only within a strength-dependent span |v| <= V
              (the threshold and the span rule are this implementation's
              reading; see center_test)
  extinction  Eq. 3 with sigma_c = 0 and a power-law continuum
  tau         d tau = chi dm with the trapezoid rule, tau_0 = chi_0 m_0
  source      Eq. 6 with epsilon = 1: S = B_lambda(T), per nm
  transfer    Eq. 7, piecewise-linear S in tau, diffusion lower boundary,
              linear extrapolation of S to the surface
  flux        Eq. 8: F = 2 pi int_0^1 I(0, mu) mu dmu by 3-point Gauss-Legendre
              in mu ("gauss3"), or F = 2 pi int S E2 dtau ("e2")
  ratio       Eq. 9 with an identity instrument operator
  adjoint     reverse of every step above for the four corrections of Eq. 30
              (per-line log gf, per-line damping scale, per-species abundance,
              microturbulence), Sec. 6

Units: CGS inside; wavelengths in nm at the interface; energies in eV;
masses in amu; microturbulence in km/s; flux per nm.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import wofz, expn, erfcx

# CODATA 2018
C_LIGHT = 2.99792458e10          # cm s^-1
H_PLANCK = 6.62607015e-27        # erg s
K_BOLTZ = 1.380649e-16           # erg K^-1
E_CHARGE = 4.803204712570263e-10  # esu
M_ELECTRON = 9.1093837015e-28    # g
AMU = 1.66053906660e-24          # g
EV = 1.602176634e-12             # erg
LN10 = math.log(10.0)
SQRT_PI = math.sqrt(math.pi)

LINE_CONST = math.pi * E_CHARGE ** 2 / (M_ELECTRON * C_LIGHT)   # pi e^2 / (m_e c)
SAHA_CONST = (2.0 * math.pi * M_ELECTRON * K_BOLTZ / H_PLANCK ** 2) ** 1.5

# 3-point Gauss-Legendre on [0, 1]
GAUSS3_MU = np.array([0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)])
GAUSS3_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


# ----------------------------------------------------------------------------- grid
def wavelengths_nm(grid, pix=None):
    """Eq. 1."""
    i = np.arange(grid.N, dtype=np.float64) if pix is None else np.asarray(pix, np.float64)
    return grid.lam_first_nm * (1.0 + 1.0 / grid.R) ** i


# ---------------------------------------------------------------------- populations
def ion_fractions(atm):
    """Saha ionisation (Eq. 11) between stages I and II with Delta I = 0.

    Returns f[S, 2, D] with f_I + f_II = 1.  Species with an infinite
    ionisation energy have a single stage (f_I = 1).
    """
    T = atm.T[None, :]
    chi = atm.chi_ion_eV[:, None] * EV
    ratioU = 2.0 * atm.U[:, 1, :] / atm.U[:, 0, :]
    with np.errstate(over="ignore"):
        phi = ratioU * SAHA_CONST * T ** 1.5 * np.exp(-chi / (K_BOLTZ * T)) / atm.ne[None, :]
    phi = np.where(np.isfinite(chi), phi, 0.0)
    fI = 1.0 / (1.0 + phi)
    fII = phi / (1.0 + phi)
    return np.stack([fI, fII], axis=1)


def population_factor(atm, dA):
    """n_{s,r} / (rho U_{s,r}) with n_{s,r} = 10^dA_s n_s f_r  (Eq. 4, Eq. 11, Eq. 30)."""
    f = ion_fractions(atm)
    n = (10.0 ** np.asarray(dA))[:, None, None] * atm.n_species[:, None, :] * f
    return n / (atm.rho[None, None, :] * atm.U)


# -------------------------------------------------------------------- line params
def line_depth_params(atm, lines, dgf, ddamp, dA, xi_kms, ddamp_family=None):
    """Per (line, depth): Doppler width dnu_D [Hz], damping ratio a and the
    frequency-integrated line strength s (per unit mass), Eqs. 4-5 and 30.

    kappa_{l}(nu_i, j) = s_lj * H(a_lj, v) / (sqrt(pi) dnu_D,lj).
    The damping width is 10^ddamp (g_rad 10^d_rad + g_S n_e 10^d_S +
    g_vdW n_pert 10^d_vdW): Eq. 30 corrects each family; ddamp scales the
    total (both default to 0).  Returns dict of [L, D] arrays (gam_fam holds
    the three corrected family widths, [3, L, D]) plus the per-line rest
    frequency.
    """
    T = atm.T[None, :]
    mass = atm.mass_amu[lines.species][:, None] * AMU
    xi = xi_kms * 1.0e5
    dv = np.sqrt(2.0 * K_BOLTZ * T / mass + xi * xi)                  # Eq. 5
    nu_l = C_LIGHT / (lines.lam0_nm * 1.0e-7)
    dnu = nu_l[:, None] * dv / C_LIGHT                                # Eq. 5
    fam = np.zeros((3, lines.L)) if ddamp_family is None else np.asarray(ddamp_family, np.float64)
    scale = 10.0 ** np.asarray(ddamp)[:, None]                        # Eq. 30
    gam_fam = np.stack([10.0 ** (lines.log_grad + fam[0])[:, None] * np.ones_like(T),
                        10.0 ** (lines.log_gstark + fam[1])[:, None] * atm.ne[None, :],
                        10.0 ** (lines.log_gvdw + fam[2])[:, None] * atm.npert[None, :]]) * scale
    gamma = gam_fam[0] + gam_fam[1] + gam_fam[2]
    a = gamma / (4.0 * math.pi * dnu)                                 # Eq. 5
    P = population_factor(atm, dA)[lines.species, lines.ion, :]      # [L, D]
    gf = 10.0 ** (lines.loggf + np.asarray(dgf))                      # Eq. 30
    boltz = np.exp(-lines.E_eV[:, None] * EV / (K_BOLTZ * T))
    stim = 1.0 - np.exp(-H_PLANCK * nu_l[:, None] / (K_BOLTZ * T))   # at nu_l
    s = LINE_CONST * P * gf[:, None] * boltz * stim                   # Eq. 4
    return dict(dnu=dnu, a=a, s=s, nu_l=nu_l, dv=dv, gam_fam=gam_fam, gamma=gamma)


def voigt(a, v):
    """H(a, v) = Re w(v + i a)."""
    return wofz(v + 1j * a).real


def voigt_w(a, v):
    w = wofz(v + 1j * a)
    return w.real, w.imag


# ----------------------------------------------------------------------- opacity
def _lines_sorted(lines):
    order = np.argsort(lines.lam0_nm, kind="stable")
    return order, lines.lam0_nm[order]


def window_pairs(grid, lines, window_nm, pix):
    """All (pixel, line) pairs with |lambda_i - lambda_l| <= W, for the pixels pix.

    Returns (pixel position in pix, line index), grouped by pixel.
    """
    pix = np.asarray(pix, dtype=np.int64)
    lam = wavelengths_nm(grid, pix)
    order, lam_sorted = _lines_sorted(lines)
    lo = np.searchsorted(lam_sorted, lam - window_nm * (1 + 1e-9), side="left")
    hi = np.searchsorted(lam_sorted, lam + window_nm * (1 + 1e-9), side="right")
    counts = hi - lo
    p_idx = np.repeat(np.arange(pix.size), counts)
    starts = np.repeat(lo - np.concatenate([[0], np.cumsum(counts)[:-1]]), counts)
    cand = order[np.arange(p_idx.size) + starts]
    keep = np.abs(lam[p_idx] - lines.lam0_nm[cand]) <= window_nm
    return p_idx[keep], cand[keep]


def _pair_terms(wl, params, p_idx, l_idx, pix, want_w=False):
    """Per pair and depth: line params and v for the pairs (p_idx into pix, l_idx)."""
    lines = wl.lines.take(l_idx)
    dgf = np.asarray(params.dgf)[l_idx]
    ddamp = np.asarray(params.ddamp)[l_idx]
    fam = getattr(params, "ddamp_family", None)
    fam = None if fam is None else np.asarray(fam)[:, l_idx]
    lp = line_depth_params(wl.atm, lines, dgf, ddamp, params.dA, params.xi_kms, fam)
    nu_i = C_LIGHT / (wavelengths_nm(wl.grid, np.asarray(pix)[p_idx]) * 1.0e-7)
    v = (nu_i[:, None] - lp["nu_l"][:, None]) / lp["dnu"]
    return lp, v


def _blocks(n_items, work_per_item, budget=3_000_000):
    step = max(1, int(budget // max(1, work_per_item)))
    for s in range(0, n_items, step):
        yield s, min(n_items, s + step)


def line_opacity(wl, params=None, pix=None):
    """kappa_line[D, len(pix)] = sum over in-window lines of s H / (sqrt(pi) dnu_D) (Eqs. 3-4)."""
    params = params or wl.params
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    D = wl.atm.D
    out = np.zeros((D, pix.size))
    p_idx, l_idx = window_pairs(wl.grid, wl.lines, wl.window_nm, pix)
    # process pairs in blocks to bound memory; the sum per pixel is the definition
    for b0, b1 in _blocks(p_idx.size, D):
        pp, ll = p_idx[b0:b1], l_idx[b0:b1]
        lp, v = _pair_terms(wl, params, pp, ll, pix)
        kap = lp["s"] * voigt(lp["a"], v) / (SQRT_PI * lp["dnu"])
        kap = kap * _center_mask(wl, lp, wl.lines.lam0_nm[ll][:, None], v)
        np.add.at(out.T, pp, kap)
    return out


def continuum_opacity(wl, pix=None):
    """Power-law continuum per unit mass, depth independent; sigma_c = 0."""
    lam = wavelengths_nm(wl.grid, pix)
    a = wl.atm
    return a.kappa0 * (lam / a.lam_ref_nm) ** a.alpha


def continuum_at(wl, lam_nm):
    """The same power-law continuum at arbitrary wavelengths (nm)."""
    a = wl.atm
    return a.kappa0 * (np.asarray(lam_nm, np.float64) / a.lam_ref_nm) ** a.alpha


def center_test(wl, lp, lam0_nm):
    """Continuum-referenced centre test and wing span of a (line, depth) pair.

    With R = K / kappa_c(lambda_l), K = s / (sqrt(pi) dnu) the line opacity per
    unit H, and eta = wl.center_eta:
      keep  iff  R H(a, 0) >= eta,   H(a, 0) = erfcx(a)   (centre opacity vs continuum)
      V     =  max( sqrt(ln(R / eta)) if R > eta else 0,  sqrt(a R / (sqrt(pi) eta)) ),
    the Doppler-core and Lorentz-wing radii at which the profile falls to eta
    times the continuum.  A kept pair contributes at pixel i iff |v_i| <= V.
    lp holds [.., D] arrays (s, dnu, a); lam0_nm broadcasts against them.
    Returns (keep, V) as [.., D] arrays.
    """
    eta = wl.center_eta
    K = lp["s"] / (SQRT_PI * lp["dnu"])
    R = K / continuum_at(wl, lam0_nm)
    a = lp["a"]
    keep = R * erfcx(a) >= eta
    with np.errstate(divide="ignore", invalid="ignore"):
        vd = np.sqrt(np.maximum(np.log(R / eta), 0.0))
    vl = np.sqrt(a * R / (SQRT_PI * eta))
    return keep, np.maximum(vd, vl)


def _center_mask(wl, lp, lam0_nm, v):
    """1 where the centre test keeps the pair and |v| <= V, else 0; all ones when off."""
    if not wl.center_eta:
        return 1.0
    keep, V = center_test(wl, lp, lam0_nm)
    return (keep & (np.abs(v) <= V)).astype(np.float64)


# ---------------------------------------------------------------------- transfer
def planck_lambda_per_nm(lam_nm, T):
    """B_lambda(T) = 2 h c^2 lambda^-5 / (exp(hc / lambda k T) - 1), per nm.  S[D, n]."""
    lam = np.asarray(lam_nm)[None, :] * 1.0e-7
    TT = np.asarray(T)[:, None]
    return 2.0 * H_PLANCK * C_LIGHT ** 2 / lam ** 5 / np.expm1(H_PLANCK * C_LIGHT / (lam * K_BOLTZ * TT)) * 1.0e-7


def optical_depth(chi, m):
    """tau_0 = chi_0 m_0; tau_{j+1} = tau_j + (chi_j + chi_{j+1}) (m_{j+1} - m_j) / 2."""
    tau = np.empty_like(chi)
    tau[0] = chi[0] * m[0]
    for j in range(1, chi.shape[0]):
        tau[j] = tau[j - 1] + 0.5 * (chi[j - 1] + chi[j]) * (m[j] - m[j - 1])
    return tau


def lin_weight(x):
    """(1 - (1 + x) e^-x) / x, with its Taylor series for small x."""
    x = np.asarray(x, dtype=np.float64)
    small = x < 0.05
    xs = np.where(small, x, 0.0)
    series = np.zeros_like(x)
    for n in range(12, 1, -1):   # sum_{n>=2} (-1)^n (n-1) x^(n-1) / n!
        series = series + (-1.0) ** n * (n - 1) * xs ** (n - 1) / math.factorial(n)
    xl = np.where(small, 1.0, x)
    direct = (1.0 - (1.0 + xl) * np.exp(-xl)) / xl
    return np.where(small, series, direct)


def _surface_extension(S, tau):
    """S extrapolated linearly to tau = 0 from the first segment."""
    slope0 = (S[1] - S[0]) / (tau[1] - tau[0])
    return S[0] - tau[0] * slope0


def intensity_surface(S, tau, mu):
    """Emergent I(0, mu) for piecewise-linear S (Eq. 7) with diffusion lower boundary."""
    D = S.shape[0]
    I = S[D - 1] + mu * (S[D - 1] - S[D - 2]) / (tau[D - 1] - tau[D - 2])
    for j in range(D - 2, -1, -1):
        x = (tau[j + 1] - tau[j]) / mu
        e = np.exp(-x)
        I = I * e + S[j] * (1.0 - e) + (S[j + 1] - S[j]) * lin_weight(x)
    S_top = _surface_extension(S, tau)
    x = tau[0] / mu
    e = np.exp(-x)
    return I * e + S_top * (1.0 - e) + (S[0] - S_top) * lin_weight(x)


def flux_gauss3(S, tau):
    """Eq. 8: F = 2 pi sum_k w_k mu_k I(0, mu_k)."""
    F = 0.0
    for mu, w in zip(GAUSS3_MU, GAUSS3_W):
        F = F + 2.0 * math.pi * w * mu * intensity_surface(S, tau, mu)
    return F


def flux_e2(S, tau):
    """F = 2 pi int_0^inf S(t) E2(t) dt for piecewise-linear S, linear beyond the last depth."""
    D = S.shape[0]
    S_top = _surface_extension(S, tau)
    knots_t = [np.zeros_like(tau[0])] + [tau[j] for j in range(D)]
    knots_S = [S_top] + [S[j] for j in range(D)]
    F = 0.0
    for k in range(D):
        ta, tb = knots_t[k], knots_t[k + 1]
        Sa, Sb = knots_S[k], knots_S[k + 1]
        s = (Sb - Sa) / (tb - ta)
        E3a, E3b = expn(3, ta), expn(3, tb)
        E4a, E4b = expn(4, ta), expn(4, tb)
        F = F + Sa * (E3a - E3b) + s * (E4a - E4b - (tb - ta) * E3b)
    sD = (S[D - 1] - S[D - 2]) / (tau[D - 1] - tau[D - 2])
    F = F + S[D - 1] * expn(3, tau[D - 1]) + sD * expn(4, tau[D - 1])
    return 2.0 * math.pi * F


def emergent_flux(S, tau, quadrature):
    if quadrature == "gauss3":
        return flux_gauss3(S, tau)
    if quadrature == "e2":
        return flux_e2(S, tau)
    raise ValueError(quadrature)


def flux_from_opacity(wl, kappa_line, pix=None):
    """Both transfer branches (total and continuum-only) for the pixels pix."""
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    lam = wavelengths_nm(wl.grid, pix)
    kc = continuum_opacity(wl, pix)[None, :] * np.ones((wl.atm.D, 1))
    S = planck_lambda_per_nm(lam, wl.atm.T)
    m = wl.atm.m
    F = emergent_flux(S, optical_depth(kc + kappa_line, m), wl.quadrature)
    Fc = emergent_flux(S, optical_depth(kc, m), wl.quadrature)
    return F, Fc


def synthesize(wl, params=None, pix=None):
    """Forward synthesis: (F, Fc) per nm at the pixels pix (default: all)."""
    kl = line_opacity(wl, params, pix)
    return flux_from_opacity(wl, kl, pix)


# ------------------------------------------------------------------------ adjoint
def _lin_weight_deriv(x):
    """d/dx of (1 - (1 + x) e^-x) / x."""
    x = np.asarray(x, dtype=np.float64)
    small = x < 0.05
    xs = np.where(small, x, 0.0)
    series = np.zeros_like(x)
    for n in range(13, 1, -1):   # derivative of the series term by term
        series = series + (-1.0) ** n * (n - 1) * (n - 1) * xs ** (n - 2) / math.factorial(n)
    xl = np.where(small, 1.0, x)
    e = np.exp(-xl)
    # f = (1 - e - x e)/x ; f' = x e / x - (1 - e - x e)/x^2 = e - f/x
    f = (1.0 - (1.0 + xl) * e) / xl
    direct = e - f / xl
    return np.where(small, series, direct)


def intensity_surface_adjoint(S, tau, mu, gI):
    """Reverse of intensity_surface: returns dL/dtau[D, n] for the seed gI = dL/dI(0, mu)."""
    D = S.shape[0]
    # forward pass storing the intermediate intensities
    Is = [None] * (D + 1)
    I = S[D - 1] + mu * (S[D - 1] - S[D - 2]) / (tau[D - 1] - tau[D - 2])
    Is[D - 1] = I
    for j in range(D - 2, -1, -1):
        x = (tau[j + 1] - tau[j]) / mu
        e = np.exp(-x)
        I = I * e + S[j] * (1.0 - e) + (S[j + 1] - S[j]) * lin_weight(x)
        Is[j] = I
    gtau = np.zeros_like(tau)
    # top slab
    dt01 = tau[1] - tau[0]
    slope0 = (S[1] - S[0]) / dt01
    S_top = S[0] - tau[0] * slope0
    x = tau[0] / mu
    e = np.exp(-x)
    # I0 = Is[0] e + S_top (1 - e) + (S0 - S_top) lw(x)
    g_Iin = gI * e
    g_x = gI * (-Is[0] * e + S_top * e + (S[0] - S_top) * _lin_weight_deriv(x))
    g_Stop = gI * ((1.0 - e) - lin_weight(x))
    gtau[0] += g_x / mu
    # S_top = S0 - tau0 (S1 - S0) / (tau1 - tau0)
    gtau[0] += g_Stop * (-slope0)
    g_slope = g_Stop * (-tau[0])
    # slope0 = (S1 - S0)/(tau1 - tau0)
    gtau[1] += g_slope * (-slope0 / dt01)
    gtau[0] += g_slope * (slope0 / dt01)
    # segments, from the surface downward (reverse of the upward sweep)
    for j in range(0, D - 1):
        x = (tau[j + 1] - tau[j]) / mu
        e = np.exp(-x)
        # Is[j] = Is[j+1] e + S_j (1 - e) + (S_{j+1} - S_j) lw(x)
        g_x = g_Iin * (-Is[j + 1] * e + S[j] * e + (S[j + 1] - S[j]) * _lin_weight_deriv(x))
        gtau[j + 1] += g_x / mu
        gtau[j] -= g_x / mu
        g_Iin = g_Iin * e
    # bottom boundary: I_D = S_D + mu (S_D - S_{D-1}) / (tau_D - tau_{D-1})
    dS = S[D - 1] - S[D - 2]
    dt = tau[D - 1] - tau[D - 2]
    g_dt = g_Iin * (-mu * dS / dt ** 2)
    gtau[D - 1] += g_dt
    gtau[D - 2] -= g_dt
    return gtau


def flux_e2_adjoint(S, tau, gF):
    """Reverse of flux_e2 with respect to tau (dE_n/dt = -E_{n-1})."""
    D = S.shape[0]
    dt01 = tau[1] - tau[0]
    slope0 = (S[1] - S[0]) / dt01
    S_top = S[0] - tau[0] * slope0
    knots_S = [S_top] + [S[j] for j in range(D)]
    g_knot_t = [0.0] * (D + 1)
    g_Stop = 0.0
    c = 2.0 * math.pi * gF
    knots_t = [np.zeros_like(tau[0])] + [tau[j] for j in range(D)]
    for k in range(D):
        ta, tb = knots_t[k], knots_t[k + 1]
        Sa, Sb = knots_S[k], knots_S[k + 1]
        dtk = tb - ta
        s = (Sb - Sa) / dtk
        E2a, E2b = expn(2, ta), expn(2, tb)
        E3a, E3b = expn(3, ta), expn(3, tb)
        E4a, E4b = expn(4, ta), expn(4, tb)
        # term = Sa (E3a - E3b) + s (E4a - E4b - dtk E3b)
        g_s = c * (E4a - E4b - dtk * E3b)
        g_ta = c * (Sa * (-E2a) + s * (-E3a + E3b))
        g_tb = c * (Sa * E2b + s * (E3b - E3b + dtk * E2b))
        # s = (Sb - Sa)/(tb - ta)
        g_ta = g_ta + g_s * s / dtk
        g_tb = g_tb - g_s * s / dtk
        if k == 0:
            g_Stop = g_Stop + c * (E3a - E3b) - g_s / dtk
        g_knot_t[k] = g_knot_t[k] + g_ta
        g_knot_t[k + 1] = g_knot_t[k + 1] + g_tb
    dtD = tau[D - 1] - tau[D - 2]
    sD = (S[D - 1] - S[D - 2]) / dtD
    tD = tau[D - 1]
    g_tD = c * (S[D - 1] * (-expn(2, tD)) + sD * (-expn(3, tD)))
    g_sD = c * expn(4, tD)
    gtau = np.zeros_like(tau)
    for j in range(D):
        gtau[j] += g_knot_t[j + 1]
    gtau[D - 1] += g_tD - g_sD * sD / dtD
    gtau[D - 2] += g_sD * sD / dtD
    # S_top = S0 - tau0 slope0, slope0 = (S1 - S0)/(tau1 - tau0)
    gtau[0] += g_Stop * (-slope0)
    g_slope = g_Stop * (-tau[0])
    gtau[1] += g_slope * (-slope0 / dt01)
    gtau[0] += g_slope * (slope0 / dt01)
    return gtau


def optical_depth_adjoint(gtau, m):
    """Reverse of optical_depth: dL/dchi from dL/dtau."""
    D = gtau.shape[0]
    suffix = np.cumsum(gtau[::-1], axis=0)[::-1]     # Gamma_j = sum_{k >= j} dL/dtau_k
    gchi = np.zeros_like(gtau)
    gchi[0] = suffix[0] * m[0]
    for j in range(1, D):
        half = 0.5 * (m[j] - m[j - 1]) * suffix[j]
        gchi[j - 1] += half
        gchi[j] += half
    return gchi


def opacity_adjoint(wl, kappa_line, dLdF, pix=None):
    """g[D, n] = dL/dkappa_line for a seed dL/dF on the total branch."""
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    lam = wavelengths_nm(wl.grid, pix)
    kc = continuum_opacity(wl, pix)[None, :] * np.ones((wl.atm.D, 1))
    S = planck_lambda_per_nm(lam, wl.atm.T)
    tau = optical_depth(kc + kappa_line, wl.atm.m)
    if wl.quadrature == "gauss3":
        gtau = np.zeros_like(tau)
        for mu, w in zip(GAUSS3_MU, GAUSS3_W):
            gtau += intensity_surface_adjoint(S, tau, mu, 2.0 * math.pi * w * mu * dLdF)
    else:
        gtau = flux_e2_adjoint(S, tau, dLdF)
    return optical_depth_adjoint(gtau, wl.atm.m)


def line_gradients(wl, params, g, pix, line_subset=None, absolute=False):
    """Per-line gradients from g = dL/dkappa_line at the pixels pix.

    dkappa/d dgf   = ln10 kappa
    dkappa/d ddamp = ln10 K a dH/da                  (K = s / (sqrt(pi) dnu))
    dkappa/d xi    = -K (H + a dH/da + v dH/dv) * d ln dnu / d xi,
                     d ln dnu / d xi = xi / dv^2 (xi in the units of dv)
    with dH/dv = -2 (v H - a L), dH/da = 2 (v L + a H) - 2/sqrt(pi), w = H + i L.
    dkappa/d d_beta = ln10 K a dH/da * g_beta / Gamma for damping family beta
    (its share of the corrected width; the three sum to dkappa/d ddamp).
    Returns (G_gf[L], G_damp[L], G_xi_per_line[L], G_damp_family[3, L]) over
    all lines (zero for lines not in line_subset when given).  With absolute=True every term enters with
    its absolute value: sum |g dkappa/dp|, the scale against which the
    rounding error of the sum is measured (its condition).
    """
    pix = np.asarray(pix, np.int64)
    L = wl.lines.L
    Ggf, Gd, Gxi = np.zeros(L), np.zeros(L), np.zeros(L)
    Gdf = np.zeros((3, L))
    p_idx, l_idx = window_pairs(wl.grid, wl.lines, wl.window_nm, pix)
    if line_subset is not None:
        sel = np.isin(l_idx, np.asarray(line_subset))
        p_idx, l_idx = p_idx[sel], l_idx[sel]
    D = wl.atm.D
    xi = params.xi_kms * 1.0e5
    for b0, b1 in _blocks(p_idx.size, D):
        pp, ll = p_idx[b0:b1], l_idx[b0:b1]
        lp, v = _pair_terms(wl, params, pp, ll, pix)
        a = lp["a"]
        H, Lw = voigt_w(a, v)
        K = lp["s"] / (SQRT_PI * lp["dnu"])
        Hv = -2.0 * (v * H - a * Lw)
        Ha = 2.0 * (v * Lw + a * H) - 2.0 / SQRT_PI
        gij = g.T[pp]                                  # [pairs, D]
        kap = K * H
        dlndnu_dxi = xi / lp["dv"] ** 2 * 1.0e5        # per km/s
        t_gf = LN10 * gij * kap
        t_d = LN10 * gij * K * a * Ha
        t_xi = gij * (-K) * (H + a * Ha + v * Hv) * dlndnu_dxi
        mask = _center_mask(wl, lp, wl.lines.lam0_nm[ll][:, None], v)   # piecewise constant in the parameters
        t_gf, t_d, t_xi = t_gf * mask, t_d * mask, t_xi * mask
        t_df = t_d[None] * (lp["gam_fam"] / lp["gamma"][None])
        if absolute:
            t_gf, t_d, t_xi, t_df = np.abs(t_gf), np.abs(t_d), np.abs(t_xi), np.abs(t_df)
        np.add.at(Ggf, ll, np.sum(t_gf, axis=1))
        np.add.at(Gd, ll, np.sum(t_d, axis=1))
        np.add.at(Gxi, ll, np.sum(t_xi, axis=1))
        for f in range(3):
            np.add.at(Gdf[f], ll, np.sum(t_df[f], axis=1))
    return Ggf, Gd, Gxi, Gdf


def adjoint(wl, params, dLdF, pix=None, line_subset=None, conditions=False):
    """Vector-Jacobian product of F (total branch) with respect to the corrections.

    dLdF is the seed at the pixels pix (the continuum branch does not depend on
    any corrected quantity).  Returns dict(g_loggf[L], g_damp[L], g_abund[S],
    g_xi) -- the abundance and xi entries are complete only when pix covers
    every pixel that any line reaches.  conditions=True adds abs_* entries,
    the sums of the absolute values of the same terms.
    """
    params = params or wl.params
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    kl = line_opacity(wl, params, pix)
    g = opacity_adjoint(wl, kl, np.asarray(dLdF, np.float64), pix)
    Ggf, Gd, Gxi, Gdf = line_gradients(wl, params, g, pix, line_subset)
    GA = np.zeros(wl.atm.S)
    np.add.at(GA, wl.lines.species, Ggf)     # dA_s enters exactly like dgf of its lines
    out = dict(g_loggf=Ggf, g_damp=Gd, g_abund=GA, g_xi=float(np.sum(Gxi)), g_damp_family=Gdf, g_kappa=g)
    if conditions:
        Agf, Ad, Axi, Adf = line_gradients(wl, params, g, pix, line_subset, absolute=True)
        AA = np.zeros(wl.atm.S)
        np.add.at(AA, wl.lines.species, Agf)
        out.update(abs_loggf=Agf, abs_damp=Ad, abs_abund=AA, abs_xi=float(np.sum(Axi)), abs_damp_family=Adf)
    return out


def window_pixels(wl, line_idx):
    """All pixels within W of any of the given lines (sorted, unique)."""
    lam0 = wl.lines.lam0_nm[np.asarray(line_idx)]
    h = math.log1p(1.0 / wl.grid.R)
    lo = np.floor(np.log((lam0 - wl.window_nm) / wl.grid.lam_first_nm) / h).astype(np.int64) - 1
    hi = np.ceil(np.log((lam0 + wl.window_nm) / wl.grid.lam_first_nm) / h).astype(np.int64) + 1
    lo = np.clip(lo, 0, wl.grid.N - 1)
    hi = np.clip(hi, 0, wl.grid.N - 1)
    return np.unique(np.concatenate([np.arange(a, b + 1) for a, b in zip(lo, hi)]))


def chi2_seed(F, Fc, y, sigma):
    """dL/dF and dL/dFc for L = sum ((F/Fc - y)/sigma)^2 (Eq. 9 ratio, identity instrument)."""
    f = F / Fc
    r = 2.0 * (f - y) / sigma ** 2
    return r / Fc, -r * F / Fc ** 2
