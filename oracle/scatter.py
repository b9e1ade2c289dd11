"""FP64 CPU oracle of the transfer with continuum scattering (Sec. 2.1, Eqs. 3
and 6-8).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It shares no code with the
GPU library.

With continuum scattering sigma_c the extinction is chi = kappa_c + sigma_c +
sum_l kappa_l (Eq. 3), the thermal fraction is eps = (kappa_c + sum_l kappa_l)
/ chi and the source function S = eps B + (1 - eps) J (Eq. 6), J the mean
intensity.  The paper iterates the scattering term; the result of that
iteration is its fixed point, which this module computes directly: with the
mean-intensity operator Lambda of the discretised formal solution (J =
Lambda S, a D x D matrix per pixel), S solves

    (I - diag(1 - eps) Lambda) S = eps B .

Discretisation (the one the path uses for the emergent intensity): S is
piecewise linear in tau between depths and extrapolated linearly to tau = 0
over the surface segment; the outward intensity starts from the diffusion
approximation I = S + mu dS/dtau at the deepest layer, the inward intensity
from I = 0 at tau = 0; J_j = 1/2 sum_k w_k (I+_j(mu_k) + I-_j(mu_k)) with the
3-point Gauss-Legendre nodes on [0, 1] of the flux (Eq. 8).  The continuum
branch scatters too (chi_c = kappa_c + sigma_c, eps_c = kappa_c / chi_c).
Scattering opacity per unit mass: sigma_c(lambda, j) = sigma_c,j (lambda /
lambda_ref)^sigma_alpha from the atmosphere (reading: the paper gives no
scattering law for synthesis; Thomson scattering is grey, Rayleigh ~ lambda^-4).

Every function accepts complex tau and kappa, so that the gradient of the flux
with respect to the line opacity can be taken by complex-step differentiation
(Im f(x + i h) / h, exact to rounding).
"""
from __future__ import annotations

import math

import numpy as np

from . import synth as O


def _lw(x):
    """(1 - (1 + x) e^-x) / x with its Taylor series for small |x| (branch on Re x)."""
    x = np.asarray(x)
    small = np.real(x) < 0.05
    xs = np.where(small, x, 0.0)
    series = np.zeros_like(x)
    for n in range(12, 1, -1):
        series = series + (-1.0) ** n * (n - 1) * xs ** (n - 1) / math.factorial(n)
    xl = np.where(small, 1.0, x)
    return np.where(small, series, (1.0 - (1.0 + xl) * np.exp(-xl)) / xl)


def scattering_opacity(wl, pix=None):
    """sigma_c [D, n] per unit mass at the pixels pix (zeros without scattering)."""
    a = wl.atm
    lam = O.wavelengths_nm(wl.grid, pix)
    sig = getattr(a, "sigma_c", None)
    if sig is None:
        return np.zeros((a.D, lam.size))
    return np.asarray(sig, np.float64)[:, None] * (lam[None, :] / a.lam_ref_nm) ** getattr(a, "sigma_alpha", 0.0)


def intensity_profiles(S, tau, mu):
    """Outward and inward intensities I+_j, I-_j [D, n] along direction mu."""
    D = S.shape[0]
    Iout = np.empty_like(S)
    Iout[D - 1] = S[D - 1] + mu * (S[D - 1] - S[D - 2]) / (tau[D - 1] - tau[D - 2])
    for j in range(D - 2, -1, -1):
        x = (tau[j + 1] - tau[j]) / mu
        e = np.exp(-x)
        Iout[j] = Iout[j + 1] * e + S[j] * (1.0 - e) + (S[j + 1] - S[j]) * _lw(x)
    Iin = np.empty_like(S)
    S_top = S[0] - tau[0] * (S[1] - S[0]) / (tau[1] - tau[0])
    x = tau[0] / mu
    e = np.exp(-x)
    Iin[0] = S[0] * (1.0 - e) + (S_top - S[0]) * _lw(x)
    for j in range(1, D):
        x = (tau[j] - tau[j - 1]) / mu
        e = np.exp(-x)
        Iin[j] = Iin[j - 1] * e + S[j] * (1.0 - e) + (S[j - 1] - S[j]) * _lw(x)
    return Iout, Iin


def mean_intensity(S, tau):
    """J = Lambda S by direct sweeps, [D, n]."""
    J = np.zeros_like(S)
    for mu, w in zip(O.GAUSS3_MU, O.GAUSS3_W):
        Iout, Iin = intensity_profiles(S, tau, mu)
        J = J + 0.5 * w * (Iout + Iin)
    return J


def emergent_flux(S, tau):
    """Eq. 8 with the outward intensity continued over the surface segment."""
    F = 0.0
    S_top = S[0] - tau[0] * (S[1] - S[0]) / (tau[1] - tau[0])
    for mu, w in zip(O.GAUSS3_MU, O.GAUSS3_W):
        Iout, _ = intensity_profiles(S, tau, mu)
        x = tau[0] / mu
        e = np.exp(-x)
        I0 = Iout[0] * e + S_top * (1.0 - e) + (S[0] - S_top) * _lw(x)
        F = F + 2.0 * math.pi * w * mu * I0
    return F


def lambda_matrix(tau):
    """Lambda [n, D, D] with J[:, i] = Lambda[i] @ S[:, i], built by carrying the
    coefficient rows of I+ and I- through the same sweeps."""
    D, n = tau.shape
    Lam = np.zeros((n, D, D), dtype=tau.dtype)
    r = np.arange(n)
    for mu, w in zip(O.GAUSS3_MU, O.GAUSS3_W):
        A = np.zeros((n, D), dtype=tau.dtype)
        g = mu / (tau[D - 1] - tau[D - 2])
        A[r, D - 1] += 1.0 + g
        A[r, D - 2] -= g
        Lam[:, D - 1, :] += 0.5 * w * A
        for j in range(D - 2, -1, -1):
            x = (tau[j + 1] - tau[j]) / mu
            e = np.exp(-x)
            lw = _lw(x)
            A = A * e[:, None]
            A[r, j] += (1.0 - e) - lw
            A[r, j + 1] += lw
            Lam[:, j, :] += 0.5 * w * A
        A = np.zeros((n, D), dtype=tau.dtype)
        x = tau[0] / mu
        e = np.exp(-x)
        lw = _lw(x)
        c = tau[0] / (tau[1] - tau[0])              # S_top = S_0 (1 + c) - S_1 c
        A[r, 0] += (1.0 - e) + lw * c
        A[r, 1] -= lw * c
        Lam[:, 0, :] += 0.5 * w * A
        for j in range(1, D):
            x = (tau[j] - tau[j - 1]) / mu
            e = np.exp(-x)
            lw = _lw(x)
            A = A * e[:, None]
            A[r, j] += (1.0 - e) - lw
            A[r, j - 1] += lw
            Lam[:, j, :] += 0.5 * w * A
    return Lam


def source_function(eps, B, tau):
    """The fixed point S = eps B + (1 - eps) Lambda S, solved per pixel, [D, n]."""
    D, n = tau.shape
    Lam = lambda_matrix(tau)
    M = np.eye(D)[None, :, :] - (1.0 - eps.T)[:, :, None] * Lam
    rhs = (eps * B).T[:, :, None]
    return np.linalg.solve(M, rhs)[:, :, 0].T


def _branch(kappa_abs, sigma, B, m):
    chi = kappa_abs + sigma
    tau = O.optical_depth(chi, m)
    S = source_function(kappa_abs / chi, B, tau)
    return emergent_flux(S, tau)


def flux_from_opacity(wl, kappa_line, pix=None):
    """Both branches with scattering (Gauss-3 flux) for the pixels pix."""
    if wl.quadrature != "gauss3":
        raise ValueError("scattering is defined with the Gauss-3 angle quadrature")
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    lam = O.wavelengths_nm(wl.grid, pix)
    kc = O.continuum_opacity(wl, pix)[None, :] * np.ones((wl.atm.D, 1))
    sig = scattering_opacity(wl, pix)
    B = O.planck_lambda_per_nm(lam, wl.atm.T)
    m = wl.atm.m
    return _branch(kc + kappa_line, sig, B, m), _branch(kc + 0.0 * kappa_line, sig, B, m)


def synthesize(wl, params=None, pix=None):
    """Forward synthesis with scattering: (F, Fc) per nm at the pixels pix."""
    return flux_from_opacity(wl, O.line_opacity(wl, params, pix), pix)


def opacity_adjoint(wl, kappa_line, dLdF, pix=None, h=1e-30):
    """g[D, n] = dL/dkappa_line for the seed dLdF on the total branch, by
    complex-step differentiation, one depth at a time (pixels are independent)."""
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    lam = O.wavelengths_nm(wl.grid, pix)
    kc = O.continuum_opacity(wl, pix)[None, :] * np.ones((wl.atm.D, 1))
    sig = scattering_opacity(wl, pix)
    B = O.planck_lambda_per_nm(lam, wl.atm.T)
    m = wl.atm.m
    g = np.zeros_like(kappa_line)
    for j in range(wl.atm.D):
        kl = kappa_line.astype(np.complex128)
        kl[j] += 1j * h
        g[j] = np.asarray(dLdF) * np.imag(_branch(kc + kl, sig, B, m)) / h
    return g


def adjoint(wl, params, dLdF, pix=None, conditions=False):
    """As synth.adjoint, for the transfer with scattering."""
    params = params or wl.params
    pix = np.arange(wl.grid.N) if pix is None else np.asarray(pix, np.int64)
    kl = O.line_opacity(wl, params, pix)
    g = opacity_adjoint(wl, kl, dLdF, pix)
    Ggf, Gd, Gxi, Gdf = O.line_gradients(wl, params, g, pix)
    GA = np.zeros(wl.atm.S)
    np.add.at(GA, wl.lines.species, Ggf)
    out = dict(g_loggf=Ggf, g_damp=Gd, g_abund=GA, g_xi=float(np.sum(Gxi)), g_damp_family=Gdf, g_kappa=g)
    if conditions:
        Agf, Ad, Axi, Adf = O.line_gradients(wl, params, g, pix, absolute=True)
        AA = np.zeros(wl.atm.S)
        np.add.at(AA, wl.lines.species, Agf)
        out.update(abs_loggf=Agf, abs_damp=Ad, abs_abund=AA, abs_xi=float(np.sum(Axi)), abs_damp_family=Adf)
    return out
