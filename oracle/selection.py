"""FP64 CPU oracle of the atmosphere-dependent line-selection keep test
(Sec. 3, Eqs. 17-19).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It shares no code with the
GPU library.

For one atmosphere, the keep test decides which catalogue lines can matter in
any layer, from a per-(species, ion stage, frequency bin) summary:

  Eq. 17  C_jb = eta_sel (kappa_c + sigma_c)(nu_b, j) / (1 - exp(-h nu_b / k T_j)),
  Eq. 18  Q_srb = max_j (n_{s,r} / U_{s,r})_j / (rho_j (dnu_D / nu)_{js} C_jb),
  Eq. 19  R_l = C_0 (gf)_l Q_{s(l) r(l) b(l)} / nu_b(l),
          keep l iff R_l >= 1 and R_l exp(-E_l / k T_*) >= 1,

with T_* the temperature of the deepest layer.  Readings where the text
leaves things open:
  - C_0 = sqrt(pi) e^2 / (m_e c): with it, R_l exp(-E_l/kT_j) times the
    depth-j term of Q is the Doppler-core centre opacity of Eq. 4
    (s / (sqrt(pi) dnu_D), the profile's peak for a = 0) over eta_sel times the
    continuum, with the stimulated-emission factor taken at nu_b on both sides;
  - bins are equal intervals of width bin_ln in ln lambda starting at the
    first grid wavelength; a line's bin is floor(ln(lambda_l / lambda_first) /
    bin_ln), clamped to the bins that cover the grid (so lines outside it use
    the edge bins); nu_b is the frequency at the bin's centre in ln lambda;
  - the continuum is the path's power law with sigma_c = 0; the populations,
    the Doppler widths (thermal and microturbulent, Eq. 5) and gf include the
    corrections of Eq. 30 passed with the call (dA, xi, dgf).
"""
from __future__ import annotations

import math

import numpy as np

from . import synth as O

C_SEL = O.SQRT_PI * O.E_CHARGE ** 2 / (O.M_ELECTRON * O.C_LIGHT)   # C_0 = sqrt(pi) e^2 / (m_e c)


def n_bins(grid, bin_ln):
    lam_last = grid.lam_first_nm * (1.0 + 1.0 / grid.R) ** (grid.N - 1)
    return int(math.floor(math.log(lam_last / grid.lam_first_nm) / bin_ln)) + 1


def bin_of(grid, lam0_nm, bin_ln):
    B = n_bins(grid, bin_ln)
    b = np.floor(np.log(np.asarray(lam0_nm, np.float64) / grid.lam_first_nm) / bin_ln)
    return np.clip(b, 0, B - 1).astype(np.int64)


def bin_centre_nm(grid, b, bin_ln):
    return grid.lam_first_nm * np.exp((np.asarray(b, np.float64) + 0.5) * bin_ln)


def select_lines(wl, params=None, eta_sel=1e-3, bin_ln=1e-3):
    """Keep mask and strength proxies for the lines of wl.  Returns dict(keep
    [L] bool, R [L], R_deep [L] = R exp(-E/kT_*), b [L], Q [S, 2, B])."""
    params = params or wl.params
    atm, lines, grid = wl.atm, wl.lines, wl.grid
    B = n_bins(grid, bin_ln)
    lam_b = bin_centre_nm(grid, np.arange(B), bin_ln)                  # [B]
    nu_b = O.C_LIGHT / (lam_b * 1.0e-7)
    kc = atm.kappa0 * (lam_b / atm.lam_ref_nm) ** atm.alpha           # sigma_c = 0
    T = atm.T
    C = eta_sel * kc[None, :] / (-np.expm1(-O.H_PLANCK * nu_b[None, :] / (O.K_BOLTZ * T[:, None])))   # [D, B], Eq. 17
    P = O.population_factor(atm, params.dA)                            # [S, 2, D] = n / (rho U)
    xi = params.xi_kms * 1.0e5
    dv_c = np.sqrt(2.0 * O.K_BOLTZ * T[None, :] / (atm.mass_amu[:, None] * O.AMU) + xi * xi) / O.C_LIGHT   # [S, D]
    Q = np.max(P[:, :, :, None] / (dv_c[:, None, :, None] * C[None, None, :, :]), axis=2)   # [S, 2, B], Eq. 18
    b = bin_of(grid, lines.lam0_nm, bin_ln)
    gf = 10.0 ** (lines.loggf + np.asarray(params.dgf))
    R = C_SEL * gf * Q[lines.species, lines.ion, b] / nu_b[b]          # Eq. 19
    R_deep = R * np.exp(-lines.E_eV * O.EV / (O.K_BOLTZ * T[-1]))
    return dict(keep=(R >= 1.0) & (R_deep >= 1.0), R=R, R_deep=R_deep, b=b, Q=Q)
