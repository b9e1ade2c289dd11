"""Pins of the line-selection keep test oracle (Sec. 3, Eqs. 17-19): in an
isothermal atmosphere with lines at their bins' centre frequencies, R_l
exp(-E_l/kT_*) equals the largest Doppler-core centre opacity of Eq. 4 (from
the synthesis oracle's own line strength) over eta_sel times the continuum,
which pins C_0 and every factor; in a grey atmosphere it bounds that ratio
from above (the test is conservative); Q by explicit loops over depths; R
scales as 1/eta_sel and the kept set shrinks as eta_sel grows."""
import copy
import math

import numpy as np

import workloads as W
from oracle import selection as OS
from oracle import synth as O


def _at_bin_centres(wl, bin_ln, seed=3):
    """Move every line to the centre (in ln lambda) of a random bin."""
    rng = np.random.default_rng(seed)
    B = OS.n_bins(wl.grid, bin_ln)
    b = rng.integers(0, B, wl.lines.L)
    wl.lines.lam0_nm = OS.bin_centre_nm(wl.grid, b, bin_ln)
    return b


def _core_ratio(wl, params, eta_sel, bin_ln):
    """max_j and per-depth K_lj / (eta kappa_c(lambda_l)), K = s / (sqrt(pi) dnu_D)."""
    lp = O.line_depth_params(wl.atm, wl.lines, params.dgf, params.ddamp, params.dA, params.xi_kms)
    kc = O.continuum_at(wl, wl.lines.lam0_nm)
    return lp["s"] / (O.SQRT_PI * lp["dnu"]) / (eta_sel * kc[:, None])


def _case(seed=5, isothermal=False):
    wl = W.tiny(seed=seed, L=300, N=3000, D=30, S=5, n_molecular=1, lam_lo=1500.0)
    wl.params = W.random_params(np.random.default_rng(seed), wl.lines.L, 5, 1.3)
    if isothermal:
        wl.atm.T[:] = 5200.0
    return wl


def test_isothermal_equals_core_opacity_ratio():
    wl = _case(isothermal=True)
    bin_ln = 2e-3
    b = _at_bin_centres(wl, bin_ln)
    r = OS.select_lines(wl, wl.params, 1e-3, bin_ln)
    np.testing.assert_array_equal(r["b"], b)
    ratio = _core_ratio(wl, wl.params, 1e-3, bin_ln)
    np.testing.assert_allclose(r["R_deep"], ratio.max(axis=1), rtol=1e-11)
    assert 0 < r["keep"].sum() < wl.lines.L                 # the case exercises both outcomes


def test_grey_atmosphere_bound_is_conservative():
    wl = _case(seed=6)
    assert np.all(np.diff(wl.atm.T) > 0)                    # T_* is the hottest layer
    bin_ln = 1e-3
    _at_bin_centres(wl, bin_ln, seed=4)
    r = OS.select_lines(wl, wl.params, 1e-3, bin_ln)
    ratio = _core_ratio(wl, wl.params, 1e-3, bin_ln)       # [L, D]
    assert np.all(r["R_deep"] >= ratio.max(axis=1) * (1 - 1e-12))
    boltz = np.exp(-wl.lines.E_eV[:, None] * O.EV / (O.K_BOLTZ * wl.atm.T[None, :]))
    assert np.all(r["R"] >= (ratio / boltz).max(axis=1) * (1 - 1e-12))
    # a dropped line is below eta_sel times the continuum at its centre in every layer
    drop = ~r["keep"]
    assert drop.any() and np.all(ratio[drop] < 1.0)


def test_Q_by_explicit_loops():
    wl = _case(seed=7)
    wl.atm = copy.deepcopy(wl.atm)
    bin_ln, eta = 5e-3, 2e-3
    r = OS.select_lines(wl, wl.params, eta, bin_ln)
    a = wl.atm
    P = O.population_factor(a, wl.params.dA)
    B = OS.n_bins(wl.grid, bin_ln)
    for s in range(a.S):
        for ion in range(2):
            for bb in range(B):
                lam = wl.grid.lam_first_nm * math.exp((bb + 0.5) * bin_ln)
                nu = O.C_LIGHT / (lam * 1e-7)
                best = 0.0
                for j in range(a.D):
                    kc = a.kappa0 * (lam / a.lam_ref_nm) ** a.alpha
                    C = eta * kc / (1.0 - math.exp(-O.H_PLANCK * nu / (O.K_BOLTZ * a.T[j])))
                    xi = wl.params.xi_kms * 1e5
                    dv = math.sqrt(2 * O.K_BOLTZ * a.T[j] / (a.mass_amu[s] * O.AMU) + xi * xi)
                    best = max(best, P[s, ion, j] / (dv / O.C_LIGHT * C))
                assert abs(r["Q"][s, ion, bb] - best) <= 1e-12 * best


def test_threshold_scaling_and_monotone_keep():
    wl = _case(seed=8)
    r1 = OS.select_lines(wl, wl.params, 1e-4, 1e-3)
    r2 = OS.select_lines(wl, wl.params, 1e-2, 1e-3)
    np.testing.assert_allclose(r1["R"], 100.0 * r2["R"], rtol=1e-12)
    assert np.all(r1["keep"] | ~r2["keep"]) and r1["keep"].sum() > r2["keep"].sum()


def test_edge_bins_and_corrections():
    wl = _case(seed=9)
    wl.lines.lam0_nm[:3] = [1400.0, 1499.9999, 1700.0]   # outside the grid: edge bins
    r = OS.select_lines(wl, wl.params, 1e-3, 1e-3)
    B = OS.n_bins(wl.grid, 1e-3)
    assert list(r["b"][:3]) == [0, 0, B - 1]
    # +1 dex on a line's gf multiplies its R by 10; +1 dex of abundance does so for its species
    p = copy.deepcopy(wl.params)
    p.dgf = np.array(p.dgf, float)
    p.dgf[5] += 1.0
    r2 = OS.select_lines(wl, p, 1e-3, 1e-3)
    np.testing.assert_allclose(r2["R"][5], 10.0 * r["R"][5], rtol=1e-12)
    p = copy.deepcopy(wl.params)
    s = wl.lines.species[7]
    p.dA = np.array(p.dA, float)
    p.dA[s] += 1.0
    r3 = OS.select_lines(wl, p, 1e-3, 1e-3)
    m = wl.lines.species == s
    np.testing.assert_allclose(r3["R"][m], 10.0 * r["R"][m], rtol=1e-12)
