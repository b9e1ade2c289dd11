"""Pins of the oracle's continuum-referenced centre test and wing spans.

The rule (oracle.synth.center_test) is this implementation's reading of the
paper's description (Sec. 2.2, Table 2).  These tests check it by properties
computed independently with the Faddeeva function, not by retyping it:
limits that reduce to the plain windowed sum or to the bare continuum, the
size of what is dropped and of what is kept relative to eta times the
continuum, monotonicity in eta, and the adjoint against finite differences.
"""
import copy

import numpy as np
import pytest
from scipy.special import wofz

import workloads as W
from oracle import synth as O


def _tiny(eta, seed=71, L=25, N=600, D=8):
    wl = W.tiny(seed=seed, L=L, N=N, D=D, S=4, n_molecular=1, xi=1.2)
    wl.params = W.random_params(np.random.default_rng(seed), L, 4, 1.2)
    wl.center_eta = eta
    return wl


def test_vanishing_threshold_is_the_plain_sum():
    plain = _tiny(0.0)
    ct = _tiny(1e-300)
    np.testing.assert_array_equal(O.line_opacity(ct), O.line_opacity(plain))


def test_huge_threshold_leaves_the_continuum():
    wl = _tiny(1e300)
    assert np.all(O.line_opacity(wl) == 0.0)
    F, Fc = O.synthesize(wl)
    np.testing.assert_array_equal(F, Fc)


@pytest.mark.parametrize("eta", [1e-4, 1e-3, 1e-2])
def test_dropped_and_kept_pairs_bracket_the_threshold(eta):
    """Brute force over every in-window (pixel, line, depth): a dropped pair's
    opacity is at most 3 eta kappa_c, a kept pair's at least 0.3 eta kappa_c
    (H from wofz at the pair's own v; kappa_c at the line centre)."""
    wl = _tiny(eta)
    pix = np.arange(wl.grid.N)
    p_idx, l_idx = O.window_pairs(wl.grid, wl.lines, wl.window_nm, pix)
    lp, v = O._pair_terms(wl, wl.params, p_idx, l_idx, pix)
    keep, V = O.center_test(wl, lp, wl.lines.lam0_nm[l_idx][:, None])
    inc = keep & (np.abs(v) <= V)
    K = lp["s"] / (np.sqrt(np.pi) * lp["dnu"])
    ratio = K * wofz(v + 1j * lp["a"]).real / O.continuum_at(wl, wl.lines.lam0_nm[l_idx])[:, None]
    assert inc.any() and (~inc).any()
    assert ratio[~inc].max() <= 3.0 * eta
    assert ratio[inc].min() >= 0.3 * eta
    # the keep decision is the centre value: H(a, 0) from wofz agrees with erfcx
    centre = K * wofz(1j * lp["a"]).real / O.continuum_at(wl, wl.lines.lam0_nm[l_idx])[:, None]
    assert np.all((centre >= eta * (1 + 1e-12)) <= keep) and np.all(keep <= (centre >= eta * (1 - 1e-12)))


def test_flux_monotone_and_converging_in_threshold():
    """Dropping absorbers raises the flux (T increases inward), and the change
    from the plain sum shrinks as eta does."""
    F0, Fc = O.synthesize(_tiny(0.0))
    prev = None
    for eta in (1e-2, 1e-3, 1e-4):
        F, Fc2 = O.synthesize(_tiny(eta))
        np.testing.assert_array_equal(Fc2, Fc)
        assert np.all(F >= F0 * (1 - 1e-13))
        dev = np.max(np.abs(F / Fc - F0 / Fc))
        if prev is not None:
            assert dev < prev
        prev = dev
    assert prev < 1e-3


def test_adjoint_with_center_test_matches_finite_differences():
    wl = _tiny(1e-3, seed=72, L=12, N=400, D=8)
    rng = np.random.default_rng(3)
    seed = rng.normal(size=wl.grid.N)
    adj = O.adjoint(wl, wl.params, seed)

    def loss(p):
        F, _ = O.synthesize(wl, p)
        return float(seed @ F)

    def mask(p):
        pix = np.arange(wl.grid.N)
        p_idx, l_idx = O.window_pairs(wl.grid, wl.lines, wl.window_nm, pix)
        lp, v = O._pair_terms(wl, p, p_idx, l_idx, pix)
        keep, V = O.center_test(wl, lp, wl.lines.lam0_nm[l_idx][:, None])
        return keep & (np.abs(v) <= V)

    h = 1e-6
    m0 = mask(wl.params)
    checked = 0
    for kind, idx in (("dgf", 0), ("dgf", 5), ("ddamp", 3), ("ddamp", 9), ("dA", 1), ("xi", 0)):
        p1, p2 = copy.deepcopy(wl.params), copy.deepcopy(wl.params)
        if kind == "xi":
            p1.xi_kms += h
            p2.xi_kms -= h
            ref = adj["g_xi"]
        else:
            getattr(p1, kind)[idx] += h
            getattr(p2, kind)[idx] -= h
            ref = {"dgf": adj["g_loggf"], "ddamp": adj["g_damp"], "dA": adj["g_abund"]}[kind][idx]
        if not (np.array_equal(mask(p1), m0) and np.array_equal(mask(p2), m0)):
            continue                                  # a pair crossed the threshold: no derivative there
        fd = (loss(p1) - loss(p2)) / (2 * h)
        assert abs(fd - ref) <= 1e-5 * abs(ref), (kind, idx, fd, ref)
        checked += 1
    assert checked >= 4
