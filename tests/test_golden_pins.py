"""Pins of the stored FP64 oracle reference for the 1500-1700 nm
differentiation workload (tests/golden/fit_1500_1700nm_golden.npz, written by
tests/golden/make_fit_1500_1700nm_golden.py from the oracle alone).

* The stored oracle adjoint agrees with FP64 central differences of the
  oracle's own forward synthesis (Richardson-combined steps h and h/2) for
  20 log gf, 20 damping, 9 abundance and the microturbulence corrections:
  the definition of the derivative, independent of the adjoint code.  The
  criterion is relative for gradients at least 1e-2 of the largest and
  absolute (a fraction of the largest) below that, where a central
  difference is rounding noise.
* The stored target and seed are what the oracle gives on re-evaluation at
  sampled pixels (the chi^2 objective of Sec. 5 on the Eq. 9 ratio).
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import synth as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fit_1500_1700nm_golden.npz")


@pytest.fixture(scope="module")
def golden():
    return np.load(GOLDEN)


def s17_ok(g, fd, rtol, atol_frac):
    """|g - fd| <= rtol |fd| where |fd| >= 1e-2 max|fd|, else <= atol_frac max|fd|
    (a central difference of a near-zero gradient is rounding noise)."""
    gmax = np.max(np.abs(fd))
    big = np.abs(fd) >= 1e-2 * gmax
    err = np.abs(np.asarray(g) - fd)
    return np.where(big, err <= rtol * np.abs(fd), err <= atol_frac * gmax), big


def test_adjoint_matches_finite_differences(golden):
    z = golden
    fd, fh, adj = z["fd_value"], z["fd_value_half"], z["fd_adjoint"]
    rich = (4.0 * fh - fd) / 3.0
    ok, big = s17_ok(adj, rich, 1e-5, 1e-7)
    assert ok.all(), [(z["fd_kind"][i], int(z["fd_index"][i]), rich[i], adj[i]) for i in np.flatnonzero(~ok)[:5]]
    assert big.sum() >= 15                       # most of the 50 are well above the noise floor
    # the two step sizes agree where the difference is resolved: converged, not noise
    ok_h, _ = s17_ok(fd, fh, 1e-4, 1e-6)
    assert ok_h.all()
    assert set(z["fd_kind"]) == {"loggf", "damp", "abund", "xi"}


def test_target_and_seed_reproduce(golden):
    z = golden
    wl = W.giant_1500_1700nm_fit()
    rng = np.random.default_rng(5)
    pix = np.unique(np.concatenate([[0, wl.grid.N - 1], rng.integers(0, wl.grid.N, 14)]))
    Ft, Fct = O.synthesize(wl, wl.extra["truth"], pix=pix)
    y = Ft / Fct + wl.extra["noise"][pix]
    np.testing.assert_allclose(z["y"][pix], y, rtol=1e-6)
    F, Fc = O.synthesize(wl, wl.params, pix=pix)
    dF, _ = O.chi2_seed(F, Fc, z["y"][pix].astype(np.float64), wl.extra["sigma"])
    scale = np.max(np.abs(z["seed"]))
    assert np.max(np.abs(z["seed"][pix] - dF)) <= 1e-5 * scale


# ------------------------------------------------ full-pixel flux goldens
# tests/golden/flux_1500_1700nm_golden.npz and flux_300_1000nm_slices_golden.npz
# (written by tests/golden/make_flux_goldens.py from the oracle alone).  The
# stored values are what the oracle gives on re-evaluation at sampled pixels,
# and the slices are the 2-nm pieces they claim to be.
FLUX_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flux_1500_1700nm_golden.npz")
SLICE_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flux_300_1000nm_slices_golden.npz")
BATCH_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flux_batch_stars_golden.npz")


def test_flux_golden_1500_1700nm_reproduces():
    z = np.load(FLUX_GOLDEN)
    wl = W.giant_1500_1700nm()
    assert z["F"].shape == (wl.grid.N,) and str(z["workload"]) == wl.name
    rng = np.random.default_rng(6)
    pix = np.unique(np.concatenate([[0, wl.grid.N - 1], rng.integers(0, wl.grid.N, 10)]))
    F, Fc = O.synthesize(wl, pix=pix)
    np.testing.assert_allclose(z["F"][pix], F, rtol=1e-12)
    np.testing.assert_allclose(z["Fc"][pix], Fc, rtol=1e-12)
    assert np.all(z["F"] > 0) and np.all(z["F"] <= z["Fc"])


def test_flux_golden_batch_stars_reproduce():
    """Every pixel of three batch stars (own atmosphere, window and catalogue):
    sampled pixels of each recomputed by the oracle."""
    z = np.load(BATCH_GOLDEN)
    rng = np.random.default_rng(8)
    for b in z["stars"]:
        wl = W.batch_star(int(b))
        F = z["F_%d" % b]
        assert F.shape == (wl.grid.N,)
        pix = np.unique(np.concatenate([[0, wl.grid.N - 1], rng.integers(0, wl.grid.N, 3)]))
        Fo, Fco = O.synthesize(wl, pix=pix)
        np.testing.assert_allclose(F[pix], Fo, rtol=1e-12)
        np.testing.assert_allclose(z["Fc_%d" % b][pix], Fco, rtol=1e-12)
        assert np.all(F > 0) and np.all(F <= z["Fc_%d" % b])


def test_flux_golden_300_1000nm_slices():
    z = np.load(SLICE_GOLDEN)
    wl = W.solar_300_1000nm()
    lam = O.wavelengths_nm(wl.grid)
    pix = z["pix"]
    starts = np.flatnonzero(np.diff(pix) != 1) + 1
    pieces = np.split(pix, starts)
    assert len(pieces) == 3
    assert pieces[0][0] == 0 and pieces[2][-1] == wl.grid.N - 1
    assert abs(lam[pieces[1][0]] - 650.0) < 0.01
    for p in pieces:                               # each slice spans 2 nm
        assert 1.99 < lam[p[-1]] - lam[p[0]] < 2.0
    rng = np.random.default_rng(7)
    sel = np.unique(np.concatenate([[0, pix.size - 1], rng.integers(0, pix.size, 4)]))
    F, Fc = O.synthesize(wl, pix=pix[sel])
    np.testing.assert_allclose(z["F"][sel], F, rtol=1e-12)
    np.testing.assert_allclose(z["Fc"][sel], Fc, rtol=1e-12)
