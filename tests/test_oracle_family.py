"""Pins of the per-family damping corrections of Eq. 30 in the oracle: equal
family corrections act as one scale of the total width; the three family
gradients sum to the total-width gradient; each matches FP64 central
differences of the oracle's forward synthesis."""
import copy

import numpy as np

import workloads as W
from oracle import synth as O


def _tiny(seed=101, L=15, N=500, D=8):
    wl = W.tiny(seed=seed, L=L, N=N, D=D, S=4, n_molecular=1, xi=1.1)
    rng = np.random.default_rng(seed)
    wl.params = W.random_params(rng, L, 4, 1.1)
    wl.params.ddamp_family = rng.normal(0.0, 0.2, (3, L))
    return wl


def test_equal_family_corrections_scale_the_total():
    wl = _tiny()
    p = wl.params
    delta = np.random.default_rng(5).normal(0.0, 0.3, wl.lines.L)
    pf = W.Params(p.dgf, np.zeros_like(p.ddamp), p.dA, p.xi_kms, np.stack([delta] * 3))
    pt = W.Params(p.dgf, delta, p.dA, p.xi_kms, None)
    np.testing.assert_allclose(O.line_opacity(wl, pf), O.line_opacity(wl, pt), rtol=1e-12)


def test_family_gradients_sum_to_the_total():
    wl = _tiny()
    seed = np.random.default_rng(6).normal(size=wl.grid.N)
    r = O.adjoint(wl, wl.params, seed)
    np.testing.assert_allclose(r["g_damp_family"].sum(axis=0), r["g_damp"], rtol=1e-10,
                               atol=1e-12 * np.max(np.abs(r["g_damp"])))


def test_family_gradients_match_finite_differences():
    wl = _tiny(seed=102, L=10, N=400)
    seed = np.random.default_rng(7).normal(size=wl.grid.N)
    r = O.adjoint(wl, wl.params, seed)

    def loss(p):
        return float(seed @ O.synthesize(wl, p)[0])

    h = 1e-5
    for f in range(3):
        for l in (0, 4, 9):
            p1, p2 = copy.deepcopy(wl.params), copy.deepcopy(wl.params)
            p1.ddamp_family[f, l] += h
            p2.ddamp_family[f, l] -= h
            fd = (loss(p1) - loss(p2)) / (2 * h)
            g = r["g_damp_family"][f, l]
            assert abs(fd - g) <= 1e-5 * abs(g) + 1e-9 * np.max(np.abs(r["g_damp_family"])), (f, l, fd, g)
