"""Pins of the line-calibration oracle (Sec. 6, Eq. 30): the greedy correction
groups on a hand-worked catalogue and by their defining properties on random
ones (a partition into same-species, same-ion groups inside the tolerances of
their strongest line, which no later group could have joined; the limits of
zero and unbounded tolerances); expansion and group sums as transposes; and
the gradient of the multi-standard objective against FP64 central
differences of the objective itself."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import calibration as OC
from oracle import instrument as I

DE = 2.0 * OC.CM1_EV
DLAM = 0.035


def _hand_catalogue():
    """Seven lines; columns lambda (nm), E (eV), species, ion, log gf."""
    rows = [(1500.000, 2.0000, 0, 0, -1.0),    # 0
            (1500.030, 2.0002, 0, 0, -2.0),    # 1
            (1500.060, 2.0001, 0, 0, -0.5),    # 2  strongest
            (1500.001, 2.0000, 0, 1, -3.0),    # 3  other ion
            (1500.000, 2.0000, 1, 0, -2.5),    # 4  other species
            (1500.000, 2.0003, 0, 0, -4.0),    # 5  3e-4 eV from line 0 (> 2 cm^-1)
            (1499.966, 1.9998, 0, 0, -1.5)]    # 6  0.034 nm, 2e-4 eV from line 0
    a = np.array(rows)
    return a[:, 0], a[:, 1], a[:, 2].astype(int), a[:, 3].astype(int), a[:, 4]


def test_groups_hand_worked():
    """Visiting order by log gf: 2, 0, 6, 1, 4, 3, 5.  Line 2 takes line 1
    (0.03 nm, 1e-4 eV) but not line 0 (0.06 nm); line 0 then seeds a group and
    takes line 6 (0.034 nm, 2e-4 eV) although line 6 is 0.094 nm from line 2
    (no chaining); line 5 misses line 0 by energy; lines 3 and 4 differ in ion
    or species."""
    q, G = OC.correction_groups(*_hand_catalogue(), DE, DLAM)
    assert G == 5
    np.testing.assert_array_equal(q, [1, 0, 0, 3, 2, 4, 1])


def test_groups_hand_worked_anchor_and_inactive():
    """Anchor complex {0, 5} is group 0; then line 2 seeds {1, 2}, line 6 is
    alone (line 0 is taken), line 4 seeds its own; line 3 is not calibrated."""
    lam, E, sp, ion, gf = _hand_catalogue()
    anchor = np.array([7, -1, -1, -1, -1, 7, -1])
    active = np.array([1, 1, 1, 0, 1, 1, 1], bool)
    q, G = OC.correction_groups(lam, E, sp, ion, gf, DE, DLAM, active=active, anchor=anchor)
    assert G == 4
    np.testing.assert_array_equal(q, [0, 1, 1, -1, 3, 0, 2])


def _random_catalogue(seed, n=1500):
    rng = np.random.Generator(np.random.PCG64(seed))
    lines, _ = W.complex_lines(rng, n, 1500.0, 1503.0, 3)
    gf = np.round(lines.loggf, 1)                     # many ties in strength
    return lines.lam0_nm, lines.E_eV, lines.species, lines.ion, gf


@pytest.mark.parametrize("seed", [1, 2])
def test_groups_properties(seed):
    lam, E, sp, ion, gf = _random_catalogue(seed)
    q, G = OC.correction_groups(lam, E, sp, ion, gf, DE, DLAM)
    assert q.min() == 0 and q.max() == G - 1 and np.unique(q).size == G
    seeds = []
    for g in range(G):
        m = np.flatnonzero(q == g)
        # the seed is the first line in visiting order: strongest, then lowest index
        s = m[np.lexsort((m, -gf[m]))][0]
        seeds.append(s)
        assert np.all(sp[m] == sp[s]) and np.all(ion[m] == ion[s])
        assert np.all(np.abs(lam[m] - lam[s]) <= DLAM) and np.all(np.abs(E[m] - E[s]) <= DE)
        # maximality: no line of a later group was within reach of this seed
        later = np.flatnonzero(q > g)
        reach = (sp[later] == sp[s]) & (ion[later] == ion[s]) & (np.abs(lam[later] - lam[s]) <= DLAM) \
            & (np.abs(E[later] - E[s]) <= DE)
        assert not reach.any()
    # groups are numbered in visiting order
    key = [(-gf[s], s) for s in seeds]
    assert key == sorted(key)


def test_groups_limits():
    lam, E, sp, ion, gf = _random_catalogue(3, n=400)
    # zero tolerances: only exact duplicates group; this catalogue has none
    q, G = OC.correction_groups(lam, E, sp, ion, gf, 0.0, 0.0)
    assert G == lam.size
    lam2, E2 = np.concatenate([lam, lam[:5]]), np.concatenate([E, E[:5]])
    sp2, ion2, gf2 = np.concatenate([sp, sp[:5]]), np.concatenate([ion, ion[:5]]), np.concatenate([gf, gf[:5] - 1])
    q, G = OC.correction_groups(lam2, E2, sp2, ion2, gf2, 0.0, 0.0)
    assert G == lam.size and np.array_equal(q[-5:], q[:5])
    # unbounded tolerances: one group per (species, ion) present
    q, G = OC.correction_groups(lam, E, sp, ion, gf, np.inf, np.inf)
    pairs = {(a, b) for a, b in zip(sp, ion)}
    assert G == len(pairs)
    for g in range(G):
        m = q == g
        assert np.unique(sp[m]).size == 1 and np.unique(ion[m]).size == 1


def test_expand_and_group_sums_are_transposes():
    rng = np.random.default_rng(4)
    q = np.array([2, -1, 0, 2, 1, 1, -1, 2])
    theta = rng.normal(size=(4, 3))
    y = rng.normal(size=(4, q.size))
    dgf, fam = OC.expand(q, theta)
    x = np.vstack([dgf, fam])
    assert np.all(x[:, q < 0] == 0.0)
    assert abs(np.sum(y * x) - np.sum(OC.group_sums(q, 3, y) * theta)) <= 1e-13


def _oracle_standards(cal, theta_true, noise_seed):
    q, G = OC.correction_groups(cal.lines.lam0_nm, cal.lines.E_eV, cal.lines.species, cal.lines.ion,
                                cal.lines.loggf, DE, DLAM, active=cal.active)
    rng = np.random.default_rng(noise_seed)
    stds = []
    for s in cal.standards:
        inst = I.Instrument(s.wl.grid, s.lam_obs_nm, s.lsf_sigma_ln, s.vb_max_kms)
        st = OC.Standard(s.wl, inst, s.vel, np.zeros(s.lam_obs_nm.size), s.w, s.c)
        st.y = OC.model(st, q, theta_true[:, :G] if theta_true is not None else np.zeros((4, G))) \
            + rng.normal(0.0, 0.002, s.lam_obs_nm.size)
        stds.append(st)
    return stds, q, G


def test_objective_gradient_matches_finite_differences():
    cal = W.calibration_tiny(seed=31, n_records=16, N=1200, D=16)
    truth = W.calibration_truth(np.random.default_rng(8), 64)
    stds, q, G = _oracle_standards(cal, truth, 9)
    theta = 0.5 * W.calibration_truth(np.random.default_rng(10), G)
    loss, grad, absg = OC.objective(stds, q, G, theta)
    assert loss > 0.0
    h = 1e-5
    for r in range(4):
        for g in {0, G // 2, G - 1}:
            tp, tm = theta.copy(), theta.copy()
            tp[r, g] += h
            tm[r, g] -= h
            fd = (OC.objective(stds, q, G, tp, with_grad=False) - OC.objective(stds, q, G, tm, with_grad=False)) / (2 * h)
            assert abs(fd - grad[r, g]) <= 1e-5 * abs(grad[r, g]) + 1e-7 * absg[r, g], (r, g, fd, grad[r, g])
