"""FP64 CPU oracle of the line-list calibration workload (Sec. 6, Eq. 30).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It shares no code with the
GPU library.

Sec. 6 calibrates four logarithmic corrections per group of catalogue lines
(Eq. 30: oscillator strength and the radiative, Stark and van der Waals
damping constants); every line of a group takes its group's four values.

Groups.  Optional curated anchor complexes are kept first, one group each.
Then a greedy pass visits the remaining lines from the strongest down and
gives every unvisited line a new group holding it and every other unassigned
line of the same species and ionisation stage within dE in lower excitation
energy and dlam in wavelength of it.  Readings where the text is brief:
"strength" is log gf (larger first, ties by catalogue index); the tolerances
are measured from the visiting line (the group's seed), not chained from
member to member; both bounds are inclusive; groups are numbered anchors
first (ascending anchor id), then in visiting order; lines outside the
calibration set belong to no group (index -1) and keep zero corrections.

Objective.  Each standard spectrum s is synthesised with the expanded
corrections, passed through the instrument operator (Eq. 31) to its observed
pixels, and compared with its observed spectrum y_s by a weighted mean square
(the telluric weights w_s; each standard carries its own overall weight c_s):

    L(theta) = sum_s c_s sum_p w_sp (f_sp(theta) - y_sp)^2 .

The gradient with respect to the group corrections theta [4][G] (rows: log gf,
radiative, Stark, van der Waals, dex) is the sum over each group's lines of the
per-line gradients of the synthesis adjoint.
"""
from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from . import instrument as I
from . import synth as O

# one wavenumber in energy: h c = 1.239841984e-6 eV m (CODATA), per cm^-1
CM1_EV = 1.239841984e-4


def correction_groups(lam0_nm, E_eV, species, ion, loggf, dE_eV, dlam_nm, active=None, anchor=None):
    """Group index per line ([L] int64, -1 = not calibrated) and the group count.

    active: optional [L] bool, the lines to calibrate (default all).
    anchor: optional [L] int, >= 0 for a line of a curated anchor complex
            (one group per distinct id), -1 otherwise.
    """
    lam0_nm = np.asarray(lam0_nm, np.float64)
    E_eV = np.asarray(E_eV, np.float64)
    species = np.asarray(species)
    ion = np.asarray(ion)
    loggf = np.asarray(loggf, np.float64)
    L = lam0_nm.size
    act = np.ones(L, bool) if active is None else np.asarray(active, bool)
    q = np.full(L, -1, np.int64)
    G = 0
    if anchor is not None:
        anchor = np.asarray(anchor)
        for a in np.unique(anchor[(anchor >= 0) & act]):
            q[(anchor == a) & act] = G
            G += 1
    order = sorted(range(L), key=lambda l: (-loggf[l], l))
    for s in order:
        if not act[s] or q[s] >= 0:
            continue
        take = (act & (q < 0) & (species == species[s]) & (ion == ion[s])
                & (np.abs(E_eV - E_eV[s]) <= dE_eV) & (np.abs(lam0_nm - lam0_nm[s]) <= dlam_nm))
        q[take] = G
        G += 1
    return q, G


def expand(q, theta):
    """Per-line corrections from group corrections theta [4][G]: (dgf [L],
    ddamp_family [3][L]); lines with q = -1 get zeros."""
    theta = np.asarray(theta, np.float64)
    q = np.asarray(q)
    x = np.zeros((4, q.size))
    m = q >= 0
    x[:, m] = theta[:, q[m]]
    return x[0], x[1:4]


def group_sums(q, G, x_line):
    """out[r, g] = sum over lines l with q[l] = g of x_line[r, l] (rows of x_line)."""
    x_line = np.atleast_2d(np.asarray(x_line, np.float64))
    q = np.asarray(q)
    out = np.zeros((x_line.shape[0], G))
    m = q >= 0
    for r in range(x_line.shape[0]):
        np.add.at(out[r], q[m], x_line[r, m])
    return out


def weighted_mse(f, y, w, c):
    """c sum_p w_p (f_p - y_p)^2 and its gradient with respect to f."""
    d = np.asarray(f, np.float64) - np.asarray(y, np.float64)
    w = np.asarray(w, np.float64)
    return c * float(np.sum(w * d * d)), 2.0 * c * w * d


class Standard:
    """One standard spectrum: a workload (atmosphere, grid, shared line list,
    its own abundance corrections and microturbulence), an instrument with the
    velocities (v_r, v_b), the observed spectrum y, weights w and weight c."""

    def __init__(self, wl, inst, vel, y, w, c):
        self.wl, self.inst, self.vel = wl, inst, (float(vel[0]), float(vel[1]))
        self.y, self.w, self.c = np.asarray(y, np.float64), np.asarray(w, np.float64), float(c)


def _params(std, q, theta):
    """The standard's corrections with the line terms expanded from theta."""
    dgf, fam = expand(q, theta)
    p = std.wl.params
    return SimpleNamespace(dgf=dgf, ddamp=np.zeros_like(dgf), dA=p.dA, xi_kms=p.xi_kms, ddamp_family=fam)


def model(std, q, theta):
    """Observed-pixel model f_s(theta) of one standard."""
    F, Fc = O.synthesize(std.wl, _params(std, q, theta))
    return I.forward(std.inst, F, Fc, *std.vel)[2]


def objective(standards, q, G, theta, with_grad=True):
    """L(theta), and (with_grad) dL/dtheta [4][G] with the sums of absolute
    values of the same terms [4][G] (a conditioning scale for comparisons)."""
    loss = 0.0
    grad = np.zeros((4, G))
    absg = np.zeros((4, G))
    for std in standards:
        par = _params(std, q, theta)
        F, Fc = O.synthesize(std.wl, par)
        f = I.forward(std.inst, F, Fc, *std.vel)[2]
        l, df = weighted_mse(f, std.y, std.w, std.c)
        loss += l
        if not with_grad:
            continue
        dF = I.adjoint(std.inst, F, Fc, *std.vel, df)[0]
        r = O.adjoint(std.wl, par, dF, conditions=True)
        grad += group_sums(q, G, np.vstack([r["g_loggf"], r["g_damp_family"]]))
        absg += group_sums(q, G, np.vstack([r["abs_loggf"], r["abs_damp_family"]]))
    return (loss, grad, absg) if with_grad else loss
