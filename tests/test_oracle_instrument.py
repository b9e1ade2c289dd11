"""Pins of the instrument-operator oracle (Eq. 31 and Eq. 9), by closed forms and
properties: a constant spectrum passes unchanged; Gaussians compose (widths add
in quadrature, a whole-pixel shift moves the centre); linear interpolation is
exact on a linear ramp; each transpose passes the dot-product test; the
velocity and flux gradients agree with FP64 central differences."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import instrument as I


def _setup(P=160, R_lsf=(20000.0, 25000.0), vb_max=8.0):
    grid = W.grid_for(1550.0, 1556.0, 3.0e5)
    x0, h = math.log(grid.lam_first_nm), math.log1p(1.0 / grid.R)
    xN = x0 + (grid.N - 1) * h
    xp = np.linspace(x0 + 0.15 * (xN - x0), xN - 0.15 * (xN - x0), P)
    Rl = np.linspace(*R_lsf, P)
    inst = I.Instrument(grid, np.exp(xp), 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)) * Rl), vb_max)
    return grid, inst


def test_constant_spectrum_is_preserved():
    grid, inst = _setup()
    one = np.ones(grid.N)
    for vr, vb in ((0.0, 1.0), (13.7, 4.2), (-40.0, 7.9)):
        KF, KFc, f = I.forward(inst, 2.5 * one, one, vr, vb)
        np.testing.assert_allclose(KF, 2.5, rtol=1e-14)
        np.testing.assert_allclose(f, 2.5, rtol=1e-14)


def test_gaussian_line_composes_in_quadrature():
    """B, an integer-pixel S and K applied to a Gaussian absorption line give a
    Gaussian with sigma^2 = sigma0^2 + sigma_b^2 + sigma_p^2 centred at x0 + s
    (continuous-limit identity; widths of several pixels keep the discrete
    sums at their integrals)."""
    grid, inst = _setup()
    x = math.log(grid.lam_first_nm) + np.arange(grid.N) * inst.h
    xc = x[grid.N // 2]
    s0 = 6.0 * inst.h
    A = 0.6
    F = 1.0 - A * np.exp(-(x - xc) ** 2 / (2 * s0 ** 2))
    t = 7.0                                          # whole-pixel shift: interpolation exact
    vr = math.expm1(t * inst.h) * I.C_KMS
    vb = 4.5
    sb = vb / I.C_KMS
    KF, _, _ = I.forward(inst, F, np.ones(grid.N), vr, vb)
    xp = np.log(inst.lam_obs_nm)
    st2 = s0 ** 2 + sb ** 2 + inst.sigma_ln ** 2
    ref = 1.0 - A * s0 / np.sqrt(st2) * np.exp(-(xp - xc - t * inst.h) ** 2 / (2 * st2))
    # truncating the LSF at 4 sigma removes ~6e-5 of its weight: the bound below
    np.testing.assert_allclose(KF, ref, atol=2e-4 * A)
    assert np.max(np.abs(KF - ref)) < np.max(np.abs(ref - 1.0)) * 1e-3


def test_shift_is_exact_on_a_ramp():
    G = 3.0 + 0.25 * np.arange(500.0)
    for t in (0.37, -2.81, 11.5):
        S = I.shift(G, t)
        interior = slice(20, 480)
        np.testing.assert_allclose(S[interior], 3.0 + 0.25 * (np.arange(500.0)[interior] - t), rtol=1e-14)


@pytest.mark.parametrize("op", ["broaden", "shift", "lsf"])
def test_transposes(op):
    grid, inst = _setup()
    rng = np.random.default_rng(1)
    N, P = grid.N, inst.lam_obs_nm.size
    x = rng.normal(size=N)
    if op == "broaden":
        y = rng.normal(size=N)
        lhs = y @ I.broaden(x, 2.7, inst.J)
        rhs = I._broaden_T(y, 2.7, inst.J) @ x
    elif op == "shift":
        y = rng.normal(size=N)
        lhs = y @ I.shift(x, -3.4)
        rhs = I._shift_T(y, -3.4) @ x
    else:
        y = rng.normal(size=P)
        lhs = y @ I.apply_lsf(inst, x)
        rhs = I._lsf_T(inst, y, N) @ x
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_adjoint_matches_finite_differences():
    grid, inst = _setup(P=90)
    rng = np.random.default_rng(2)
    x = np.arange(grid.N)
    F = 1.0 - 0.5 * np.exp(-((x - 500.0) / 7.0) ** 2) - 0.3 * np.exp(-((x - 700.0) / 4.0) ** 2)
    Fc = 1.0 + 1e-4 * x
    vr, vb = 11.3, 3.7
    dL = rng.normal(size=inst.lam_obs_nm.size)
    dF, dFc, gvr, gvb = I.adjoint(inst, F, Fc, vr, vb, dL)
    L = lambda F_, Fc_, vr_, vb_: float(dL @ I.forward(inst, F_, Fc_, vr_, vb_)[2])
    h = 1e-4
    fd_vr = (L(F, Fc, vr + h, vb) - L(F, Fc, vr - h, vb)) / (2 * h)
    fd_vb = (L(F, Fc, vr, vb + h) - L(F, Fc, vr, vb - h)) / (2 * h)
    assert abs(fd_vr - gvr) <= 1e-6 * abs(gvr)
    assert abs(fd_vb - gvb) <= 1e-6 * abs(gvb)
    for i in (480, 500, 695, 710):
        e = np.zeros(grid.N)
        e[i] = 1e-6
        fd = (L(F + e, Fc, vr, vb) - L(F - e, Fc, vr, vb)) / 2e-6
        fdc = (L(F, Fc + e, vr, vb) - L(F, Fc - e, vr, vb)) / 2e-6
        assert abs(fd - dF[i]) <= 1e-6 * np.max(np.abs(dF))
        assert abs(fdc - dFc[i]) <= 1e-6 * np.max(np.abs(dFc))


# ------------------------------------------------- rotational broadening R
def _rot_setup(vrot_max=30.0, eps=0.6):
    grid = W.grid_for(1550.0, 1556.0, 3.0e5)
    x0, h = math.log(grid.lam_first_nm), math.log1p(1.0 / grid.R)
    xN = x0 + (grid.N - 1) * h
    xp = np.linspace(x0 + 0.2 * (xN - x0), xN - 0.2 * (xN - x0), 120)
    inst = I.Instrument(grid, np.exp(xp), np.full(120, 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)) * 22500.0)),
                        8.0, vrot_max_kms=vrot_max, limb_eps=eps)
    return grid, inst


@pytest.mark.parametrize("eps", [0.0, 0.6, 1.0])
def test_rotation_profile_is_the_disc_integral(eps):
    """The rotation profile is the flux of a linearly limb-darkened disc
    (I = 1 - eps + eps mu) integrated along the chord of constant projected
    velocity, over the disc's whole flux: both integrals by quadrature."""
    from scipy import integrate
    I0 = lambda mu: 1.0 - eps + eps * mu
    total = integrate.dblquad(lambda z, y: I0(math.sqrt(max(0.0, 1 - y * y - z * z))), -1, 1,
                              lambda y: -math.sqrt(1 - y * y), lambda y: math.sqrt(1 - y * y), epsabs=1e-12)[0]
    for y in (0.0, 0.3, 0.71, 0.95, -0.5):
        c = math.sqrt(1 - y * y)
        chord = integrate.quad(lambda z: I0(math.sqrt(max(0.0, 1 - y * y - z * z))), -c, c, epsabs=1e-13)[0]
        assert abs(I.rot_profile(y, eps) - chord / total) < 1e-9
    assert I.rot_profile(1.2, eps) == 0.0


@pytest.mark.parametrize("eps", [0.0, 0.6])
def test_rotation_cdf_and_cell_weights(eps):
    from scipy import integrate
    for y in (-1.0, -0.4, 0.0, 0.33, 0.9, 1.0, 1.5):
        ref = integrate.quad(lambda t: I.rot_profile(t, eps), -1, min(y, 1.0), epsabs=1e-13)[0]
        assert abs(I.rot_cdf(y, eps) - ref) < 1e-10
    for s in (0.3, 2.7, 11.4):
        r, dr = I.rot_weights(s, 14, eps)
        assert abs(r.sum() - 1) < 1e-13
        k = 3 if s > 3 else 0
        ref = integrate.quad(lambda u: I.rot_profile(u / s, eps) / s, k - 0.5, k + 0.5, epsabs=1e-13)[0]
        assert abs(r[14 + k] - ref) < 1e-10
        h = 1e-6 * s
        fd = (I.rot_weights(s + h, 14, eps)[0] - I.rot_weights(s - h, 14, eps)[0]) / (2 * h)
        np.testing.assert_allclose(dr, fd, atol=1e-7)
    r, dr = I.rot_weights(0.4, 3, eps)                   # narrower than a pixel: the identity
    np.testing.assert_array_equal(r, [0, 0, 0, 1, 0, 0, 0])
    np.testing.assert_array_equal(dr, 0.0)


def test_rotation_second_moment():
    """A delta line broadened by R has the profile's variance s^2 <y^2>, <y^2> =
    ((1 - eps)/4 + 2 eps/15) / (1 - eps/3), plus the cells' 1/12."""
    eps, s = 0.6, 40.0
    r, _ = I.rot_weights(s, 41, eps)
    k = np.arange(-41, 42)
    y2 = ((1 - eps) / 4 + 2 * eps / 15) / (1 - eps / 3)
    assert abs((r * k * k).sum() / (s * s * y2 + 1.0 / 12.0) - 1) < 2e-3
    assert abs((r * k).sum()) < 1e-12                     # symmetric


def test_rotation_keeps_a_constant_and_transposes():
    grid, inst = _rot_setup()
    one = np.ones(grid.N)
    KF, KFc, f = I.forward(inst, 3.0 * one, one, 5.0, 3.0, vsini=27.0)
    np.testing.assert_allclose(f, 3.0, rtol=1e-14)
    rng = np.random.default_rng(2)
    x, y = rng.normal(size=grid.N), rng.normal(size=grid.N)
    for s in (0.4, 6.2, inst.JR - 0.6):
        lhs = np.dot(I.rotate(x, s, inst.JR, inst.eps), y)
        rhs = np.dot(x, I._rotate_T(y, s, inst.JR, inst.eps))
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_rotation_adjoint_matches_finite_differences():
    """dL/dF, dL/dFc, dL/dv_r, dL/dv_b and dL/d(v sin i) of the chain K S R B
    against FP64 central differences."""
    grid, inst = _rot_setup()
    rng = np.random.default_rng(4)
    x = np.arange(grid.N)
    F = 1.0 - 0.6 * np.exp(-0.5 * ((x - grid.N / 2) / 9.0) ** 2) - 0.3 * np.exp(-0.5 * ((x - grid.N / 3) / 4.0) ** 2)
    Fc = 1.0 + 0.05 * np.sin(x / 500.0)
    vr, vb, vs = 7.3, 4.1, 18.5
    g = rng.normal(size=inst.lam_obs_nm.size)
    L = lambda *a: float(np.dot(I.forward(inst, *a)[2], g))
    dF, dFc, gvr, gvb, gvs = I.adjoint(inst, F, Fc, vr, vb, g, vsini=vs)
    h = 1e-4
    for val, fd in ((gvr, (L(F, Fc, vr + h, vb, vs) - L(F, Fc, vr - h, vb, vs)) / (2 * h)),
                    (gvb, (L(F, Fc, vr, vb + h, vs) - L(F, Fc, vr, vb - h, vs)) / (2 * h)),
                    (gvs, (L(F, Fc, vr, vb, vs + h) - L(F, Fc, vr, vb, vs - h)) / (2 * h))):
        assert abs(val - fd) <= 1e-6 * max(abs(fd), 1e-3), (val, fd)
    for i in rng.choice(grid.N, 6, replace=False):
        e = np.zeros(grid.N)
        e[i] = 1e-6
        fdF = (L(F + e, Fc, vr, vb, vs) - L(F - e, Fc, vr, vb, vs)) / 2e-6
        fdFc = (L(F, Fc + e, vr, vb, vs) - L(F, Fc - e, vr, vb, vs)) / 2e-6
        assert abs(dF[i] - fdF) <= 1e-6 * max(abs(fdF), 1e-6)
        assert abs(dFc[i] - fdFc) <= 1e-6 * max(abs(fdFc), 1e-6)
