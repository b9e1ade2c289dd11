"""FP64 CPU oracle of the instrument operator (Sec. 2.1 Eq. 9; Sec. 7 Eq. 31).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It shares no code with the
GPU library.

Eq. 31 maps the native total and continuum fluxes to observed pixels before
the ratio is taken,

    f_p = {K S(v_r) B(v_b) F}_p / {K S(v_r) B(v_b) F_c}_p ,

with B a Gaussian broadening on the logarithmic synthesis grid, S the Doppler
shift and K the wavelength-dependent line-spread function with the sampling
onto observed pixels.  The paper describes these operators but not their
discretisation; this module is the reading used (all three act on
x = ln lambda, native x_i = x_0 + i h, h = ln(1 + 1/R)):

  B   (B G)_i = sum_j g(i - j) G_j / sum_j g(i - j) over |i - j| <= J,
      g(k) = exp(-k^2 / (2 sigma^2)), sigma = v_b / (c h) pixels (v_b is the
      Gaussian velocity dispersion); the support J is fixed by the operator
      (from its largest v_b), and near the grid ends the weights are
      renormalised over the pixels that exist.
  S   (S G)_i = G at fractional pixel i - t, t = ln(1 + v_r/c) / h, by linear
      interpolation, the index clamped to the grid (flat extension).
  R   rotational broadening (optional; the paper names a GPU-resident
      rotational kernel without defining it): (R G)_i = sum_k r_k G_{i-k} /
      sum_k r_k over the pixels that exist, with r_k the integral over the
      cell [k - 1/2, k + 1/2] (in pixels) of the classical rotation profile
      of a linearly limb-darkened disc (Gray, The Observation and Analysis of
      Stellar Photospheres), in y = u / s, s = v sin i / (c h) pixels:
          G(y) = [2 (1 - eps) sqrt(1 - y^2) + (pi eps / 2)(1 - y^2)]
                 / [pi (1 - eps/3)],   |y| <= 1,
      whose antiderivative is closed form; applied after B:
          f = K S R B F / K S R B F_c.
  K   (K H)_p = sum_i w_pi H_i / sum_i w_pi over |x_i - x_p| <= T sigma_p,
      w_pi = exp(-(x_i - x_p)^2 / (2 sigma_p^2)), sigma_p the LSF width of
      observed pixel p in ln lambda (a Gaussian LSF sampled at the pixel
      centre; the paper's calibration-derived LSF is not available).

Velocities in km/s.
"""
from __future__ import annotations

import math

import numpy as np

C_KMS = 299792.458


class Instrument:
    """Observed pixels (centres lam_obs_nm), LSF widths sigma_ln (ln lambda),
    the LSF truncation T (in sigmas) and the broadening support from vb_max."""

    def __init__(self, grid, lam_obs_nm, sigma_ln, vb_max_kms, trunc=4.0, vrot_max_kms=0.0, limb_eps=0.6):
        self.grid = grid
        self.h = math.log1p(1.0 / grid.R)
        # rotation support: cells [k - 1/2, k + 1/2] that reach |u| <= s_max
        self.JR = int(math.ceil(vrot_max_kms / C_KMS / self.h + 0.5)) if vrot_max_kms > 0 else 0
        self.eps = float(limb_eps)
        self.x0 = math.log(grid.lam_first_nm)
        self.lam_obs_nm = np.asarray(lam_obs_nm, np.float64)
        self.sigma_ln = np.asarray(sigma_ln, np.float64)
        self.trunc = float(trunc)
        self.J = int(math.ceil(4.0 * vb_max_kms / C_KMS / self.h))
        # LSF support of each observed pixel on the native grid
        xp = np.log(self.lam_obs_nm)
        self.lo = np.maximum(0, np.ceil((xp - self.trunc * self.sigma_ln - self.x0) / self.h).astype(np.int64))
        self.hi = np.minimum(grid.N - 1, np.floor((xp + self.trunc * self.sigma_ln - self.x0) / self.h).astype(np.int64))


def broaden(G, sigma_px, J):
    """B: renormalised truncated Gaussian convolution on the native grid."""
    N = G.shape[-1]
    out = np.zeros_like(G)
    Z = np.zeros(N)
    for k in range(-J, J + 1):
        w = math.exp(-k * k / (2.0 * sigma_px * sigma_px))
        i0, i1 = max(0, k), min(N, N + k)          # i with 0 <= i - k < N
        out[..., i0:i1] += w * G[..., i0 - k:i1 - k]
        Z[i0:i1] += w
    return out / Z


def shift(G, t_px):
    """S: G at fractional pixel i - t by linear interpolation, index clamped."""
    N = G.shape[-1]
    pos = np.arange(N) - t_px
    k = np.floor(pos).astype(np.int64)
    f = pos - k
    k0 = np.clip(k, 0, N - 1)
    k1 = np.clip(k + 1, 0, N - 1)
    return (1.0 - f) * G[..., k0] + f * G[..., k1]


def lsf_weights(inst, p):
    """Native indices and normalised weights of observed pixel p."""
    i = np.arange(inst.lo[p], inst.hi[p] + 1)
    x = inst.x0 + i * inst.h
    w = np.exp(-(x - math.log(inst.lam_obs_nm[p])) ** 2 / (2.0 * inst.sigma_ln[p] ** 2))
    return i, w / w.sum()


def apply_lsf(inst, H):
    out = np.zeros(H.shape[:-1] + (inst.lam_obs_nm.size,))
    for p in range(inst.lam_obs_nm.size):
        i, w = lsf_weights(inst, p)
        out[..., p] = H[..., i] @ w
    return out


def rot_profile(y, eps):
    """The rotation profile G(y), |y| <= 1, normalised to unit integral."""
    y = np.asarray(y, np.float64)
    q = np.clip(1.0 - y * y, 0.0, None)
    return (2.0 * (1.0 - eps) * np.sqrt(q) + 0.5 * math.pi * eps * q) / (math.pi * (1.0 - eps / 3.0))


def rot_cdf(y, eps):
    """Integral of G from -1 to y (clamped to [-1, 1])."""
    y = np.clip(np.asarray(y, np.float64), -1.0, 1.0)
    a = (1.0 - eps) * (y * np.sqrt(1.0 - y * y) + np.arcsin(y))
    b = 0.5 * math.pi * eps * (y - y ** 3 / 3.0)
    return (a + b) / (math.pi * (1.0 - eps / 3.0)) + 0.5


def rot_weights(s_px, J, eps):
    """Cell integrals r_k, k = -J..J, of the profile scaled to half-width s_px
    pixels, and their derivatives dr_k/ds (a delta at k = 0 for s below 1/2)."""
    k = np.arange(-J, J + 1, dtype=np.float64)
    if s_px <= 0.0:
        return (k == 0).astype(np.float64), np.zeros_like(k)
    lo, hi = (k - 0.5) / s_px, (k + 0.5) / s_px
    r = rot_cdf(hi, eps) - rot_cdf(lo, eps)
    # d/ds of the bounds y = b/s is -y/s; a bound clamped at +-1 does not move
    dlo = np.where(np.abs(lo) < 1.0, rot_profile(lo, eps) * (-lo / s_px), 0.0)
    dhi = np.where(np.abs(hi) < 1.0, rot_profile(hi, eps) * (-hi / s_px), 0.0)
    return r, dhi - dlo


def rotate(G, s_px, J, eps):
    """R: renormalised convolution with the rotation cell weights."""
    if J == 0:
        return np.array(G, np.float64)
    r, _ = rot_weights(s_px, J, eps)
    N = G.shape[-1]
    out = np.zeros_like(G)
    Z = np.zeros(N)
    for k, w in zip(range(-J, J + 1), r):
        if w == 0.0:
            continue
        i0, i1 = max(0, k), min(N, N + k)
        out[..., i0:i1] += w * G[..., i0 - k:i1 - k]
        Z[i0:i1] += w
    return out / Z


def operator_params(inst, v_r, v_b):
    return v_b / C_KMS / inst.h, math.log1p(v_r / C_KMS) / inst.h


def forward(inst, F, Fc, v_r, v_b, vsini=0.0):
    """(K S R B F, K S R B Fc, f) at the observed pixels (Eq. 31; R only with a rotation support)."""
    sig, t = operator_params(inst, v_r, v_b)
    sr = vsini / C_KMS / inst.h
    op = lambda G: apply_lsf(inst, shift(rotate(broaden(np.asarray(G, np.float64), sig, inst.J), sr, inst.JR,
                                                inst.eps), t))
    KF, KFc = op(F), op(Fc)
    return KF, KFc, KF / KFc


# ------------------------------------------------------------------ adjoint
def _lsf_T(inst, dY, N):
    out = np.zeros(dY.shape[:-1] + (N,))
    for p in range(inst.lam_obs_nm.size):
        i, w = lsf_weights(inst, p)
        out[..., i] += dY[..., p, None] * w
    return out


def _shift_T(dG, t_px):
    N = dG.shape[-1]
    pos = np.arange(N) - t_px
    k = np.floor(pos).astype(np.int64)
    f = pos - k
    out = np.zeros_like(dG)
    np.add.at(out.T, np.clip(k, 0, N - 1), ((1.0 - f) * dG).T)
    np.add.at(out.T, np.clip(k + 1, 0, N - 1), (f * dG).T)
    return out


def _dshift_dt(G, t_px):
    """d(S G)/dt: the interpolation slope, zero where the index is clamped."""
    N = G.shape[-1]
    pos = np.arange(N) - t_px
    k = np.floor(pos).astype(np.int64)
    inside = (k >= 0) & (k + 1 <= N - 1)
    k0 = np.clip(k, 0, N - 1)
    k1 = np.clip(k + 1, 0, N - 1)
    return np.where(inside, -(G[..., k1] - G[..., k0]), 0.0)


def _broaden_T(dG, sigma_px, J):
    N = dG.shape[-1]
    Z = np.zeros(N)
    for k in range(-J, J + 1):
        w = math.exp(-k * k / (2.0 * sigma_px * sigma_px))
        i0, i1 = max(0, k), min(N, N + k)
        Z[i0:i1] += w
    a = dG / Z
    out = np.zeros_like(dG)
    for k in range(-J, J + 1):
        w = math.exp(-k * k / (2.0 * sigma_px * sigma_px))
        i0, i1 = max(0, k), min(N, N + k)
        out[..., i0 - k:i1 - k] += w * a[..., i0:i1]
    return out


def _dbroaden_dsigma(G, sigma_px, J):
    """d(B G)_i / d sigma with B G = sum g G / sum g, dg/dsigma = g k^2 / sigma^3."""
    N = G.shape[-1]
    num = np.zeros_like(G)
    dnum = np.zeros_like(G)
    Z = np.zeros(N)
    dZ = np.zeros(N)
    for k in range(-J, J + 1):
        w = math.exp(-k * k / (2.0 * sigma_px * sigma_px))
        dw = w * k * k / sigma_px ** 3
        i0, i1 = max(0, k), min(N, N + k)
        num[..., i0:i1] += w * G[..., i0 - k:i1 - k]
        dnum[..., i0:i1] += dw * G[..., i0 - k:i1 - k]
        Z[i0:i1] += w
        dZ[i0:i1] += dw
    return (dnum * Z - num * dZ) / Z ** 2


def _rotate_T(dG, s_px, J, eps):
    if J == 0:
        return np.array(dG, np.float64)
    r, _ = rot_weights(s_px, J, eps)
    N = dG.shape[-1]
    Z = np.zeros(N)
    for k, w in zip(range(-J, J + 1), r):
        i0, i1 = max(0, k), min(N, N + k)
        Z[i0:i1] += w
    a = dG / Z
    out = np.zeros_like(dG)
    for k, w in zip(range(-J, J + 1), r):
        i0, i1 = max(0, k), min(N, N + k)
        out[..., i0 - k:i1 - k] += w * a[..., i0:i1]
    return out


def _drotate_ds(G, s_px, J, eps):
    """d(R G)_i / ds with R G = sum r G / sum r."""
    r, dr = rot_weights(s_px, J, eps)
    N = G.shape[-1]
    num = np.zeros_like(G)
    dnum = np.zeros_like(G)
    Z = np.zeros(N)
    dZ = np.zeros(N)
    for k, w, dw in zip(range(-J, J + 1), r, dr):
        i0, i1 = max(0, k), min(N, N + k)
        num[..., i0:i1] += w * G[..., i0 - k:i1 - k]
        dnum[..., i0:i1] += dw * G[..., i0 - k:i1 - k]
        Z[i0:i1] += w
        dZ[i0:i1] += dw
    return (dnum * Z - num * dZ) / Z ** 2


def adjoint(inst, F, Fc, v_r, v_b, dL_df, vsini=0.0):
    """VJP of f = K S R B F / K S R B Fc: (dL/dF, dL/dFc, dL/dv_r, dL/dv_b), and
    dL/d(v sin i) as a fifth entry when the instrument has a rotation support."""
    F = np.asarray(F, np.float64)
    Fc = np.asarray(Fc, np.float64)
    sig, t = operator_params(inst, v_r, v_b)
    sr = vsini / C_KMS / inst.h
    N = F.size
    BF, BFc = broaden(F, sig, inst.J), broaden(Fc, sig, inst.J)
    RBF, RBFc = rotate(BF, sr, inst.JR, inst.eps), rotate(BFc, sr, inst.JR, inst.eps)
    SRBF, SRBFc = shift(RBF, t), shift(RBFc, t)
    KF, KFc = apply_lsf(inst, SRBF), apply_lsf(inst, SRBFc)
    dKF = dL_df / KFc
    dKFc = -dL_df * KF / KFc ** 2
    dSF, dSFc = _lsf_T(inst, dKF, N), _lsf_T(inst, dKFc, N)
    # v_r: through the shift t = ln(1 + v_r/c) / h
    dt = np.sum(dSF * _dshift_dt(RBF, t)) + np.sum(dSFc * _dshift_dt(RBFc, t))
    g_vr = dt / (inst.h * (C_KMS + v_r))
    dRF, dRFc = _shift_T(dSF, t), _shift_T(dSFc, t)
    # v sin i: through s = v sin i / (c h)
    g_rot = None
    if inst.JR:
        dsr = (np.sum(dRF * _drotate_ds(BF, sr, inst.JR, inst.eps)) +
               np.sum(dRFc * _drotate_ds(BFc, sr, inst.JR, inst.eps)))
        g_rot = dsr / (C_KMS * inst.h)
    dBF, dBFc = _rotate_T(dRF, sr, inst.JR, inst.eps), _rotate_T(dRFc, sr, inst.JR, inst.eps)
    # v_b: through sigma = v_b / (c h)
    ds = np.sum(dBF * _dbroaden_dsigma(F, sig, inst.J)) + np.sum(dBFc * _dbroaden_dsigma(Fc, sig, inst.J))
    g_vb = ds / (C_KMS * inst.h)
    out = (_broaden_T(dBF, sig, inst.J), _broaden_T(dBFc, sig, inst.J), g_vr, g_vb)
    return out + (g_rot,) if inst.JR else out
