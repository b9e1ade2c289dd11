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

    def __init__(self, grid, lam_obs_nm, sigma_ln, vb_max_kms, trunc=4.0):
        self.grid = grid
        self.h = math.log1p(1.0 / grid.R)
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


def operator_params(inst, v_r, v_b):
    return v_b / C_KMS / inst.h, math.log1p(v_r / C_KMS) / inst.h


def forward(inst, F, Fc, v_r, v_b):
    """(K S B F, K S B Fc, f) at the observed pixels (Eq. 31)."""
    sig, t = operator_params(inst, v_r, v_b)
    KF = apply_lsf(inst, shift(broaden(np.asarray(F, np.float64), sig, inst.J), t))
    KFc = apply_lsf(inst, shift(broaden(np.asarray(Fc, np.float64), sig, inst.J), t))
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


def adjoint(inst, F, Fc, v_r, v_b, dL_df):
    """VJP of f = K S B F / K S B Fc: (dL/dF, dL/dFc, dL/dv_r, dL/dv_b)."""
    F = np.asarray(F, np.float64)
    Fc = np.asarray(Fc, np.float64)
    sig, t = operator_params(inst, v_r, v_b)
    N = F.size
    BF, BFc = broaden(F, sig, inst.J), broaden(Fc, sig, inst.J)
    SBF, SBFc = shift(BF, t), shift(BFc, t)
    KF, KFc = apply_lsf(inst, SBF), apply_lsf(inst, SBFc)
    dKF = dL_df / KFc
    dKFc = -dL_df * KF / KFc ** 2
    dSBF, dSBFc = _lsf_T(inst, dKF, N), _lsf_T(inst, dKFc, N)
    # v_r: through the shift t = ln(1 + v_r/c) / h
    dt = np.sum(dSBF * _dshift_dt(BF, t)) + np.sum(dSBFc * _dshift_dt(BFc, t))
    g_vr = dt / (inst.h * (C_KMS + v_r))
    dBF, dBFc = _shift_T(dSBF, t), _shift_T(dSBFc, t)
    # v_b: through sigma = v_b / (c h)
    ds = np.sum(dBF * _dbroaden_dsigma(F, sig, inst.J)) + np.sum(dBFc * _dbroaden_dsigma(Fc, sig, inst.J))
    g_vb = ds / (C_KMS * inst.h)
    return _broaden_T(dBF, sig, inst.J), _broaden_T(dBFc, sig, inst.J), g_vr, g_vb
