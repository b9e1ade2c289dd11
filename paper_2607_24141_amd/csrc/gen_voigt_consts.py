"""Writes voigt_consts.h: constants of the device Voigt evaluator.

Regions of z = v + i a (float32 unless noted):

* wing, |z| >= 5.5: Gauss-Hermite quadrature of the Voigt integral
  H(a,v) = (a/pi) int exp(-t^2)/((v-t)^2+a^2) dt with the +/-t_k node pairs
  combined so every term is positive,
      H ~= (2a/pi) sum_k w_k (u + a^2 + t_k^2) / ((u - a^2 - t_k^2)^2 + 4 u a^2),
  u = v^2.  Three tiers: 6 nodes for 5.5 <= |z| < 8, 4 nodes for
  8 <= |z| < 40, 2 nodes beyond (max relative error ~1.4e-6 in each).
* core with small damping, |z| < 5.5 and a <= 0.15: the expansion of
  w(v + ia) in powers of a about the real axis,
      w = exp(-z^2) + (2i/sqrt(pi)) F(z),   F = Dawson's integral,
      H = exp(a^2-u) cos(2av) - (2/sqrt(pi)) [a F' - a^3 F'''/6 + a^5 F^(5)/120]
      L = -exp(a^2-u) sin(2av) + (2/sqrt(pi)) [F - a^2 F''/2 + a^4 F''''/24],
  with each derivative of F (even ones divided by v) replaced by a rational
  function of u fitted here on [0, 30.25]; reference values from mpmath at
  40 digits.  The Gaussian part carries the exact real-axis value, so H keeps
  its relative accuracy where exp(-v^2) and the damping term are comparable.
  The opacity kernel evaluates the same series for H with piecewise
  polynomials instead: |v| in [0, 5.5] is cut into PW_N intervals, and on
  each the damping terms Lam0, Lam2, Lam4 are Chebyshev interpolants of
  degree 5, 4, 2 in t = |v| - (interval centre), stored as monomial
  coefficients (16 floats per interval, read from LDS): no division and
  short Horner chains.
* core with larger damping: Weideman's 32-term rational expansion of w(z)
  (J.A.C. Weideman, SIAM J. Numer. Anal. 31 (1994) 1497) in float64.

Run:  python gen_voigt_consts.py > voigt_consts.h
"""
import numpy as np

N_W = 32
U_MAX = 30.25
A_SMALL = 0.15
A_TINY = 0.03      # a <= A_TINY: the a^5 terms (and the t^4 term of cos 2av) are dropped


def weideman(N):
    M = 2 * N
    k = np.arange(-M + 1, M)
    L = np.sqrt(N / np.sqrt(2.0))
    t = L * np.tan(k * np.pi / (2 * M))
    f = np.concatenate([[0.0], np.exp(-t * t) * (L * L + t * t)])
    a = np.real(np.fft.fft(np.fft.fftshift(f))) / (2 * M)
    return L, a[1:N + 1][::-1]          # highest power first (Horner order)


def dawson_derivs(v):
    """F, F', ..., F^(5) of Dawson's integral at v (mpmath, 40 digits)."""
    import mpmath as mp
    mp.mp.dps = 40
    out = np.zeros((6, len(v)))
    for i, x in enumerate(v):
        x = mp.mpf(x)
        F0 = mp.sqrt(mp.pi) / 2 * mp.exp(-x * x) * mp.erfi(x)
        d = [F0, 1 - 2 * x * F0]
        for n in range(1, 5):          # F^(n+1) = -2 v F^(n) - 2 n F^(n-1)
            d.append(-2 * x * d[n] - 2 * n * d[n - 1])
        out[:, i] = [float(y) for y in d]
    return out


def ratfit(u, f, m, n, wt, iters=40):
    """P/Q (deg m, n; Q(0) = 1) minimising the weighted max error (SK + Lawson)."""
    Qp = np.ones_like(u)
    w2 = np.ones_like(u)
    for _ in range(iters):
        A = np.hstack([np.vstack([u ** k for k in range(m + 1)]).T,
                       -(f[:, None]) * np.vstack([u ** k for k in range(1, n + 1)]).T])
        W = (wt * w2 / Qp)[:, None]
        c, *_ = np.linalg.lstsq(A * W, f * W[:, 0], rcond=None)
        p, q = c[:m + 1], np.concatenate([[1.0], c[m + 1:]])
        P, Q = np.polyval(p[::-1], u), np.polyval(q[::-1], u)
        err = np.abs((P / Q - f) * wt)
        Qp = Q
        w2 = w2 * (err / err.max()) ** 0.3 + 1e-12
        w2 /= w2.max()
    return p, q, err.max()


def horner32(c, u):
    r = np.zeros_like(u, dtype=np.float32)
    for x in c[::-1].astype(np.float32):
        r = r * u.astype(np.float32) + x
    return r


def fit_fixed_q(u, f, q, m, wt, iters=30):
    """Numerator of degree m for a given denominator q, minimising the weighted max error."""
    Q = np.polyval(q[::-1], u)
    A = np.vstack([u ** j for j in range(m + 1)]).T
    w2 = np.ones_like(u)
    for _ in range(iters):
        W = (wt / Q * w2)[:, None]
        c, *_ = np.linalg.lstsq(A * W, f * Q * W[:, 0], rcond=None)
        err = np.abs((A @ c / Q - f) * wt)
        w2 = w2 * (err / err.max()) ** 0.3 + 1e-12
        w2 /= w2.max()
    return c, err.max()


def fits():
    """Common-denominator fits: Lam_k = P_k / Q (H terms), Mu_k = R_k / S (L terms)."""
    v = np.linspace(0.0, np.sqrt(U_MAX), 1501)
    u = v * v
    F = dawson_derivs(v)
    sp = 2.0 / np.sqrt(np.pi)
    vv = np.where(v > 0, v, 1.0)
    lam = [-sp * F[1], sp * F[3] / 6.0, -sp * F[5] / 120.0]
    # odd derivatives divided by v, with their limits at v = 0 (1, -4, 32)
    mu0 = np.where(v > 0, F[0] / vv, 1.0)
    mu2 = np.where(v > 0, F[2] / vv, -4.0)
    mu4 = np.where(v > 0, F[4] / vv, 32.0)
    mus = [sp * mu0, -sp * mu2 / 2.0, sp * mu4 / 24.0]
    a = A_SMALL
    H = np.exp(a * a - u) * np.cos(2 * a * v) + a * (lam[0] + a * a * lam[1] + a ** 4 * lam[2])
    res = {}
    p0, q, e0 = ratfit(u, lam[0], 7, 8, a / H)
    res["LAM_Q"] = (q, 0.0)
    res["LAM_P0"] = (p0, e0)
    for k, m in ((1, 8), (2, 7)):
        c, e = fit_fixed_q(u, lam[k], q, m, a ** (2 * k + 1) / H)
        res["LAM_P%d" % (2 * k)] = (c, e)
    Lref = np.abs(-np.exp(a * a - u) * np.sin(2 * a * v) + v * (mus[0] + a * a * mus[1] + a ** 4 * mus[2]))
    Lw = np.maximum(v, 1e-3) / np.maximum(Lref, 0.05)
    r0, sq, e0 = ratfit(u, mus[0], 6, 7, Lw)
    res["MU_Q"] = (sq, 0.0)
    res["MU_P0"] = (r0, e0)
    for k, m in ((1, 7), (2, 6)):
        c, e = fit_fixed_q(u, mus[k], sq, m, a ** (2 * k) * Lw)
        res["MU_P%d" % (2 * k)] = (c, e)
    # float32 check of the assembled small-damping H at a = A_SMALL
    f32 = np.float32
    Qv = horner32(res["LAM_Q"][0], u)
    num = horner32(res["LAM_P0"][0], u) + f32(a * a) * (horner32(res["LAM_P2"][0], u) +
                                                         f32(a * a) * horner32(res["LAM_P4"][0], u))
    H32 = np.exp(a * a - u) * np.cos(2 * a * v) + a * (num / Qv).astype(np.float64)
    res["check_H"] = np.max(np.abs(H32 - H) / H)
    # the reduced form for a <= A_TINY against the full series at a = A_TINY
    b = A_TINY
    Hb = np.exp(b * b - u) * np.cos(2 * b * v) + b * (lam[0] + b * b * lam[1] + b ** 4 * lam[2])
    t = 4.0 * b * b * u
    cs3 = 1.0 - t / 2.0 + t * t / 24.0 - t ** 3 / 720.0
    numb = horner32(res["LAM_P0"][0], u) + f32(b * b) * horner32(res["LAM_P2"][0], u)
    Hb32 = np.exp(b * b - u) * cs3 + b * (numb / Qv).astype(np.float64)
    res["check_H_tiny"] = np.max(np.abs(Hb32 - Hb) / Hb)
    return res


PW_N = 16
PW_DEG = (5, 4, 2)


def pw_tables():
    """Per interval k of |v| in [0, U_MAX^(1/2)]: [A0..A3 | A4 A5 B0 B1 | B2 B3 B4 c | C0 C1 C2 0]
    with Lam0 ~ sum A_n t^n, Lam2 ~ sum B_n t^n, Lam4 ~ sum C_n t^n, t = |v| - c."""
    vmax = np.sqrt(U_MAX)
    h = vmax / PW_N
    sp = 2.0 / np.sqrt(np.pi)
    tab = np.zeros((PW_N, 16))
    for k in range(PW_N):
        c = (k + 0.5) * h
        coefs = []
        for i, d in enumerate(PW_DEG):
            x = np.cos((2 * np.arange(d + 1) + 1) * np.pi / (2 * (d + 1)))
            t = 0.5 * h * x
            F = dawson_derivs(c + t)
            y = [-sp * F[1], sp * F[3] / 6.0, -sp * F[5] / 120.0][i]
            coefs.append(np.linalg.solve(np.vander(t, d + 1, increasing=True), y))
        A, B, Cc = coefs
        tab[k] = [A[0], A[1], A[2], A[3], A[4], A[5], B[0], B[1], B[2], B[3], B[4], c, Cc[0], Cc[1], Cc[2], 0.0]
    return h, tab


def pw_check(h, tab):
    """Max relative error of the float32 piecewise H against wofz for a in (0, A_SMALL]."""
    from scipy.special import wofz
    f32 = np.float32
    t32 = tab.astype(f32)
    worst = {}
    for a, full in ((A_SMALL, True), (0.1, True), (A_TINY, False), (1e-2, False), (1e-3, False), (1e-5, False)):
        v = np.linspace(0.0, np.sqrt(U_MAX), 20001)[:-1]
        v = v[v * v + a * a < U_MAX]
        av = v.astype(f32)
        k = np.minimum((av * f32(1.0 / h)).astype(np.int32), PW_N - 1)
        T = t32[k]
        t = av - T[:, 11]
        L0 = T[:, 5]
        for n in (4, 3, 2, 1, 0):
            L0 = L0 * t + T[:, n]
        L2 = T[:, 10]
        for n in (9, 8, 7, 6):
            L2 = L2 * t + T[:, n]
        L4 = (T[:, 14] * t + T[:, 13]) * t + T[:, 12]
        a2 = f32(a * a)
        num = L0 + a2 * (L2 + a2 * L4) if full else L0 + a2 * L2
        u = av * av
        tt = f32(4) * a2 * u
        cs = 1 - tt / 2 + tt * tt / 24 - tt ** 3 / 720 + (tt ** 4 / 40320 if full else 0)
        H = np.exp(a2 - u).astype(np.float64) * cs + a * num.astype(np.float64)
        ref = wofz(v + 1j * a).real
        worst[a] = np.max(np.abs(H - ref) / ref)
    return worst


def arr(name, c, typ="float", fmt="%.9ef"):
    return "__device__ static constexpr %s %s[%d] = {%s};" % (typ, name, len(c), ", ".join(fmt % x for x in c))


def main():
    out = ["// Generated by gen_voigt_consts.py -- do not edit.", "#pragma once", ""]
    out.append("#define PZ_VOIGT_WING_R2 30.25f   /* |z|^2 below which the core formulas apply */")
    out.append("#define PZ_VOIGT_TIER2_R2 64.0f   /* |z| >= 8: four-node wing */")
    out.append("#define PZ_VOIGT_TIER3_R2 1600.0f /* |z| >= 40: two-node wing */")
    out.append("#define PZ_VOIGT_A2_SMALL %.6ef  /* a^2 <= this (a <= %.2f): float32 small-damping core */"
               % (A_SMALL ** 2, A_SMALL))
    out.append("#define PZ_VOIGT_A2_TINY %.6ef   /* a^2 <= this (a <= %.2f): core without the a^5 terms */"
               % (A_TINY ** 2, A_TINY))
    for n, tag in ((6, "GH6"), (4, "GH4"), (2, "GH2")):
        t, w = np.polynomial.hermite.hermgauss(n)
        pos = t > 0
        out.append(arr("PZ_%s_T2" % tag, t[pos] ** 2))
        out.append(arr("PZ_%s_W" % tag, w[pos] * 2.0 / np.pi) + "  /* w_k * 2/pi */")
    res = fits()
    out.append("/* small-damping core: max relative error of H at a = %.2f vs the truncated series: %.1e */"
               % (A_SMALL, res["check_H"]))
    out.append("/* reduced core (no a^5 terms) at a = %.2f vs the full series: %.1e */" % (A_TINY, res["check_H_tiny"]))
    for name in ("LAM_Q", "LAM_P0", "LAM_P2", "LAM_P4", "MU_Q", "MU_P0", "MU_P2", "MU_P4"):
        c, e = res[name]
        out.append(arr("PZ_%s" % name, c) + ("  /* weighted max error %.1e */" % e if e else ""))
    h, tab = pw_tables()
    worst = pw_check(h, tab)
    out.append("/* piecewise core for the opacity: %d intervals of |v|, degrees %s; max relative error of H"
               % (PW_N, PW_DEG))
    out.append("   against wofz (float32 evaluation, includes the float32 exp): %s */"
               % ", ".join("a=%g: %.1e" % (k, v) for k, v in worst.items()))
    out.append("static constexpr int PZ_PW_N = %d;" % PW_N)
    out.append("#define PZ_PW_INV_H %.9ef" % (1.0 / h))
    out.append("__device__ static constexpr float PZ_PW_TAB[%d] = {" % (PW_N * 16))
    out += ["    " + ", ".join("%.9ef" % x for x in row) + "," for row in tab]
    out.append("};")
    L, c = weideman(N_W)
    out.append("static constexpr int PZ_WEID_N = %d;" % N_W)
    out.append("#define PZ_WEID_L %.17e" % L)
    out.append("__device__ static constexpr double PZ_WEID_C[%d] = {" % N_W)
    out += ["    %.17e," % x for x in c]
    out.append("};")
    print("\n".join(out))


if __name__ == "__main__":
    main()
