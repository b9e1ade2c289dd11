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
      L = -exp(a^2-u) sin(2av) + (2/sqrt(pi)) [F - a^2 F''/2 + a^4 F''''/24].
  The Gaussian part carries the exact real-axis value, so H keeps its
  relative accuracy where exp(-v^2) and the damping term are comparable.
  The damping terms (derivatives of F, the even ones divided by v) are
  piecewise polynomials: |v| in [0, 5.5] is cut into PW_N intervals, and on
  each they are Chebyshev interpolants of degree 5, 4, 2 (for the a, a^3,
  a^5 terms) in t = |v| - (interval centre), from mpmath values at 40
  digits, stored as monomial coefficients (16 floats per interval, read from
  LDS): no division and short Horner chains.  For a <= A_TINY the a^5 terms
  are below 5e-8 of H and are dropped.
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


PW_N = 16
PW_DEG = (5, 4, 2)


def pw_tables():
    """Per interval k of |v| in [0, U_MAX^(1/2)], for the damping terms of H (Lam) and
    of L/v (Mu): [P0_0..P0_3 | P0_4 P0_5 P2_0 P2_1 | P2_2 P2_3 P2_4 c | P4_0 P4_1 P4_2 0]
    with P0 ~ sum P0_n t^n (degree 5), P2 (degree 4), P4 (degree 2), t = |v| - c."""
    vmax = np.sqrt(U_MAX)
    h = vmax / PW_N
    sp = 2.0 / np.sqrt(np.pi)

    def terms(v):
        F = dawson_derivs(v)
        lam = [-sp * F[1], sp * F[3] / 6.0, -sp * F[5] / 120.0]
        mu = [sp * F[0] / v, -sp * F[2] / (2.0 * v), sp * F[4] / (24.0 * v)]
        return lam, mu

    tabs = np.zeros((2, PW_N, 16))
    for k in range(PW_N):
        c = (k + 0.5) * h
        for i, d in enumerate(PW_DEG):
            x = np.cos((2 * np.arange(d + 1) + 1) * np.pi / (2 * (d + 1)))
            t = 0.5 * h * x                      # Chebyshev nodes avoid v = 0 exactly
            lam, mu = terms(c + t)
            V = np.vander(t, d + 1, increasing=True)
            for j, y in enumerate((lam[i], mu[i])):
                co = np.linalg.solve(V, y)
                slot = (0, 6, 12)[i]
                tabs[j, k, slot:slot + d + 1] = co
        tabs[:, k, 11] = c
    # the layout above puts P2 at slots 6..10 and P4 at 12..14; c at 11
    return h, tabs[0], tabs[1]


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


def pw_check_L(h, tab):
    """Max error of the float32 piecewise L = Im w relative to |w| (wofz)."""
    from scipy.special import wofz
    f32 = np.float32
    t32 = tab.astype(f32)
    worst = {}
    for a, full in ((A_SMALL, True), (0.1, True), (A_TINY, False), (1e-2, False), (1e-3, False)):
        v = np.linspace(0.0, np.sqrt(U_MAX), 20001)[:-1]
        v = v[v * v + a * a < U_MAX]
        av = v.astype(f32)
        k = np.minimum((av * f32(1.0 / h)).astype(np.int32), PW_N - 1)
        T = t32[k]
        t = av - T[:, 11]
        P0 = T[:, 5]
        for n in (4, 3, 2, 1, 0):
            P0 = P0 * t + T[:, n]
        P2 = T[:, 10]
        for n in (9, 8, 7, 6):
            P2 = P2 * t + T[:, n]
        P4 = (T[:, 14] * t + T[:, 13]) * t + T[:, 12]
        a2 = f32(a * a)
        num = P0 + a2 * (P2 + a2 * P4) if full else P0 + a2 * P2
        u = av * av
        tt = f32(4) * a2 * u
        sn = 1 - tt / 6 + tt * tt / 120 - tt ** 3 / 5040 + (tt ** 4 / 362880 if full else 0)
        L = v * (num.astype(np.float64) - np.exp(a2 - u).astype(np.float64) * 2 * a * sn)
        ref = wofz(v + 1j * a)
        worst[a] = np.max(np.abs(L - ref.imag) / np.abs(ref))
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
    h, tab, tab_mu = pw_tables()
    worst = pw_check(h, tab)
    worst_l = pw_check_L(h, tab_mu)
    out.append("/* piecewise small-damping core, H terms: %d intervals of |v|, degrees %s; max relative error of H"
               % (PW_N, PW_DEG))
    out.append("   against wofz (float32 evaluation, includes the float32 exp): %s */"
               % ", ".join("a=%g: %.1e" % (k, v) for k, v in worst.items()))
    out.append("static constexpr int PZ_PW_N = %d;" % PW_N)
    out.append("#define PZ_PW_INV_H %.9ef" % (1.0 / h))
    out.append("__device__ static constexpr float PZ_PW_TAB[%d] = {" % (PW_N * 16))
    out += ["    " + ", ".join("%.9ef" % x for x in row) + "," for row in tab]
    out.append("};")
    out.append("/* the same for L = Im w (adjoint): max error of L relative to |w|: %s */"
               % ", ".join("a=%g: %.1e" % (k, v) for k, v in worst_l.items()))
    out.append("__device__ static constexpr float PZ_PW_MU_TAB[%d] = {" % (PW_N * 16))
    out += ["    " + ", ".join("%.9ef" % x for x in row) + "," for row in tab_mu]
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
