// Device evaluation of the Voigt function H(a, v) = Re w(v + i a) and the
// derivative combinations the adjoint needs.
//
// Regions of z = v + i a:
//  * wing, |z| >= 5.5 (float32): Gauss-Hermite quadrature of
//      H(a,v) = (a/pi) int exp(-t^2) / ((v-t)^2 + a^2) dt
//    with the +/-t_k nodes paired,
//      H = a sum_k W_k N_k / D_k,  N_k = u + a^2 + t_k^2,
//      D_k = (u - a^2 - t_k^2)^2 + 4 u a^2,  u = v^2,  W_k = 2 w_k / pi.
//    Every term is positive, so H keeps its relative accuracy even where
//    H << |w| (small a, far wings), where complex arithmetic on w would cancel.
//    6 nodes for |z| < 8, 4 nodes for |z| < 40, 2 nodes beyond.
//  * core, |z| < 5.5 and a <= 0.15 (float32): the series of w(v + ia) in a
//    about the real axis, w = exp(-z^2) + (2i/sqrt(pi)) F(z) with F Dawson's
//    integral; the Gaussian part is exact, the derivatives of F are rational
//    fits in u (see gen_voigt_consts.py).
//  * core, |z| < 5.5 and a > 0.15 (float64): Weideman's 32-term rational
//    expansion of w(z); rare (deep layers of strongly damped lines).
//
// The wing tier is chosen per wavefront: all lanes use the most accurate tier
// any lane needs, so no lane runs a less accurate formula than its own tier.
#pragma once
#include <hip/hip_runtime.h>

#include "voigt_consts.h"

namespace pz {

static constexpr double kInvSqrtPi = 0.56418958354775628695;
static constexpr float kInvSqrtPiF = 0.5641895835f;

// ---------------------------------------------------------------- wing tiers
template <int NP>
__device__ __forceinline__ float wing_H(float a, float a2, float u, const float* T2, const float* W) {
    const float s = u - a2;
    const float q2 = 4.0f * u * a2;
    const float m = u + a2;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const float P = s - T2[k];
        const float Dk = fmaf(P, P, q2);
        acc = fmaf(W[k] * (m + T2[k]), __builtin_amdgcn_rcpf(Dk), acc);
    }
    return a * acc;
}

// H, a dH/da and X = H + a dH/da + v dH/dv.  With P = u + a^2, C = t_k^2:
//   d(N/D)/da = 2a (D - 2N^2) / D^2,
//   X_k       = 2C (C^2 + 2PC - P(3u - a^2)) / D^2  (the leading orders of
//               H, a dH/da and v dH/dv cancel analytically in the wing).
template <int NP>
__device__ __forceinline__ void wing_HD(float a, float a2, float u, const float* T2, const float* W, float& H,
                                        float& aHa, float& X) {
    const float s = u - a2;
    const float q2 = 4.0f * u * a2;
    const float P = u + a2;
    const float R3 = P * (3.0f * u - a2);
    float h = 0.0f, ha = 0.0f, x = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const float C = T2[k];
        const float Pk = s - C;
        const float Dk = fmaf(Pk, Pk, q2);
        const float Nk = P + C;
        const float r = __builtin_amdgcn_rcpf(Dk);
        const float r2 = r * r;
        h = fmaf(W[k] * Nk, r, h);
        ha = fmaf(W[k] * fmaf(-2.0f * Nk, Nk, Dk), r2, ha);
        x = fmaf(W[k] * (2.0f * C) * (fmaf(C, C, 2.0f * P * C) - R3), r2, x);
    }
    H = a * h;
    aHa = fmaf(2.0f * a2, a * ha, H);
    X = a * x;
}

// ------------------------------------------------------- small-damping core
template <int N>
__device__ __forceinline__ float horner(const float* c, float u) {
    float r = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) r = fmaf(r, u, c[k]);
    return r;
}

// exp(a^2 - u) cos(2 a v) + a [Lam0 + a^2 Lam2 + a^4 Lam4](u)
__device__ __forceinline__ float coreS_H(float a, float a2, float u) {
    const float g = __expf(a2 - u);
    const float t = 4.0f * a2 * u;                       // (2 a v)^2
    const float cs = fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
    const float q = horner<9>(PZ_LAM_Q, u);
    const float num = fmaf(a2, fmaf(a2, horner<8>(PZ_LAM_P4, u), horner<9>(PZ_LAM_P2, u)), horner<8>(PZ_LAM_P0, u));
    return fmaf(a * num, __builtin_amdgcn_rcpf(q), g * cs);
}

// H as above and L = Im w = -exp(a^2-u) sin(2av) + v [Mu0 + a^2 Mu2 + a^4 Mu4](u)
__device__ __forceinline__ void coreS_HL(float a, float a2, float v, float u, float& H, float& L) {
    const float g = __expf(a2 - u);
    const float t = 4.0f * a2 * u;
    const float cs = fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
    const float sn = fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f), -1.0f / 6.0f),
                          1.0f);                         // sin(2av) / (2av)
    const float q = horner<9>(PZ_LAM_Q, u);
    const float num = fmaf(a2, fmaf(a2, horner<8>(PZ_LAM_P4, u), horner<9>(PZ_LAM_P2, u)), horner<8>(PZ_LAM_P0, u));
    H = fmaf(a * num, __builtin_amdgcn_rcpf(q), g * cs);
    const float qm = horner<8>(PZ_MU_Q, u);
    const float nm = fmaf(a2, fmaf(a2, horner<7>(PZ_MU_P4, u), horner<8>(PZ_MU_P2, u)), horner<7>(PZ_MU_P0, u));
    L = v * fmaf(nm, __builtin_amdgcn_rcpf(qm), -g * (2.0f * a) * sn);
}

// ---------------------------------------------------------------- float64 core
// w(z) ~ [2 p(Z)/(L - iz) + 1/sqrt(pi)] / (L - iz),  Z = (L + iz)/(L - iz).
__device__ __forceinline__ void core_w(double a, double v, double& wr, double& wi) {
    const double L = PZ_WEID_L;
    const double dr = L + a, di = -v;          // L - iz, with iz = -a + i v
    const double nr = L - a, ni = v;           // L + iz
    const double inv = 1.0 / (dr * dr + di * di);
    const double Zr = (nr * dr + ni * di) * inv;
    const double Zi = (ni * dr - nr * di) * inv;
    double pr = PZ_WEID_C[0], pim = 0.0;
#pragma unroll
    for (int k = 1; k < PZ_WEID_N; ++k) {
        const double t = fma(pr, Zr, fma(-pim, Zi, PZ_WEID_C[k]));
        pim = fma(pr, Zi, pim * Zr);
        pr = t;
    }
    const double rr = dr * inv, ri = -di * inv;   // 1/(L - iz)
    const double qr = 2.0 * (pr * rr - pim * ri) + kInvSqrtPi;
    const double qi = 2.0 * (pr * ri + pim * rr);
    wr = qr * rr - qi * ri;
    wi = qr * ri + qi * rr;
}

// ------------------------------------------------------------- dispatch
// H(a, v); a2 = a^2, u = v^2.  The branches on __any are wavefront-uniform.
__device__ __forceinline__ float voigt_H(float a, float a2, float v, float u) {
    const float z2 = u + a2;
    if (__any(z2 < PZ_VOIGT_WING_R2)) {
        if (z2 < PZ_VOIGT_WING_R2) {
            if (a <= PZ_VOIGT_A_SMALL) return coreS_H(a, a2, u);
            double wr, wi;
            core_w((double)a, (double)v, wr, wi);
            return (float)wr;
        }
        return wing_H<3>(a, a2, u, PZ_GH6_T2, PZ_GH6_W);
    }
    if (__any(z2 < PZ_VOIGT_TIER2_R2)) return wing_H<3>(a, a2, u, PZ_GH6_T2, PZ_GH6_W);
    if (__any(z2 < PZ_VOIGT_TIER3_R2)) return wing_H<2>(a, a2, u, PZ_GH4_T2, PZ_GH4_W);
    return wing_H<1>(a, a2, u, PZ_GH2_T2, PZ_GH2_W);
}

// H, a dH/da and X = H + a dH/da + v dH/dv.  In the cores these follow from
// w = H + iL: dH/dv = -2(vH - aL), dH/da = 2(vL + aH) - 2/sqrt(pi).
__device__ __forceinline__ void voigt_HD(float a, float a2, float v, float u, float& H, float& aHa, float& X) {
    const float z2 = u + a2;
    if (__any(z2 < PZ_VOIGT_WING_R2)) {
        if (z2 < PZ_VOIGT_WING_R2) {
            if (a <= PZ_VOIGT_A_SMALL) {
                float L;
                coreS_HL(a, a2, v, u, H, L);
                const float aL = a * L;
                aHa = a * (2.0f * fmaf(v, L, a * H) - 2.0f * kInvSqrtPiF);
                X = fmaf(H, fmaf(2.0f, a2 - u, 1.0f), fmaf(4.0f * v, aL, -2.0f * a * kInvSqrtPiF));
            } else {
                const double ad = a, vd = v;
                double wr, wi;
                core_w(ad, vd, wr, wi);
                const double Ha = 2.0 * (vd * wi + ad * wr) - 2.0 * kInvSqrtPi;
                const double Hv = -2.0 * (vd * wr - ad * wi);
                H = (float)wr;
                aHa = (float)(ad * Ha);
                X = (float)(wr + ad * Ha + vd * Hv);
            }
            return;
        }
        wing_HD<3>(a, a2, u, PZ_GH6_T2, PZ_GH6_W, H, aHa, X);
        return;
    }
    if (__any(z2 < PZ_VOIGT_TIER2_R2)) {
        wing_HD<3>(a, a2, u, PZ_GH6_T2, PZ_GH6_W, H, aHa, X);
    } else if (__any(z2 < PZ_VOIGT_TIER3_R2)) {
        wing_HD<2>(a, a2, u, PZ_GH4_T2, PZ_GH4_W, H, aHa, X);
    } else {
        wing_HD<1>(a, a2, u, PZ_GH2_T2, PZ_GH2_W, H, aHa, X);
    }
}

}  // namespace pz
