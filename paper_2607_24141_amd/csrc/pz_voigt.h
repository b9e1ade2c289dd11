// Device evaluation of the Voigt function H(a, v) = Re w(v + i a) and the
// derivative combinations the adjoint needs.
//
// Two regions, chosen per lane from z = v + i a:
//  * wing, |z|^2 >= 30.25 (float32): 6-point Gauss-Hermite quadrature of
//      H(a,v) = (a/pi) int exp(-t^2) / ((v-t)^2 + a^2) dt
//    with the +/-t_k nodes paired,
//      H = a sum_k W_k N_k / D_k,  N_k = u + a^2 + t_k^2,
//      D_k = (u - a^2 - t_k^2)^2 + 4 u a^2,  u = v^2,  W_k = 2 w_k / pi.
//    Every term is positive, so the relative accuracy of H holds even when
//    H << |w| (small a, far wings), where a complex-arithmetic evaluation of
//    Re w would cancel.  Measured max relative error 1e-6 over the region.
//  * core, |z|^2 < 30.25 (float64): Weideman's 32-term rational expansion of
//    w(z).  Near the real axis for small a, Re w is a tiny difference of
//    O(|w|) terms; float64 keeps that difference to ~1e-9 relative, and on
//    CDNA3/4 a float64 FMA issues at the same rate as an unpacked float32 FMA.
#pragma once
#include <hip/hip_runtime.h>
#include "voigt_consts.h"

namespace pz {

static constexpr double kInvSqrtPi = 0.56418958354775628695;

// ---------------------------------------------------------------- float32 wing
__device__ __forceinline__ float wing_H(float a, float u) {
    const float a2 = a * a;
    const float s = u - a2;
    const float q2 = 4.0f * u * a2;
    const float m = u + a2;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < PZ_GH_PAIRS; ++k) {
        const float P = s - PZ_GH_T2[k];
        const float Dk = fmaf(P, P, q2);
        const float Nk = m + PZ_GH_T2[k];
        acc = fmaf(PZ_GH_W[k] * Nk, __builtin_amdgcn_rcpf(Dk), acc);
    }
    return a * acc;
}

// Wing: H, a dH/da and X = H + a dH/da + v dH/dv from the paired quadrature.
// With P = u + a^2, Q = u - a^2, C = t_k^2:
//   d(N/D)/da = 2a (D - 2N^2) / D^2,
//   X_k      = 2C (C^2 + 2PC - P(3u - a^2)) / D^2      (leading orders cancel
//                                                        analytically)
__device__ __forceinline__ void wing_HD(float a, float u, float& H, float& aHa, float& X) {
    const float a2 = a * a;
    const float s = u - a2;
    const float q2 = 4.0f * u * a2;
    const float P = u + a2;
    const float R3 = P * (3.0f * u - a2);
    float h = 0.0f, ha = 0.0f, x = 0.0f;
#pragma unroll
    for (int k = 0; k < PZ_GH_PAIRS; ++k) {
        const float C = PZ_GH_T2[k];
        const float Pk = s - C;
        const float Dk = fmaf(Pk, Pk, q2);
        const float Nk = P + C;
        const float r = __builtin_amdgcn_rcpf(Dk);
        const float r2 = r * r;
        h = fmaf(PZ_GH_W[k] * Nk, r, h);
        ha = fmaf(PZ_GH_W[k] * fmaf(-2.0f * Nk, Nk, Dk), r2, ha);
        x = fmaf(PZ_GH_W[k] * (2.0f * C) * (fmaf(C, C, 2.0f * P * C) - R3), r2, x);
    }
    H = a * h;
    aHa = fmaf(2.0f * a2, a * ha, H);
    X = a * x;
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

__device__ __forceinline__ bool in_wing(float a, float u) {
    return fmaf(a, a, u) >= PZ_VOIGT_WING_R2;
}

// H(a, v) given u = v^2 (v itself is needed only in the core).
__device__ __forceinline__ float voigt_H(float a, float v, float u) {
    if (in_wing(a, u)) return wing_H(a, u);
    double wr, wi;
    core_w((double)a, (double)v, wr, wi);
    return (float)wr;
}

// H, a dH/da and X = H + a dH/da + v dH/dv (core from w = H + iL with
// dH/dv = -2(vH - aL), dH/da = 2(vL + aH) - 2/sqrt(pi)).
__device__ __forceinline__ void voigt_HD(float a, float v, float u, float& H, float& aHa, float& X) {
    if (in_wing(a, u)) {
        wing_HD(a, u, H, aHa, X);
        return;
    }
    const double ad = a, vd = v;
    double wr, wi;
    core_w(ad, vd, wr, wi);
    const double Ha = 2.0 * (vd * wi + ad * wr) - 2.0 * kInvSqrtPi;
    const double Hv = -2.0 * (vd * wr - ad * wi);
    H = (float)wr;
    aHa = (float)(ad * Ha);
    X = (float)(wr + ad * Ha + vd * Hv);
}

}  // namespace pz
