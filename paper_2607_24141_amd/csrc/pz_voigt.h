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
//    6 nodes for |z| < 8, 4 nodes for |z| < 40, 2 nodes beyond; the pairs
//    are summed over one common denominator.
//  * core, |z| < 5.5 and a <= 0.15 (float32): the series of w(v + ia) in a
//    about the real axis, w = exp(-z^2) + (2i/sqrt(pi)) F(z) with F Dawson's
//    integral; the Gaussian part is exact.  The derivatives of F are
//    piecewise polynomials in |v| for H alone (opacity) and rational fits in u
//    where L = Im w is needed too (adjoint); see gen_voigt_consts.py.  For a <= 0.03 the a^5 terms are
//    below 5e-8 of H and are dropped (chosen per wavefront).
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
// In terms of z2 = |z|^2 = u + a^2 and C_k = t_k^2 the pair terms are
//   N_k = z2 + C_k,   D_k = (u - a^2 - C_k)^2 + 4 u a^2 = (z2 - C_k)^2 + 4 C_k a^2,
// both sums of non-negative terms.  S = sum_k W_k N_k / D_k (H = a S) is
// summed over the common denominator prod_k D_k, so one reciprocal serves all
// pairs; no cancellation.  In the wing D_k <= (z2 + C_k)^2, and the callers
// use NP = 3 only for |z| < 8 and NP = 2 only for |z| < 40 or inside a
// wavefront that also holds a core lane, far from float32 overflow.
template <int NP>
__device__ __forceinline__ float wing_S(float a2, float z2, const float* T2, const float* W) {
    float e = z2 - T2[0];
    float den = fmaf(e, e, (4.0f * T2[0]) * a2);
    float num = fmaf(W[0], z2, W[0] * T2[0]);
#pragma unroll
    for (int k = 1; k < NP; ++k) {
        e = z2 - T2[k];
        const float Dk = fmaf(e, e, (4.0f * T2[k]) * a2);
        num = fmaf(num, Dk, fmaf(W[k], z2, W[k] * T2[k]) * den);
        den *= Dk;
    }
    return num * __builtin_amdgcn_rcpf(den);
}

// With P = z2 = u + a^2, C = t_k^2 and h = sum W_k N_k / D_k:
//   ha = sum W_k (D_k - 2 N_k^2) / D_k^2     (a dH/da = a h + 2 a^3 ha),
//   x  = sum W_k 2C (C^2 + 2PC - P(3u - a^2)) / D_k^2   (X = H + a dH/da + v dH/dv = a x;
//        the leading orders of the three terms cancel analytically in the wing).
template <int NP>
__device__ __forceinline__ void wing_SD(float a2, float u, float z2, const float* T2, const float* W, float& h,
                                        float& ha, float& x) {
    const float R3 = z2 * (3.0f * u - a2);
    h = 0.0f;
    ha = 0.0f;
    x = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const float C = T2[k];
        const float e = z2 - C;
        const float Dk = fmaf(e, e, (4.0f * C) * a2);
        const float Nk = z2 + C;
        const float r = __builtin_amdgcn_rcpf(Dk);
        const float r2 = r * r;
        h = fmaf(W[k] * Nk, r, h);
        ha = fmaf(W[k] * fmaf(-2.0f * Nk, Nk, Dk), r2, ha);
        x = fmaf(W[k] * (2.0f * C) * (fmaf(C, C, 2.0f * z2 * C) - R3), r2, x);
    }
}

// ------------------------------------------------------- small-damping core
template <int N>
__device__ __forceinline__ float horner(const float* c, float u) {
    float r = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) r = fmaf(r, u, c[k]);
    return r;
}

// cos(2av) and sin(2av)/(2av) as series in t = (2av)^2; FULL keeps the t^4
// terms (needed up to a = 0.15), else they end at t^3 (a <= 0.03).
template <bool FULL>
__device__ __forceinline__ float cos_t(float t) {
    if (FULL)
        return fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
    return fmaf(t, fmaf(t, fmaf(t, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f), 1.0f);
}
template <bool FULL>
__device__ __forceinline__ float sinc_t(float t) {
    if (FULL)
        return fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f), -1.0f / 6.0f),
                    1.0f);
    return fmaf(t, fmaf(t, fmaf(t, -1.0f / 5040.0f, 1.0f / 120.0f), -1.0f / 6.0f), 1.0f);
}

// Lam(u) = Lam0 + a^2 Lam2 [+ a^4 Lam4]: the damping series of Re w.
template <bool FULL>
__device__ __forceinline__ float lam_num(float a2, float u) {
    const float p2 = horner<9>(PZ_LAM_P2, u);
    const float inner = FULL ? fmaf(a2, horner<8>(PZ_LAM_P4, u), p2) : p2;
    return fmaf(a2, inner, horner<8>(PZ_LAM_P0, u));
}
template <bool FULL>
__device__ __forceinline__ float mu_num(float a2, float u) {
    const float p2 = horner<8>(PZ_MU_P2, u);
    const float inner = FULL ? fmaf(a2, horner<7>(PZ_MU_P4, u), p2) : p2;
    return fmaf(a2, inner, horner<7>(PZ_MU_P0, u));
}

// acc + K H on the small-damping core from the piecewise table pw (in LDS):
// K H = K exp(a^2 - u) cos(2av) + K a [Lam0 + a^2 Lam2 (+ a^4 Lam4)](|v|),
// each Lam a polynomial in t = |v| - c_k on the interval k holding |v|.
template <bool FULL>
__device__ __forceinline__ float coreP_KH_acc(float acc, float a2, float K, float Ka, float v, const float4* pw) {
    const float av = fabsf(v);
    const int k = min((int)(av * PZ_PW_INV_H), PZ_PW_N - 1);
    const float4* T = pw + 4 * k;
    const float4 q0 = T[0], q1 = T[1], q2 = T[2];
    const float t = av - q2.w;
    const float L0 = fmaf(fmaf(fmaf(fmaf(fmaf(q1.y, t, q1.x), t, q0.w), t, q0.z), t, q0.y), t, q0.x);
    float inner = fmaf(fmaf(fmaf(fmaf(q2.z, t, q2.y), t, q2.x), t, q1.w), t, q1.z);
    if (FULL) {
        const float4 q3 = T[3];
        inner = fmaf(a2, fmaf(fmaf(q3.z, t, q3.y), t, q3.x), inner);
    }
    const float u = v * v;
    const float g = __expf(a2 - u);
    return fmaf(Ka, fmaf(a2, inner, L0), fmaf(K * g, cos_t<FULL>((4.0f * a2) * u), acc));
}

// Copies the piecewise core table into LDS (all threads of the workgroup;
// the caller synchronises before use).
__device__ __forceinline__ void load_pw_table(float4* dst) {
    float* d = reinterpret_cast<float*>(dst);
    for (int k = threadIdx.x; k < PZ_PW_N * 16; k += blockDim.x) d[k] = PZ_PW_TAB[k];
}

// K H as above and K a L, with L = Im w = -exp(a^2-u) sin(2av) + v Mu(u)/Q'(u):
//   K a L = v (K a Mu/Q' - 2 a^2 K exp(a^2-u) sin(2av)/(2av)).
template <bool FULL>
__device__ __forceinline__ void coreS_KHL(float a2, float K, float Ka, float v, float u, float& KH, float& KaL) {
    const float g = __expf(a2 - u);
    const float t = (4.0f * a2) * u;
    KH = fmaf(Ka * lam_num<FULL>(a2, u), __builtin_amdgcn_rcpf(horner<9>(PZ_LAM_Q, u)), K * g * cos_t<FULL>(t));
    const float Kg = K * g;
    KaL = v * fmaf(Ka * mu_num<FULL>(a2, u), __builtin_amdgcn_rcpf(horner<8>(PZ_MU_Q, u)),
                   -2.0f * a2 * Kg * sinc_t<FULL>(t));
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
// Line-depth parameters arrive as (a^2, K, K a) with K the line-strength
// factor; the functions return K-scaled results.  Every branch on __any /
// __all is wavefront-uniform; the tests run in order of how often each tier
// is taken in the far-wing-dominated windows of the workloads.

// acc + K H(a, v); pw is the piecewise core table in LDS.
__device__ __forceinline__ float voigt_acc(float acc, float a2, float K, float Ka, float v, const float4* pw) {
    const float z2 = fmaf(v, v, a2);
    if (__all(z2 >= PZ_VOIGT_TIER2_R2)) {
        if (__any(z2 < PZ_VOIGT_TIER3_R2)) return fmaf(Ka, wing_S<2>(a2, z2, PZ_GH4_T2, PZ_GH4_W), acc);
        return fmaf(Ka, wing_S<1>(a2, z2, PZ_GH2_T2, PZ_GH2_W), acc);
    }
    if (!__any(z2 < PZ_VOIGT_WING_R2)) return fmaf(Ka, wing_S<3>(a2, z2, PZ_GH6_T2, PZ_GH6_W), acc);
    // a wavefront with at least one core lane
    if (z2 < PZ_VOIGT_WING_R2) {
        if (a2 <= PZ_VOIGT_A2_SMALL) {
            if (__any(a2 > PZ_VOIGT_A2_TINY)) return coreP_KH_acc<true>(acc, a2, K, Ka, v, pw);
            return coreP_KH_acc<false>(acc, a2, K, Ka, v, pw);
        }
        double wr, wi;
        core_w(sqrt((double)a2), (double)v, wr, wi);
        return (float)fma((double)K, wr, (double)acc);
    }
    if (z2 < PZ_VOIGT_TIER2_R2) return fmaf(Ka, wing_S<3>(a2, z2, PZ_GH6_T2, PZ_GH6_W), acc);
    return fmaf(Ka, wing_S<2>(a2, z2, PZ_GH4_T2, PZ_GH4_W), acc);
}

// K H, K a dH/da and K X, X = H + a dH/da + v dH/dv.  In the cores these follow
// from w = H + iL: dH/dv = -2(vH - aL), dH/da = 2(vL + aH) - 2/sqrt(pi).
__device__ __forceinline__ void voigt_KHD(float a2, float K, float Ka, float v, float u, float& KH, float& KaHa,
                                          float& KX) {
    const float z2 = u + a2;
    float h, ha, x;
    if (__all(z2 >= PZ_VOIGT_TIER2_R2)) {
        if (__any(z2 < PZ_VOIGT_TIER3_R2))
            wing_SD<2>(a2, u, z2, PZ_GH4_T2, PZ_GH4_W, h, ha, x);
        else
            wing_SD<1>(a2, u, z2, PZ_GH2_T2, PZ_GH2_W, h, ha, x);
    } else if (!__any(z2 < PZ_VOIGT_WING_R2) || z2 >= PZ_VOIGT_WING_R2) {
        wing_SD<3>(a2, u, z2, PZ_GH6_T2, PZ_GH6_W, h, ha, x);
    } else {
        if (a2 <= PZ_VOIGT_A2_SMALL) {
            float KaL;
            if (__any(a2 > PZ_VOIGT_A2_TINY))
                coreS_KHL<true>(a2, K, Ka, v, u, KH, KaL);
            else
                coreS_KHL<false>(a2, K, Ka, v, u, KH, KaL);
            const float c = 2.0f * kInvSqrtPiF * Ka;
            KaHa = fmaf(2.0f, fmaf(v, KaL, a2 * KH), -c);
            KX = fmaf(KH, fmaf(2.0f, a2 - u, 1.0f), fmaf(4.0f * v, KaL, -c));
        } else {
            const double ad = sqrt((double)a2), vd = v, Kd = K;
            double wr, wi;
            core_w(ad, vd, wr, wi);
            const double Ha = 2.0 * (vd * wi + ad * wr) - 2.0 * kInvSqrtPi;
            const double Hv = -2.0 * (vd * wr - ad * wi);
            KH = (float)(Kd * wr);
            KaHa = (float)(Kd * ad * Ha);
            KX = (float)(Kd * (wr + ad * Ha + vd * Hv));
        }
        return;
    }
    KH = Ka * h;
    KaHa = Ka * fmaf(2.0f * a2, ha, h);
    KX = Ka * x;
}

}  // namespace pz
