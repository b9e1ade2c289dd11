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
// pairs; no cancellation.  In the wing D_k <= (z2 + C_k)^2: the products
// overflow float32 beyond |z| ~ 1600 (NP = 3) and ~ 6e4 (NP = 2), which a
// wavefront taking those tiers reaches only for lines flagged SAFE (see
// voigt_acc); those lanes then use their own tier.
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

// With z2 = u + a^2, C = t_k^2 and h = sum W_k N_k / D_k:
//   ha = sum W_k M_k / D_k^2,   M_k = D_k - 2 N_k^2 = -z2^2 - C (6 z2 - 4 a^2 + C)
//        (a dH/da = a h + 2 a^3 ha),
//   x  = sum W_k 2C Q_k / D_k^2, Q_k = C^2 + 2 C z2 - 3 z2^2 + 4 a^2 z2
//        (X = H + a dH/da + v dH/dv = a x: the leading orders of the three
//        terms cancel analytically, so x carries no cancellation).
// The pair-independent parts of M_k and Q_k are formed once.
template <int NP>
__device__ __forceinline__ void wing_SD(float a2, float z2, const float* T2, const float* W, float& h, float& ha,
                                        float& x) {
    const float mz2sq = -z2 * z2;
    const float E = fmaf(6.0f, z2, -4.0f * a2);
    const float B = z2 * fmaf(-3.0f, z2, 4.0f * a2);
    const float z2x2 = z2 + z2;
    h = 0.0f;
    ha = 0.0f;
    x = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const float C = T2[k];
        const float e = z2 - C;
        const float Dk = fmaf(e, e, (4.0f * C) * a2);
        const float r = __builtin_amdgcn_rcpf(Dk);
        h = fmaf(fmaf(W[k], z2, W[k] * C), r, h);
        const float r2 = r * r;
        ha = fmaf(fmaf(-C, E + C, mz2sq), W[k] * r2, ha);
        x = fmaf(fmaf(C, z2x2 + C, B), (2.0f * W[k] * C) * r2, x);
    }
}

// ------------------------------------------------------- small-damping core
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

// Piecewise tables of the small-damping core (in LDS): interval k of |v|
// holds [P0_0..P0_3 | P0_4 P0_5 P2_0 P2_1 | P2_2 P2_3 P2_4 c | P4_0 P4_1 P4_2 0],
// four float4 at a stride of five (the fifth unused): a 16-byte read covers
// four of the 32 banks, and at a stride of 20 words eight neighbouring
// intervals start in eight different bank quarters, so lanes in different
// intervals read without bank conflicts (at a stride of 16 words all even
// intervals would share banks, and all odd ones).  The table for L follows
// the one for H.
static constexpr int PZ_PW_STRIDE = 5;
static constexpr int PZ_PW_LDS = PZ_PW_N * PZ_PW_STRIDE;   // float4 per table in LDS

struct PwPoint {
    int k;       // interval
    float t;     // |v| - centre
};

__device__ __forceinline__ PwPoint pw_point(float v, const float4* tab) {
    const float av = fabsf(v);
    PwPoint p;
    p.k = min((int)(av * PZ_PW_INV_H), PZ_PW_N - 1);
    p.t = av - tab[PZ_PW_STRIDE * p.k + 2].w;
    return p;
}

// P0 + a^2 P2 [+ a^4 P4] at t on table interval T.
template <bool FULL>
__device__ __forceinline__ float pw_poly(const float4* T, float t, float a2) {
    const float4 q0 = T[0], q1 = T[1], q2 = T[2];
    const float P0 = fmaf(fmaf(fmaf(fmaf(fmaf(q1.y, t, q1.x), t, q0.w), t, q0.z), t, q0.y), t, q0.x);
    float inner = fmaf(fmaf(fmaf(fmaf(q2.z, t, q2.y), t, q2.x), t, q1.w), t, q1.z);
    if (FULL) {
        const float4 q3 = T[3];
        inner = fmaf(a2, fmaf(fmaf(q3.z, t, q3.y), t, q3.x), inner);
    }
    return fmaf(a2, inner, P0);
}

// acc + K H on the small-damping core:
// K H = K exp(a^2 - u) cos(2av) + K a [Lam0 + a^2 Lam2 (+ a^4 Lam4)](|v|).
template <bool FULL>
__device__ __forceinline__ float coreP_KH_acc(float acc, float a2, float K, float Ka, float v, const float4* pw) {
    const PwPoint p = pw_point(v, pw);
    const float lam = pw_poly<FULL>(pw + PZ_PW_STRIDE * p.k, p.t, a2);
    const float u = v * v;
    const float g = __expf(a2 - u);
    return fmaf(Ka, lam, fmaf(K * g, cos_t<FULL>((4.0f * a2) * u), acc));
}

// K H as above and K a L, L = Im w = -exp(a^2-u) sin(2av) + v [Mu0 + a^2 Mu2 (+ a^4 Mu4)](|v|):
//   K a L = v (K a Mu - 2 a^2 K exp(a^2-u) sin(2av)/(2av)).
template <bool FULL>
__device__ __forceinline__ void coreP_KHL(float a2, float K, float Ka, float v, const float4* pw, float& KH,
                                          float& KaL) {
    const PwPoint p = pw_point(v, pw);
    const float lam = pw_poly<FULL>(pw + PZ_PW_STRIDE * p.k, p.t, a2);
    const float mu = pw_poly<FULL>(pw + PZ_PW_STRIDE * (PZ_PW_N + p.k), p.t, a2);
    const float u = v * v;
    const float t = (4.0f * a2) * u;
    const float Kg = K * __expf(a2 - u);
    KH = fmaf(Ka, lam, Kg * cos_t<FULL>(t));
    KaL = v * fmaf(Ka, mu, -2.0f * a2 * Kg * sinc_t<FULL>(t));
}

// Copies the piecewise core tables into LDS: the H table, and with_L the L
// table after it (all threads of the workgroup; the caller synchronises).
__device__ __forceinline__ void load_pw_table(float4* dst, bool with_L) {
    float* d = reinterpret_cast<float*>(dst);
    for (int k = threadIdx.x; k < PZ_PW_N * 16; k += blockDim.x) {
        const int o = (k / 16) * (4 * PZ_PW_STRIDE) + k % 16;
        d[o] = PZ_PW_TAB[k];
        if (with_L) d[4 * PZ_PW_LDS + o] = PZ_PW_MU_TAB[k];
    }
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
// Wavefront votes on the lane mask of a compare (HIP's __all and __any first
// turn the predicate into a per-lane 0/1 value and compare that again).
__device__ __forceinline__ bool wave_all(bool c) {
    return __builtin_amdgcn_ballot_w64(c) == __builtin_amdgcn_read_exec();
}
__device__ __forceinline__ bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }

// Line-depth parameters arrive as (a^2, K, K a) with K the line-strength
// factor; the functions return K-scaled results.  Every branch on __any /
// __all is wavefront-uniform; the tests run in order of how often each tier
// is taken in the far-wing-dominated windows of the workloads.

// acc + K H(a, v); pw is the piecewise core table in LDS.  With CT the
// lane adds nothing unless v^2 + a^2 <= zmax2 (centre-test span).
// SAFE (chosen per line, wavefront-uniform): lanes far out beside near ones,
// which happen only for lines whose damping ratio spans both the 6- or
// 4-node range and the far wing across depths, take their own tier, so the
// pair products of the 6- and 4-node sums stay inside the float32 range.
template <bool CT, bool SAFE>
__device__ __forceinline__ float voigt_acc(float acc, float a2, float K, float Ka, float v, const float4* pw,
                                           float zmax2) {
    const float z2 = fmaf(v, v, a2);
    if (CT && !(z2 <= zmax2)) return acc;
    if (__all(z2 >= PZ_VOIGT_TIER2_R2)) {
        if (SAFE) {
            const unsigned long long near = __ballot(z2 < PZ_VOIGT_TIER3_R2);
            if (near != 0 && near != __ballot(1)) {
                if (z2 < PZ_VOIGT_TIER3_R2) return fmaf(Ka, wing_S<2>(a2, z2, PZ_GH4_T2, PZ_GH4_W), acc);
                return fmaf(Ka, wing_S<1>(a2, z2, PZ_GH2_T2, PZ_GH2_W), acc);
            }
        }
        if (__any(z2 < PZ_VOIGT_TIER3_R2)) return fmaf(Ka, wing_S<2>(a2, z2, PZ_GH4_T2, PZ_GH4_W), acc);
        return fmaf(Ka, wing_S<1>(a2, z2, PZ_GH2_T2, PZ_GH2_W), acc);
    }
    if (!__any(z2 < PZ_VOIGT_WING_R2) && !(SAFE && __any(z2 >= PZ_VOIGT_TIER3_R2)))
        return fmaf(Ka, wing_S<3>(a2, z2, PZ_GH6_T2, PZ_GH6_W), acc);
    // a wavefront with at least one core lane (or, SAFE, a far lane)
    if (z2 < PZ_VOIGT_WING_R2) {
        if (a2 <= PZ_VOIGT_A2_SMALL) {
            if (__any(a2 > PZ_VOIGT_A2_TINY)) return coreP_KH_acc<true>(acc, a2, K, Ka, v, pw);
            return coreP_KH_acc<false>(acc, a2, K, Ka, v, pw);
        }
        double wr, wi;
        core_w(sqrt((double)a2), (double)v, wr, wi);
        return (float)fma((double)K, wr, (double)acc);
    }
    // The wing lanes beside core lanes: without SAFE all take the six-node
    // sum (one pass instead of two; in range, as for the uniform case above).
    if (!SAFE || z2 < PZ_VOIGT_TIER2_R2) return fmaf(Ka, wing_S<3>(a2, z2, PZ_GH6_T2, PZ_GH6_W), acc);
    if (z2 >= PZ_VOIGT_TIER3_R2) return fmaf(Ka, wing_S<1>(a2, z2, PZ_GH2_T2, PZ_GH2_W), acc);
    return fmaf(Ka, wing_S<2>(a2, z2, PZ_GH4_T2, PZ_GH4_W), acc);
}

// K H, K a dH/da and K X, X = H + a dH/da + v dH/dv; pw holds the H and L
// core tables.  In the cores these follow
// from w = H + iL: dH/dv = -2(vH - aL), dH/da = 2(vL + aH) - 2/sqrt(pi).
__device__ __forceinline__ void voigt_KHD(float a2, float K, float Ka, float v, float u, const float4* pw, float& KH,
                                          float& KaHa, float& KX) {
    const float z2 = u + a2;
    float h, ha, x;
    if (wave_all(z2 >= PZ_VOIGT_TIER2_R2)) {
        if (wave_any(z2 < PZ_VOIGT_TIER3_R2))
            wing_SD<2>(a2, z2, PZ_GH4_T2, PZ_GH4_W, h, ha, x);
        else
            wing_SD<1>(a2, z2, PZ_GH2_T2, PZ_GH2_W, h, ha, x);
    } else if (!wave_any(z2 < PZ_VOIGT_WING_R2) || z2 >= PZ_VOIGT_WING_R2) {
        wing_SD<3>(a2, z2, PZ_GH6_T2, PZ_GH6_W, h, ha, x);
    } else {
        if (a2 <= PZ_VOIGT_A2_SMALL) {
            float KaL;
            if (wave_any(a2 > PZ_VOIGT_A2_TINY))
                coreP_KHL<true>(a2, K, Ka, v, pw, KH, KaL);
            else
                coreP_KHL<false>(a2, K, Ka, v, pw, KH, KaL);
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
