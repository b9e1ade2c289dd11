// Device bodies of every stage of the synthesis path.  The per-star kernels
// (pz_kernels.hip) and the persistent batch kernels (pz_batch.hip) call the
// same functions, so a batched star computes exactly what a per-star call
// computes.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "pz_internal.h"
#include "pz_voigt.h"

namespace pz {

static constexpr int WAVE = 64;

// ------------------------------------------------------------ populations
// Two-stage Saha ionisation (Sec. 3, Eq. 11) with no ionisation lowering:
//   Phi = (2 U_II / U_I) (2 pi m_e k T / h^2)^{3/2} exp(-chi / kT) / n_e,
//   f_I = 1/(1+Phi), f_II = Phi/(1+Phi); infinite chi => single stage.
// Output n_{s,r}/(rho U_{s,r}) with the abundance correction 10^dA (Eq. 30).
__device__ __forceinline__ void dev_populations(const StarDev& s, int idx) {
    if (idx == 0) s.wide_any[0] = 0;                  // raised by dev_line_consts
    if (idx >= s.S * s.D) return;
    const int sp = idx / s.D, j = idx - sp * s.D;
    const double T = s.T[j];
    const double chi = s.chi_ion[sp];
    const double U0 = s.U[(sp * 2 + 0) * s.D + j];
    const double U1 = s.U[(sp * 2 + 1) * s.D + j];
    const double saha = pow(2.0 * PI * M_ELECTRON * K_BOLTZ / (H_PLANCK * H_PLANCK), 1.5);
    double fI = 1.0, fII = 0.0;
    if (isfinite(chi)) {
        const double phi = 2.0 * U1 / U0 * saha * T * sqrt(T) * exp(-chi * EV_ERG / (K_BOLTZ * T)) / s.ne[j];
        if (phi <= 1.0) {
            fI = 1.0 / (1.0 + phi);
            fII = phi * fI;
        } else {
            fII = 1.0 / (1.0 + 1.0 / phi);
            fI = fII / phi;
        }
    }
    const double n = (s.dA ? exp10((double)s.dA[sp]) : 1.0) * s.n_species[sp * s.D + j];
    s.pop[(sp * 2 + 0) * s.D + j] = n * fI / (s.rho[j] * U0);
    s.pop[(sp * 2 + 1) * s.D + j] = n * fII / (s.rho[j] * U1);
    // reciprocal Doppler width (Eq. 5), per species and depth
    const double xi = (double)s.xi[0] * 1.0e5;
    s.inv_dv[sp * s.D + j] = 1.0 / sqrt(2.0 * K_BOLTZ * T / (s.mass[sp] * AMU_G) + xi * xi);
}

// ------------------------------------------------- line-selection keep test
// Per sorted line (Sec. 3, Eqs. 17-19), after dev_populations, in float64:
//   b     = floor(ln(lambda_l / lambda_first) / bin_ln) clamped to [0, B)
//   nu_b  = frequency at the bin's centre in ln lambda
//   C_jb  = eta kappa_c(nu_b) / (1 - exp(-h nu_b / k T_j))            (sigma_c = 0)
//   Q     = max_j pop_{s,r,j} / ((dv_{s,j} / c) C_jb)                  (pop = n / (rho U))
//   R_l   = sqrt(pi) e^2 / (m_e c) 10^(loggf + dgf) Q / nu_b
//   keep  = R_l >= 1 and R_l exp(-E_l / k T_deepest) >= 1
// Q is taken per line over the line's own (species, ion, bin): the same max
// over the same terms as a per-bin table, so no table is stored.
__device__ __forceinline__ void dev_select(const StarDev& s, int l, double eta, double bin_ln, int B,
                                           unsigned char* keep, double* R_out, double* Rd_out, int* n_keep) {
    if (l >= s.L) return;
    const int caller = s.ln.perm[l];
    const int spion = s.ln.spion[l], sp = spion >> 1;
    const double bf = floor(log(s.ln.lam_cm[l] * 1.0e7 / s.lam_first_nm) / bin_ln);
    const double b = fmin(fmax(bf, 0.0), (double)(B - 1));
    const double lam_b = s.lam_first_nm * exp((b + 0.5) * bin_ln);          // nm
    const double nu_b = C_LIGHT / (lam_b * 1.0e-7);
    const double kc = s.kappa0 * pow(lam_b / s.lam_ref_nm, s.alpha);
    double Q = 0.0;
    for (int j = 0; j < s.D; ++j) {
        const double C = eta * kc / (-expm1(-H_PLANCK * nu_b / (K_BOLTZ * s.T[j])));
        Q = fmax(Q, s.pop[spion * s.D + j] * s.inv_dv[sp * s.D + j] * C_LIGHT / C);
    }
    const double loggf = s.ln.loggf[l] + (s.dgf ? (double)s.dgf[caller] : 0.0);
    const double R = sqrt(PI) * E_CHARGE * E_CHARGE / (M_ELECTRON * C_LIGHT) * exp10(loggf) * Q / nu_b;
    const double Rd = R * exp(-s.ln.E_eV[l] * EV_ERG / (K_BOLTZ * s.T[s.D - 1]));
    const bool k = R >= 1.0 && Rd >= 1.0;
    if (keep) keep[caller] = k ? 1 : 0;
    if (R_out) R_out[caller] = R;
    if (Rd_out) Rd_out[caller] = Rd;
    if (k && n_keep) atomicAdd(n_keep, 1);
}

// ------------------------------------------------------ line-depth params
// Per line (Eqs. 4, 5, 30), in float64:
//   x = (pi e^2/m_e c) 10^(loggf+dgf) lambda_l / sqrt(pi)
//   y, z, w = 10^ddamp lambda_l / (4 pi) x (g_rad 10^d_rad, g_S 10^d_S, g_vdW 10^d_vdW)
// Block-wide maxima of n_e and n_pert over depth and of 1/dv over (species,
// depth): with them (g_rad + g_S max n_e + g_vdW max n_pert) max(1/dv) bounds
// every line's damping ratio a from above.  Every thread of the workgroup
// calls this (it synchronises); red holds 3 doubles per thread.
__device__ __forceinline__ double3 damp_bounds(const StarDev& s, double* red) {
    const int t = threadIdx.x, n = blockDim.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int j = t; j < s.D; j += n) {
        a = fmax(a, s.ne[j]);
        b = fmax(b, s.npert[j]);
    }
    for (int k = t; k < s.S * s.D; k += n) c = fmax(c, s.inv_dv[k]);
    red[t] = a;
    red[n + t] = b;
    red[2 * n + t] = c;
    __syncthreads();
    for (int w = n / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int r = 0; r < 3; ++r) red[r * n + t] = fmax(red[r * n + t], red[r * n + t + w]);
        __syncthreads();
    }
    const double3 out = make_double3(red[0], red[n], red[2 * n]);
    __syncthreads();
    return out;
}

// bnd: damp_bounds of the workgroup.
__device__ __forceinline__ void dev_line_consts(const StarDev& s, int l, double3 bnd) {
    if (l >= s.L) return;
    const int caller = s.ln.perm[l];
    const double lam = s.ln.lam_cm[l];
    const double loggf = s.ln.loggf[l] + (s.dgf ? (double)s.dgf[caller] : 0.0);
    const double line_const = PI * E_CHARGE * E_CHARGE / (M_ELECTRON * C_LIGHT);
    const double damp = (s.ddamp ? exp10((double)s.ddamp[caller]) : 1.0) * lam / (4.0 * PI);
    const float* df = s.ddamp_family;                    // per-family corrections, [3][L] caller order
    s.lc[l] = make_double4(line_const * exp10(loggf) * lam / sqrt(PI),
                           damp * exp10(s.ln.lgr[l] + (df ? (double)df[caller] : 0.0)),
                           damp * exp10(s.ln.lgs[l] + (df ? (double)df[s.L + caller] : 0.0)),
                           damp * exp10(s.ln.lgw[l] + (df ? (double)df[2 * s.L + caller] : 0.0)));
    {   // damping-ratio range over depth: flags lines whose wavefronts can mix near and far wing tiers
        const double4 c = s.lc[l];
        bool wide = false;
        if (fma(c.w, bnd.y, fma(c.z, bnd.x, c.y)) * bnd.z > 1.0e3) {   // else a <= 1000 at every depth
            const int sp = s.ln.spion[l] >> 1;
            double amin = 1e300, amax = 0.0;
            for (int j = 0; j < s.D; ++j) {
                const double a = fma(c.w, s.npert[j], fma(c.z, s.ne[j], c.y)) * s.inv_dv[sp * s.D + j];
                amin = fmin(amin, a);
                amax = fmax(amax, a);
            }
            wide = (amin < 8.0 && amax > 1.0e3) || (amin < 40.0 && amax > 3.0e4);
        }
        s.wide_a[l] = wide ? 1 : 0;
        if (wide) atomicOr(s.wide_any, 1);
    }
    if (s.center) {
        s.xlim[l] = 0.0f;                                // raised by dev_line_params
        s.inv_kcl[l] = 1.0 / (s.kappa0 * pow(lam * 1.0e7 / s.lam_ref_nm, s.alpha));   // 1 / kappa_c(lambda_l)
    }
}

// Per (line, depth), in float64 then rounded (Eqs. 4-5, 30):
//   dv = sqrt(2kT/m + xi^2),  dnu_D = dv / lambda_l
//   a  = 10^ddamp (g_rad + g_S n_e + g_vdW n_pert) / (4 pi dnu_D)
//   K  = (pi e^2/m_e c) n/(rho U) 10^(loggf+dgf) e^{-E/kT} (1 - e^{-h nu_l/kT}) / (sqrt(pi) dnu_D)
// stored as (c/dv, a^2, K, K a); v = (lambda_l/lambda_i - 1) c/dv.  The
// per-line and per-(species, depth) factors come from dev_line_consts and
// dev_populations.
// Every lane of the wavefront must call this (lanes past L*D included):
// the centre test reduces across the wavefront.
__device__ __forceinline__ void dev_line_params(const StarDev& s, long idx) {
    const long n = (long)s.L * s.D;                       // < 2^32 (the plan checks L D)
    const bool valid = idx < n;
    const unsigned id = (unsigned)(valid ? idx : n - 1);  // out-of-range lanes compute a copy, store nothing
    const int l = (int)(id / (unsigned)s.D), j = (int)(id - (unsigned)l * (unsigned)s.D);
    const double T = s.T[j];
    const int spion = s.ln.spion[l];
    const double inv_dv = s.inv_dv[(spion >> 1) * s.D + j];
    const double4 c = s.lc[l];
    const double a = fma(c.w, s.npert[j], fma(c.z, s.ne[j], c.y)) * inv_dv;
    const double ikT = 1.0 / (K_BOLTZ * T);
    const double K = c.x * s.pop[spion * s.D + j] * exp(-s.ln.E_eV[l] * EV_ERG * ikT) *
                     (-expm1(-(H_PLANCK * C_LIGHT) / s.ln.lam_cm[l] * ikT)) * inv_dv;
    if (valid) s.lp[idx] = make_float4((float)(C_LIGHT * inv_dv), (float)(a * a), (float)K, (float)(K * a));
    if (!s.center) return;
    // continuum-referenced centre test, decided in float64: keep iff
    // K H(a,0) >= eta kappa_c(lambda_l); a kept pair deposits where
    // |v| <= V = max(sqrt(ln(R/eta)), sqrt(a R / (sqrt(pi) eta))), R = K / kappa_c
    const double eta = s.center_eta;
    const double R = K * s.inv_kcl[l];
    float zm = -1.0f, xl = 0.0f;
    if (R * __ocml_erfcx_f64(a) >= eta) {
        const double vd = R > eta ? sqrt(log(R / eta)) : 0.0;
        const double V = fmax(vd, sqrt(a * R / (sqrt(PI) * eta)));
        zm = (float)(V * V + a * a);
        xl = (float)(V / (C_LIGHT * inv_dv));              // detuning |x| = V dv / c
    }
    if (valid) s.zmax[idx] = zm;
    // Largest |x| over each line's depths: one wavefront-wide max and one
    // atomic per distinct line in the wavefront (non-negative floats order as
    // their bit patterns; the result does not depend on the order).
    const int lane = (int)(threadIdx.x & 63);
    bool done = !valid || !(xl > 0.0f);
    for (;;) {
        const unsigned long long b = __ballot(!done);
        if (b == 0) break;
        const int first = __ffsll(b) - 1;
        const int lc = __shfl(l, first, 64);
        float m = l == lc ? xl : 0.0f;
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if (lane == first) atomicMax(reinterpret_cast<int*>(&s.xlim[lc]), __float_as_int(m));
        if (l == lc) done = true;
    }
}

}  // namespace pz

#include "pz_opacity.h"

namespace pz {

// ------------------------------------------------------- formal solution
// Piecewise-linear S(tau) between depths, diffusion lower boundary and a
// linear extrapolation of S to tau = 0 (Eq. 7), summed from the surface down:
//   I(0, mu) = C_top + sum_j A_j c_j + A_{D-1} I_D,
//   A_j = exp(-tau_j / mu),  x_j = (tau_{j+1} - tau_j)/mu,
//   c_j = S_j (1 - e^{-x_j}) + (S_{j+1} - S_j) lw(x_j),
//   lw(x) = (1 - (1 + x) e^{-x}) / x,
//   C_top = S_top (1 - e^{-x_t}) + (S_0 - S_top) lw(x_t), x_t = tau_0/mu,
//   S_top = S_0 - tau_0 (S_1 - S_0)/(tau_1 - tau_0),
//   I_D = S_{D-1} + mu (S_{D-1} - S_{D-2}) / (tau_{D-1} - tau_{D-2}).
// This is the bottom-up recurrence of the formal solution unrolled into a
// sum, so a single top-down pass with O(1) state per ray suffices.
// 3-point Gauss-Legendre on [0, 1]: mu = 1/2 -+ sqrt(3/5)/2, 1/2; w = 5/18, 8/18, 5/18
static constexpr double kMu0 = 0.1127016653792583, kMu1 = 0.5, kMu2 = 0.8872983346207417;
__constant__ float c_mu[3] = {(float)kMu0, (float)kMu1, (float)kMu2};
__constant__ float c_inv_mu[3] = {(float)(1.0 / kMu0), (float)(1.0 / kMu1), (float)(1.0 / kMu2)};
__constant__ float c_wmu[3] = {(float)(2.0 * PI * 5.0 / 18.0 * kMu0), (float)(2.0 * PI * 8.0 / 18.0 * kMu1),
                               (float)(2.0 * PI * 5.0 / 18.0 * kMu2)};  // 2 pi w_k mu_k

struct ExpTerms {
    float e, om, lw, dlw;   // e^-x, 1 - e^-x, lw(x), lw'(x)
};

__device__ __forceinline__ ExpTerms exp_terms(float x, bool need_d) {
    ExpTerms r;
    r.e = expf(-x);
    r.om = -expm1f(-x);
    if (x < 0.05f) {
        // series of lw and lw' (sum_{n>=2} (-1)^n (n-1) x^{n-1}/n! and its derivative)
        r.lw = x * fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 144.0f, -1.0f / 30.0f), 0.125f), -1.0f / 3.0f), 0.5f);
        r.dlw = need_d ? fmaf(x, fmaf(x, fmaf(x, fmaf(x, 5.0f / 144.0f, -2.0f / 15.0f), 0.375f), -2.0f / 3.0f), 0.5f) : 0.0f;
    } else {
        const float inv = 1.0f / x;
        r.lw = fmaf(-x, r.e, r.om) * inv;
        r.dlw = need_d ? fmaf(-r.lw, inv, r.e) : 0.0f;
    }
    return r;
}

struct Ray3 {
    float F[3], A[3];
    __device__ void top(float S0, float S1, float t0, float t1) {
        const float S_top = S0 - t0 * (S1 - S0) / (t1 - t0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const ExpTerms et = exp_terms(t0 * c_inv_mu[k], false);
            F[k] = fmaf(S_top, et.om, (S0 - S_top) * et.lw);
            A[k] = et.e;
        }
    }
    __device__ void seg(float Sa, float Sb, float ta, float tb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const ExpTerms et = exp_terms((tb - ta) * c_inv_mu[k], false);
            const float c = fmaf(Sa, et.om, (Sb - Sa) * et.lw);
            F[k] = fmaf(A[k], c, F[k]);
            A[k] *= et.e;
        }
    }
    __device__ float bottom(float Sa, float Sb, float ta, float tb) {
        const float grad = (Sb - Sa) / (tb - ta);
        float out = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float ID = fmaf(c_mu[k], grad, Sb);
            out = fmaf(c_wmu[k], fmaf(A[k], ID, F[k]), out);
        }
        return out;
    }
};

struct PixelSetup {
    float kc;        // continuum per unit mass
    float c1;        // 2 h c^2 / lambda^5 per nm
    float c2;        // h c / (lambda k)
};

__device__ __forceinline__ PixelSetup pixel_setup(const StarDev& s, int i) {
    const double lnl = log(s.lam_first_nm) + (double)i * s.h;
    const double lam_cm = exp(lnl) * 1.0e-7;
    PixelSetup p;
    p.kc = (float)(s.kappa0 * exp(s.alpha * (lnl - log(s.lam_ref_nm))));
    const double l2 = lam_cm * lam_cm;
    p.c1 = (float)(2.0 * H_PLANCK * C_LIGHT * C_LIGHT / (l2 * l2 * lam_cm) * 1.0e-7);
    p.c2 = (float)(H_PLANCK * C_LIGHT / (lam_cm * K_BOLTZ));
    return p;
}

__device__ __forceinline__ float planck(const PixelSetup& p, float invT) {
    return p.c1 / expm1f(p.c2 * invT);
}

// A pixel's kappa_line column kappa_line[j][i], read from global memory or
// from a copy staged in LDS (64 columns interleaved, conflict-free).
struct GlobalKCol {
    const float* p;
    size_t st;
    __device__ __forceinline__ float operator[](int j) const { return p[(size_t)j * st]; }
};
struct LdsKCol {
    const float* p;
    __device__ __forceinline__ float operator[](int j) const { return p[j * WAVE]; }
};

// Copies pixel i's column into col (stride WAVE): sixteen loads in flight per
// wait instead of one per depth step.  Only the calling thread reads it back.
__device__ __forceinline__ void stage_kappa_column(const StarDev& s, int i, float* col) {
    const float* kl = s.kappa + i;
    const int D = s.D;
    for (int j0 = 0; j0 < D; j0 += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = kl[(size_t)min(j0 + u, D - 1) * s.Npad];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (j0 + u < D) col[(j0 + u) * WAVE] = v[u];
    }
}

// tau scan and Gauss-3 flux of pixel i on the total branch (TOT: F) and/or
// the continuum branch (CONT: Fc); both branches share the source function.
template <bool TOT, bool CONT, class KCol>
__device__ __forceinline__ void dev_flux(const StarDev& s, int i, const KCol& kl) {
    if (i >= s.N) return;
    const PixelSetup p = pixel_setup(s, i);
    const int D = s.D;
    float m0 = (float)s.m[0];
    float S0 = planck(p, (float)(1.0 / s.T[0]));
    float chi_t = TOT ? p.kc + kl[0] : 0.0f;
    float tt0 = chi_t * m0;
    float tc0 = p.kc * m0;
    float m1 = (float)s.m[1];
    float S1 = planck(p, (float)(1.0 / s.T[1]));
    float chi_t1 = TOT ? p.kc + kl[1] : 0.0f;
    float tt1 = fmaf(0.5f * (chi_t + chi_t1), m1 - m0, tt0);
    float tc1 = fmaf(p.kc, m1 - m0, tc0);
    Ray3 rt, rc;
    if (TOT) rt.top(S0, S1, tt0, tt1);
    if (CONT) rc.top(S0, S1, tc0, tc1);
    float Sa = S0, Sb = S1, ta = tt0, tb = tt1, ca = tc0, cb = tc1;
    float chi_b = chi_t1, mb = m1;
    for (int j = 1; j < D; ++j) {
        if (j > 1) {
            const float mj = (float)s.m[j];
            Sa = Sb;
            Sb = planck(p, (float)(1.0 / s.T[j]));
            if (TOT) {
                const float chi_j = p.kc + kl[j];
                ta = tb;
                tb = fmaf(0.5f * (chi_b + chi_j), mj - mb, ta);
                chi_b = chi_j;
            }
            if (CONT) {
                ca = cb;
                cb = fmaf(p.kc, mj - mb, ca);
            }
            mb = mj;
        }
        if (TOT) rt.seg(Sa, Sb, ta, tb);
        if (CONT) rc.seg(Sa, Sb, ca, cb);
    }
    if (TOT) s.F[i] = rt.bottom(Sa, Sb, ta, tb);
    if (CONT) s.Fc[i] = rc.bottom(Sa, Sb, ca, cb);
}

// ------------------------------------------------------------ E2 quadrature
// Exponential integrals E_n(x), n = 2..4, x >= 0, in float64:
//   x <= 1: power series E_n(x) = (-x)^{n-1}/(n-1)! (psi(n) - ln x)
//                                 - sum_{k != n-1} (-x)^k / ((k - n + 1) k!),
//           psi(n) = -gamma + sum_{m<n} 1/m;
//   x > 1:  continued fraction E_n(x) = e^{-x} / (x + n - 1 n/(x + n + 2 - 2 (n+1)/(x + n + 4 - ...)))
//           evaluated with the modified Lentz method.
// Both loops have fixed upper bounds.
__device__ __forceinline__ double expint_n(int n, double x) {
    if (x <= 0.0) return 1.0 / (n - 1);
    if (x > 700.0) return 0.0;
    if (x <= 1.0) {
        const double euler = 0.57721566490153286061;
        double psi = -euler;
        for (int m = 1; m < n; ++m) psi += 1.0 / m;
        double term = 1.0;                       // (-x)^k / k!
        double sum = (n == 1) ? 0.0 : -1.0 / (1.0 - n);   // k = 0
        double lead = 0.0;
        for (int k = 1; k < 60; ++k) {
            term *= -x / k;
            if (k == n - 1) {
                lead = term * (psi - log(x));
            } else {
                const double t = term / (k - n + 1);
                sum -= t;
                if (k > n && fabs(t) < 1e-18 * fabs(sum)) break;
            }
        }
        return lead + sum;
    }
    const double tiny = 1e-300;
    double b = x + n, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 400; ++i) {
        const double an = -(double)i * (n - 1 + i);
        b += 2.0;
        d = 1.0 / (an * d + b);
        c = b + an / c;
        const double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return h * exp(-x);
}

// E3(x) and E4(x) = (e^-x - x E3(x)) / 3 (the recurrence E_{n+1} = (e^-x -
// x E_n) / n; its cancellation for large x costs at most ~3 of float64's 16
// digits below x = 700, beyond which both are 0).
__device__ __forceinline__ void expint34(double x, double& E3, double& E4) {
    if (x <= 0.0) {
        E3 = 0.5;
        E4 = 1.0 / 3.0;
        return;
    }
    if (x > 700.0) {
        E3 = 0.0;
        E4 = 0.0;
        return;
    }
    E3 = expint_n(3, x);
    E4 = (exp(-x) - x * E3) * (1.0 / 3.0);
}

// F = 2 pi int_0^inf S E2 dt for piecewise-linear S(tau): segment [ta, tb]
// with S = Sa + s (t - ta) adds Sa (E3(ta) - E3(tb)) + s (E4(ta) - E4(tb) - (tb - ta) E3(tb));
// below the last depth S continues linearly: S_D E3(tau_D) + s_D E4(tau_D);
// above the first depth the top slab runs from tau = 0 with the first slope.
struct RayE2 {
    double F, E3a, E4a;
    __device__ void start() {
        F = 0.0;
        E3a = 0.5;            // E3(0)
        E4a = 1.0 / 3.0;      // E4(0)
    }
    __device__ void seg(double Sa, double Sb, double ta, double tb) {
        double E3b, E4b;
        expint34(tb, E3b, E4b);
        const double sl = (Sb - Sa) / (tb - ta);
        F += Sa * (E3a - E3b) + sl * (E4a - E4b - (tb - ta) * E3b);
        E3a = E3b;
        E4a = E4b;
    }
    __device__ double bottom(double Sa, double Sb, double ta, double tb) const {
        const double sD = (Sb - Sa) / (tb - ta);
        return 2.0 * PI * (F + Sb * E3a + sD * E4a);
    }
};

// E2 flux of pixel i on the total branch (TOT: F) and/or the continuum
// branch (CONT: Fc), float64.
template <bool TOT, bool CONT, class KCol>
__device__ __forceinline__ void dev_flux_e2(const StarDev& s, int i, const KCol& kl) {
    if (i >= s.N) return;
    const double lnl = log(s.lam_first_nm) + (double)i * s.h;
    const double lam_cm = exp(lnl) * 1.0e-7;
    const double kc = s.kappa0 * exp(s.alpha * (lnl - log(s.lam_ref_nm)));
    const double l2 = lam_cm * lam_cm;
    const double c1 = 2.0 * H_PLANCK * C_LIGHT * C_LIGHT / (l2 * l2 * lam_cm) * 1.0e-7;
    const double c2 = H_PLANCK * C_LIGHT / (lam_cm * K_BOLTZ);
    const int D = s.D;
    double S0 = c1 / expm1(c2 / s.T[0]), S1 = c1 / expm1(c2 / s.T[1]);
    double chi0 = TOT ? kc + (double)kl[0] : 0.0, chi1 = TOT ? kc + (double)kl[1] : 0.0;
    double t0 = chi0 * s.m[0], t1 = t0 + 0.5 * (chi0 + chi1) * (s.m[1] - s.m[0]);
    double c0 = kc * s.m[0], cc1 = c0 + kc * (s.m[1] - s.m[0]);
    RayE2 rt, rc;
    rt.start();
    rc.start();
    // top slab: S_top at tau = 0 from the first segment's slope
    if (TOT) rt.seg(S0 - t0 * (S1 - S0) / (t1 - t0), S0, 0.0, t0);
    if (CONT) rc.seg(S0 - c0 * (S1 - S0) / (cc1 - c0), S0, 0.0, c0);
    double Sa = S0, Sb = S1, ta = t0, tb = t1, ca = c0, cb = cc1, chib = chi1, mb = s.m[1];
    for (int j = 1; j < D; ++j) {
        if (j > 1) {
            const double mj = s.m[j];
            Sa = Sb;
            Sb = c1 / expm1(c2 / s.T[j]);
            if (TOT) {
                const double chij = kc + (double)kl[j];
                ta = tb;
                tb = ta + 0.5 * (chib + chij) * (mj - mb);
                chib = chij;
            }
            if (CONT) {
                ca = cb;
                cb = ca + kc * (mj - mb);
            }
            mb = mj;
        }
        if (TOT) rt.seg(Sa, Sb, ta, tb);
        if (CONT) rc.seg(Sa, Sb, ca, cb);
    }
    if (TOT) s.F[i] = (float)rt.bottom(Sa, Sb, ta, tb);
    if (CONT) s.Fc[i] = (float)rc.bottom(Sa, Sb, ca, cb);
}

// Reverse of the E2 flux for the total branch.  With knots t_{-1} = 0,
// t_k = tau_k and slope s_k of segment k, the E2 terms of adjacent segments
// cancel at every knot (S is continuous), leaving
//   segment k >= 1:  dF/dtau_k     += -P_k s_k / dtau_k
//                    dF/dtau_{k-1} += s_k (E3(tau_k) - E3(tau_{k-1})) + P_k s_k / dtau_k,
//                    P_k = E4(t_{k-1}) - E4(t_k) - dtau_k E3(t_k);
//   top slab:        through E3(0) - E3(tau_0), P_0 and the extrapolated S_top;
//   bottom:          dF/dtau_{D-1} += -s_D E3 - E4 s_D/dtau, dF/dtau_{D-2} += E4 s_D/dtau;
// all times 2 pi; then the trapezoid suffix sums as for Gauss-3.
// col: pixel i's float64 LDS column (stride WAVE), holding kappa_line on
// entry and dL/dtau after (each depth written once, as in dev_reverse_scan).
__device__ __forceinline__ void dev_reverse_scan_e2(const StarDev& s, int i, double* col) {
    if (i >= s.N) return;
    const int D = s.D;
    const double G = 2.0 * PI * (double)s.dLdF[i];
    const double lnl = log(s.lam_first_nm) + (double)i * s.h;
    const double lam_cm = exp(lnl) * 1.0e-7;
    const double kc = s.kappa0 * exp(s.alpha * (lnl - log(s.lam_ref_nm)));
    const double l2 = lam_cm * lam_cm;
    const double c1 = 2.0 * H_PLANCK * C_LIGHT * C_LIGHT / (l2 * l2 * lam_cm) * 1.0e-7;
    const double c2 = H_PLANCK * C_LIGHT / (lam_cm * K_BOLTZ);
    const double S0 = c1 / expm1(c2 / s.T[0]), S1 = c1 / expm1(c2 / s.T[1]);
    const double chi0 = kc + col[0], chi1 = kc + col[WAVE];
    const double t0 = chi0 * s.m[0];
    const double t1 = t0 + 0.5 * (chi0 + chi1) * (s.m[1] - s.m[0]);
    const double d01 = t1 - t0, sig = (S1 - S0) / d01;
    double E3a, E4a;
    expint34(t0, E3a, E4a);
    double g0, g1;                                     // top-slab terms of dL/dtau_0, dL/dtau_1
    {
        const double dE3 = 0.5 - E3a;                       // E3(0) - E3(tau_0)
        const double P0 = 1.0 / 3.0 - E4a - t0 * E3a;        // E4(0) - E4(tau_0) - tau_0 E3(tau_0)
        g0 = G * (dE3 * (-sig - t0 * sig / d01) + P0 * sig / d01);
        g1 = G * (dE3 * (t0 * sig / d01) - P0 * sig / d01);
    }
    double Sa = S0, Sb = S1, ta = t0, tb = t1, chib = chi1, mb = s.m[1];
    double pend = g1, last = 0.0;                      // pend: what depth j + 1 already holds
    for (int j = 0; j < D - 1; ++j) {
        if (j > 0) {
            const double mj = s.m[j + 1];
            const double chij = kc + col[(j + 1) * WAVE];
            Sa = Sb;
            ta = tb;
            Sb = c1 / expm1(c2 / s.T[j + 1]);
            tb = ta + 0.5 * (chib + chij) * (mj - mb);
            chib = chij;
            mb = mj;
        }
        double E3b, E4b;
        expint34(tb, E3b, E4b);
        const double dt = tb - ta, sl = (Sb - Sa) / dt;
        const double P = E4a - E4b - dt * E3b;
        const double gj = (j == 0 ? g0 : pend) + G * (sl * (E3b - E3a) + P * sl / dt);
        if (j < D - 2)
            col[j * WAVE] = gj;
        else
            last = gj;
        pend = (j == 0 ? g1 : 0.0) + G * (-P * sl / dt);
        E3a = E3b;
        E4a = E4b;
    }
    {
        const double dt = tb - ta, sD = (Sb - Sa) / dt;
        col[(D - 2) * WAVE] = last + G * (E4a * sD / dt);
        col[(D - 1) * WAVE] = pend + G * (-sD * E3a - E4a * sD / dt);
    }
    double suffix = 0.0, gnext = 0.0;
    float* out = s.gk + i;
    const size_t st = s.Npad;
    for (int j = D - 1; j >= 0; --j) {
        suffix += col[j * WAVE];
        double g = (j == D - 1) ? 0.0 : 0.5 * (s.m[j + 1] - s.m[j]) * gnext;
        g += (j == 0) ? s.m[0] * suffix : 0.5 * (s.m[j] - s.m[j - 1]) * suffix;
        out[(size_t)j * st] = (float)g;
        gnext = suffix;
    }
}

// ---------------------------------------------------------- reverse scan
// dL/dkappa_line[j][i] for the seed dL/dF_i (total branch only: the
// continuum branch depends on no correction).  dF/dtau_k is local in k in the
// summed form of the formal solution:
//   from A_k:           -A_k c_k / mu                        (k <= D-2)
//   from x_j:           +A_j c'_j / mu to tau_{j+1}, -A_j c'_j / mu to tau_j,
//                       c'_j = S_j e_j + (S_{j+1} - S_j) lw'(x_j)
//   bottom:             -A_{D-1} I_D / mu to tau_{D-1};  -/+ A_{D-1} mu dS/dtau^2
//   top slab:           via x_t and S_top (tau_0 and tau_1)
// then dL/dchi_j from the trapezoid tau scan by suffix sums Gamma_j.  The
// suffix sums are small differences of O(A S / mu) terms (S changes little
// between adjacent depths near the surface), so this scan runs in float64;
// only the result is rounded to float32.
struct ExpTerms64 {
    double e, om, lw, dlw;   // e^-x, 1 - e^-x, lw(x), lw'(x)
};

__device__ __forceinline__ ExpTerms64 exp_terms64(double x) {
    ExpTerms64 r;
    r.e = exp(-x);
    r.om = -expm1(-x);
    if (x < 1.0e-2) {
        // sum_{n>=2} (-1)^n (n-1) x^{n-1}/n! and its derivative, through n = 8
        double lw = 0.0, dlw = 0.0, fact = 2.0, xp = 1.0;
#pragma unroll
        for (int n = 2; n <= 8; ++n) {
            if (n > 2) fact *= n;
            const double sg = (n & 1) ? -1.0 : 1.0;
            dlw += sg * (n - 1) * (n - 1) * xp / fact;
            xp *= x;
            lw += sg * (n - 1) * xp / fact;
        }
        r.lw = lw;
        r.dlw = dlw;
    } else {
        r.lw = (r.om - x * r.e) / x;
        r.dlw = r.e - r.lw / x;
    }
    return r;
}

// Pixel i's column of a workgroup of WAVE pixels: col[j * WAVE], float64 in
// LDS.  On entry it holds kappa_line[j][i]; the scan overwrites slot j with
// dL/dtau_j once kappa_line[j] has been read (each slot is written once: the
// term a segment adds to the next depth is carried in a register), then the
// trapezoid adjoint runs up from the bottom.
__device__ __forceinline__ void stage_kappa_column64(const StarDev& s, int i, double* col) {
    const float* kl = s.kappa + i;
    const int D = s.D;
    for (int j0 = 0; j0 < D; j0 += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = kl[(size_t)min(j0 + u, D - 1) * s.Npad];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (j0 + u < D) col[(j0 + u) * WAVE] = (double)v[u];
    }
}

__device__ __forceinline__ void dev_reverse_scan(const StarDev& s, int i, double* col) {
    if (i >= s.N) return;
    const int D = s.D;
    const double G = s.dLdF[i];
    const double mu[3] = {kMu0, kMu1, kMu2};
    const double wmu[3] = {2.0 * PI * 5.0 / 18.0 * kMu0, 2.0 * PI * 8.0 / 18.0 * kMu1, 2.0 * PI * 5.0 / 18.0 * kMu2};
    // pixel constants in float64
    const double lnl = log(s.lam_first_nm) + (double)i * s.h;
    const double lam_cm = exp(lnl) * 1.0e-7;
    const double kc = s.kappa0 * exp(s.alpha * (lnl - log(s.lam_ref_nm)));
    const double l2 = lam_cm * lam_cm;
    const double c1 = 2.0 * H_PLANCK * C_LIGHT * C_LIGHT / (l2 * l2 * lam_cm) * 1.0e-7;
    const double c2 = H_PLANCK * C_LIGHT / (lam_cm * K_BOLTZ);
    // surface quantities
    const double m0 = s.m[0], m1 = s.m[1];
    const double S0 = c1 / expm1(c2 / s.T[0]);
    const double S1 = c1 / expm1(c2 / s.T[1]);
    const double chi0 = kc + col[0], chi1 = kc + col[WAVE];
    const double t0 = chi0 * m0;
    const double t1 = t0 + 0.5 * (chi0 + chi1) * (m1 - m0);
    const double dt01 = t1 - t0;
    const double sig = (S1 - S0) / dt01;
    const double S_top = S0 - t0 * sig;
    double A[3], g0 = 0.0, g1 = 0.0;                    // surface terms of dL/dtau_0, dL/dtau_1
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double Gk = G * wmu[k];
        const ExpTerms64 et = exp_terms64(t0 / mu[k]);
        const double dCdx = S_top * et.e + (S0 - S_top) * et.dlw;
        const double dCdS = et.om - et.lw;
        g0 += Gk * (dCdx / mu[k] + dCdS * (-sig - t0 * sig / dt01));
        g1 += Gk * dCdS * (t0 * sig / dt01);
        A[k] = et.e;
    }
    // segments [j, j + 1]: ga to dL/dtau_j, gb to dL/dtau_{j+1}
    double Sa = S0, Sb = S1, ta = t0, tb = t1, chib = chi1, mb = m1;
    double pend = g1, last = 0.0;                      // pend: what depth j already holds
    for (int j = 0; j < D - 1; ++j) {
        if (j > 0) {
            const double mj = s.m[j + 1];
            const double chij = kc + col[(j + 1) * WAVE];
            Sa = Sb;
            ta = tb;
            Sb = c1 / expm1(c2 / s.T[j + 1]);
            tb = ta + 0.5 * (chib + chij) * (mj - mb);
            chib = chij;
            mb = mj;
        }
        double ga = 0.0, gb = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const ExpTerms64 et = exp_terms64((tb - ta) / mu[k]);
            const double c = Sa * et.om + (Sb - Sa) * et.lw;
            const double dc = Sa * et.e + (Sb - Sa) * et.dlw;
            const double w = G * wmu[k] * A[k] / mu[k];
            ga -= w * (c + dc);
            gb += w * dc;
            A[k] *= et.e;
        }
        const double gj = (j == 0 ? g0 : pend) + ga;   // depth j is complete but for the bottom term
        if (j < D - 2)
            col[j * WAVE] = gj;
        else
            last = gj;
        pend = j == 0 ? g1 + gb : gb;
    }
    // bottom boundary (Sa, Sb, ta, tb are now the last segment)
    {
        const double dS = Sb - Sa, dtl = tb - ta;
        double g_last = 0.0, g_prev = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double Gk = G * wmu[k] * A[k];
            const double ID = Sb + mu[k] * dS / dtl;
            const double q = mu[k] * dS / (dtl * dtl);
            g_last += Gk * (-ID / mu[k] - q);
            g_prev += Gk * q;
        }
        col[(D - 2) * WAVE] = last + g_prev;
        col[(D - 1) * WAVE] = pend + g_last;
    }
    // dL/dchi_j from the trapezoid rule via suffix sums
    double suffix = 0.0, gnext = 0.0;
    float* out = s.gk + i;
    const size_t st = s.Npad;
    for (int j = D - 1; j >= 0; --j) {
        suffix += col[j * WAVE];
        double g = (j == D - 1) ? 0.0 : 0.5 * (s.m[j + 1] - s.m[j]) * gnext;
        g += (j == 0) ? s.m[0] * suffix : 0.5 * (s.m[j] - s.m[j - 1]) * suffix;
        out[(size_t)j * st] = (float)g;
        gnext = suffix;
    }
}

// -------------------------------------------------------- gather (adjoint)
// One wavefront per line: its lanes are 8 pixels x 8 depth groups and step
// through the window 8 pixels at a time; the line's per-depth parameters stay
// in registers.  The Voigt function and its derivatives are recomputed:
//   dL/d dgf   = ln10 sum g K H
//   dL/d ddamp = ln10 sum g K a dH/da
//   dL/d xi    = sum g (-K) (H + a dH/da + v dH/dv) d ln dnu_D / d xi,
//   d ln dnu_D / d xi = xi / dv^2 = xi (s / c)^2 with s = c/dv  (per km/s: x 1e10)
// A fixed-order butterfly reduces across lanes, so the sums are deterministic.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
    return x;
}

// Far-wing series for the gather, |z|^2 = v^2 + a^2 >= 64 and b = a^2 <= 4.
// The asymptotic expansion w(z) ~ (i/sqrt(pi)) sum_n (2n-1)!!/2^n z^-(2n+1),
// its real part re-expanded in r = 1/|z|^2 (Im z^(2n+1) = a sum_j
// C(2n+1, 2j+1) (-b)^j (1/r - b)^(n-j)), gives with d|z|^2/da = 2a and
// d|z|^2/dv = 2v
//   H       = (a/sqrt(pi)) r sum_m e_m r^m,
//   a dH/da = (a/sqrt(pi)) r sum_m (e_m + 2b e_m' - 2b m e_(m-1)) r^m,
//   X = H + a dH/da + v dH/dv = (a/sqrt(pi)) r sum_(m>=1) (2b e_m' - 2m e_m) r^m,
// e_0 = 1, e_1 = 3/2, e_2 = 15/4 - 2b, e_3 = 105/8 - 15b,
// e_4 = 945/16 - 105b + 12b^2 (X's leading orders cancel in closed form).
// Cut after r^4, in float32, against the float64 Faddeeva function over
// |z| >= 8, b <= 4: H within 6.9e-7, a dH/da 1.5e-5, X 9.1e-5 relative (the
// node-pair sums: 1e-6, 1e-6, 1.6e-4), in 34 operations against 43.
static constexpr float kFarZ2 = 64.0f, kFarB = 4.0f;

// The series' sums: H = c r ph, a dH/da = c r pa, X = c r^2 px, c = a/sqrt(pi).
__device__ __forceinline__ void far_series(float b, float z2, float& r, float& ph, float& pa, float& px) {
    r = __builtin_amdgcn_rcpf(z2);
    const float e2 = fmaf(-2.0f, b, 3.75f), e3 = fmaf(-15.0f, b, 13.125f);
    const float e4 = fmaf(fmaf(12.0f, b, -105.0f), b, 59.0625f);
    const float f1 = fmaf(-2.0f, b, 1.5f), f2 = fmaf(-12.0f, b, 3.75f);
    const float f3 = fmaf(fmaf(12.0f, b, -67.5f), b, 13.125f);
    const float f4 = fmaf(fmaf(180.0f, b, -420.0f), b, 59.0625f);
    const float g2 = fmaf(4.0f, b, -15.0f), g3 = fmaf(60.0f, b, -78.75f);
    const float g4 = fmaf(fmaf(-48.0f, b, 630.0f), b, -472.5f);
    ph = fmaf(fmaf(fmaf(fmaf(e4, r, e3), r, e2), r, 1.5f), r, 1.0f);
    pa = fmaf(fmaf(fmaf(fmaf(f4, r, f3), r, f2), r, f1), r, 1.0f);
    px = fmaf(fmaf(fmaf(g4, r, g3), r, g2), r, -3.0f);
}

// One call per wavefront; l must be wavefront-uniform; pw holds the H and L
// core tables and lq the line's rows written by stage_line_params (both LDS).
// A step whose lanes are all at |z|^2 >= 64 with a^2 <= 4 takes the far-wing
// series, other steps voigt_KHD.
// FAM: the damping term is split over the three families by their share of
// the width at each depth, w_beta = Gamma_beta / Gamma.
template <bool CT, bool FAM>
__device__ __forceinline__ void gather_body(const StarDev& s, int l, int lane, const float4* pw, const float4* lq) {
    constexpr int WPX = 8, NDG = 8, DPT = (MAXD + NDG - 1) / NDG;
    const int px = lane % WPX, dg = lane / WPX;
    int ilo = s.ln.ilo[l], ihi = s.ln.ihi[l];
    const int ic = s.ln.ic[l];
    const float delta = s.ln.delta[l];
    const int D = s.D;
    const float4* lp = lq;
    const float* zm = CT ? s.zmax + (size_t)l * D : nullptr;
    if (CT) {
        // pixels whose detuning x = expm1(delta - k h) can reach the line's
        // largest span: |x| <= xl  <=>  delta - k h in [log1p(-xl), log1p(xl)]
        const double xl = (double)s.xlim[l] * (1.0 + 1e-5);
        if (!(xl > 0.0)) {
            ihi = ilo - 1;                                // no depth kept
        } else if (xl < 1e-2) {
            const double h = s.h, dl = (double)delta;
            ilo = max(ilo, ic + (int)floor((dl - log1p(xl)) / h) - 1);
            ihi = min(ihi, ic + (int)ceil((dl - log1p(-xl)) / h) + 1);
        }
    }
    float sgf = 0.0f, sd = 0.0f, sxi = 0.0f, sds = 0.0f, sdw = 0.0f;
    for (int p0 = ilo; p0 <= ihi; p0 += WPX) {
        const int i = p0 + px;
        if (i <= ihi) {
            const float x = detuning(i - ic, delta, s.h_hi, s.h_lo);
            const float* g = s.gk + i;
#pragma unroll 1
            for (int d = 0; d < DPT; ++d) {
                const int j = d * NDG + dg;
                if (j < D) {
                    const float4 q = lp[j];
                    const float v = x * q.x;
                    if (CT && !(fmaf(v, v, q.y) <= zm[j])) continue;
                    const float gj = g[(size_t)j * s.Npad];
                    const float u = v * v, z2 = u + q.y;
                    const float4 e = lp[MAXD + j];
                    // g K H = w th, g K a dH/da = w ta, g K X e.x = w tx
                    float w, th, ta, tx;
                    if (wave_all(z2 >= kFarZ2) && wave_all(q.y <= kFarB)) {
                        float r;
                        far_series(q.y, z2, r, th, ta, tx);
                        w = (gj * r) * (q.w * kInvSqrtPiF);
                        tx *= r * e.x;
                    } else {
                        voigt_KHD(q.y, q.z, q.w, v, u, pw, th, ta, tx);
                        w = gj;
                        tx *= e.x;
                    }
                    sgf = fmaf(w, th, sgf);
                    sxi = fmaf(w, tx, sxi);
                    if (FAM) {
                        const float t = w * ta;
                        sd = fmaf(t, e.y, sd);
                        sds = fmaf(t, e.z, sds);
                        sdw = fmaf(t, e.w, sdw);
                    } else {
                        sd = fmaf(w, ta, sd);
                    }
                }
            }
        }
    }
    sgf = wave_sum(sgf);
    sd = wave_sum(sd);
    sxi = wave_sum(sxi);
    if (FAM) {
        sds = wave_sum(sds);
        sdw = wave_sum(sdw);
    }
    if (lane == 0) {
        s.gline[l] = (float)LN10 * sgf;
        s.gline[s.L + l] = (float)LN10 * sd;
        s.gline[2 * s.L + l] = sxi;
        if (FAM) {
            s.gline[3 * s.L + l] = (float)LN10 * sds;
            s.gline[4 * s.L + l] = (float)LN10 * sdw;
        }
    }
}

__device__ __forceinline__ void dev_gather(const StarDev& s, int l, int lane, const float4* pw, const float4* lq) {
    if (l >= s.L) return;
    if (s.fam) {
        if (s.center)
            gather_body<true, true>(s, l, lane, pw, lq);
        else
            gather_body<false, true>(s, l, lane, pw, lq);
    } else {
        if (s.center)
            gather_body<true, false>(s, l, lane, pw, lq);
        else
            gather_body<false, false>(s, l, lane, pw, lq);
    }
}

// A wavefront copies line l's per-depth parameters to its LDS rows (l must
// be wavefront-uniform; nothing for l >= L): lq[j] = (c/dv, a^2, K, K a) and
// lq[MAXD + j] = (-xi (c/dv)^2 per km/s -- the microturbulence factor of the
// xi term, with its sign -- and, with damping families, the radiative, Stark
// and van der Waals shares of the width at depth j).
__device__ __forceinline__ void stage_line_params(const StarDev& s, int l, int lane, float4* lq) {
    if (l >= s.L) return;
    const float xi_f = s.xi[0] * (float)(1.0e10 / (C_LIGHT * C_LIGHT));
    float gr = 0.0f, gs = 0.0f, gw = 0.0f;
    if (s.fam) {
        const double4 c = s.lc[l];
        gr = (float)c.y;
        gs = (float)c.z;
        gw = (float)c.w;
    }
    for (int k = lane; k < s.D; k += WAVE) {
        const float4 q = s.lp[(size_t)l * s.D + k];
        lq[k] = q;
        float4 e = make_float4(-xi_f * q.x * q.x, 0.0f, 0.0f, 0.0f);
        if (s.fam) {
            const float Gs = gs * (float)s.ne[k], Gw = gw * (float)s.npert[k];
            const float inv = 1.0f / (gr + Gs + Gw);
            e.y = gr * inv;
            e.z = Gs * inv;
            e.w = Gw * inv;
        }
        lq[MAXD + k] = e;
    }
}

// ----------------------------------------------------------- reductions
__device__ __forceinline__ void dev_scatter(const StarDev& s, int l) {
    if (l >= s.L) return;
    const int c = s.ln.perm[l];
    if (s.g_loggf) s.g_loggf[c] = s.gline[l];
    if (s.g_damp) {
        s.g_damp[c] = s.gline[s.L + l];
        if (s.fam) {                                      // [3][L]: radiative, Stark, van der Waals
            s.g_damp[s.L + c] = s.gline[3 * s.L + l];
            s.g_damp[2 * s.L + c] = s.gline[4 * s.L + l];
        }
    }
}

// Abundance gradient of species b = sum of the dgf gradients of its lines
// (10^dA and 10^dgf scale the same strength at fixed atmosphere);
// microturbulence = sum of the per-line terms.  Two fixed-order levels:
// block (c, b) sums chunk c (RCHUNK lines) of list b into partial[b][c]
// (b = S is the xi list), then one block per list sums its partials.
__device__ __forceinline__ float block_sum256(float acc, float* red) {
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// 256-thread workgroups.
__device__ __forceinline__ void dev_reduce_partial(const StarDev& s, int c, int b, float* red) {
    int o0, o1;
    if (b < s.S) {
        o0 = s.sp_off[b] + c * RCHUNK;
        o1 = min(s.sp_off[b + 1], o0 + RCHUNK);
    } else {
        o0 = c * RCHUNK;
        o1 = min(s.L, o0 + RCHUNK);
    }
    if (o0 >= o1) {
        if (threadIdx.x == 0) s.partial[b * s.n_rchunk + c] = 0.0f;
        return;
    }
    float acc = 0.0f;
    if (b < s.S) {
        for (int k = o0 + threadIdx.x; k < o1; k += 256) acc += s.gline[s.sp_idx[k]];
    } else {
        for (int k = o0 + threadIdx.x; k < o1; k += 256) acc += s.gline[2 * s.L + k];
    }
    const float tot = block_sum256(acc, red);
    if (threadIdx.x == 0) s.partial[b * s.n_rchunk + c] = tot;
}

__device__ __forceinline__ void dev_reduce_final(const StarDev& s, int b, float* red) {
    float acc = 0.0f;
    for (int c = threadIdx.x; c < s.n_rchunk; c += 256) acc += s.partial[b * s.n_rchunk + c];
    const float tot = block_sum256(acc, red);
    if (threadIdx.x == 0) {
        if (b < s.S) {
            if (s.g_abund) s.g_abund[b] = tot;
        } else if (s.g_xi) {
            s.g_xi[0] = tot;
        }
    }
}

// ------------------------------------------------------------- loss seed
// f = F/Fc, r = 2 (f - y)/sigma^2: dL/dF = r/Fc, dL/dFc = -r F/Fc^2.
__device__ __forceinline__ void dev_chi2_seed(int N, const float* F, const float* Fc, const float* y, float inv_s2,
                                              float* gF, float* gFc, int i) {
    if (i >= N) return;
    const float inv_c = 1.0f / Fc[i];
    const float f = F[i] * inv_c;
    const float r = 2.0f * (f - y[i]) * inv_s2;
    gF[i] = r * inv_c;
    if (gFc) gFc[i] = -r * f * inv_c;
}

// One 1024-thread workgroup: fixed-order sum of ((f - y)/sigma)^2.
__device__ __forceinline__ void dev_chi2_loss(int N, const float* F, const float* Fc, const float* y, float inv_s2,
                                              float* loss, float* red) {
    float acc = 0.0f;
    for (int i = threadIdx.x; i < N; i += 1024) {
        const float d = F[i] / Fc[i] - y[i];
        acc = fmaf(d * d, inv_s2, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
}

}  // namespace pz
