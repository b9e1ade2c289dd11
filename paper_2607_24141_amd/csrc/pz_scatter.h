// Transfer with continuum scattering (Sec. 2.1, Eqs. 3 and 6-8), per pixel in
// float64.  With sigma_c the scattering opacity per unit mass,
//   chi = kappa_abs + sigma_c,  eps = kappa_abs / chi,  S = eps B + (1 - eps) J,
// kappa_abs = kappa_c + sum kappa_line (total branch) or kappa_c (continuum
// branch).  J = Lambda S is the mean intensity of the discretised formal
// solution (piecewise-linear S in tau, linear extrapolation to tau = 0 over the
// surface segment, diffusion lower boundary I = S + mu dS/dtau; inward I = 0 at
// tau = 0), J_j = 1/2 sum_k w_k (I+_j(mu_k) + I-_j(mu_k)) on the 3-point
// Gauss-Legendre nodes of the flux.
//
// Forward: the fixed point S* = eps B + (1 - eps) Lambda S* by accelerated
// Lambda iteration (Jacobi with the diagonal Lambda*_jj of the same operator):
//   S <- S + (eps B + (1 - eps) Lambda S - S) / (1 - (1 - eps) Lambda*),
// from S = B until max_j |dS_j / S_j| <= tol (or the iteration cap), every
// fourth iteration followed by Ng's extrapolation from the last four iterates
// (Ng 1974: the combination of them whose next differences are smallest in
// the relative least-squares sense), then the
// emergent flux F = 2 pi sum_k w_k mu_k I+(0, mu_k).  Six threads per pixel:
// the two branches, and in each the three ray directions, which sweep their
// share of J in parallel and then update a third of the depths each.
//
// Backward (total branch): with gS = dF/dS* G and gtau the direct flux terms,
// the adjoint lambda solves (I - diag(1 - eps) Lambda)^T lambda = gS by the same
// preconditioned iteration with Lambda^T; then
//   dL/deps_j = lambda_j (B_j - J*_j),
//   dL/dtau  += VJP of J(S*, tau) with the cotangent (1 - eps) lambda,
//   dL/dchi   = trapezoid adjoint of dL/dtau,
//   dL/dkappa_line_j = dL/dchi_j + dL/deps_j sigma_j / chi_j^2.
// It runs on the same three threads per pixel (one per ray direction), reuses
// the forward's segment tables, so no exponential is evaluated, and adds the
// directions' partial sums in a fixed order.
// Workspace columns are [D] with stride Npad (coalesced across pixels).
#pragma once

namespace pz {

struct Col {
    double* p;
    size_t st;
    __device__ __forceinline__ double& operator[](int j) const { return p[(size_t)j * st]; }
};

// workspace arrays (each [D][Npad] float64): per branch b (tau, eps, S, Ld, B, the three
// per-direction parts of J, the segment coefficients of each direction m: e^-x, 1 - e^-x, lw(x)
// of the segment ending at depth j, j >= 1, and of the surface segment [0, tau_0] at j = 0, and
// the three previous iterates of S), then
// the backward's lambda, right-hand side and one intensity profile per direction.  The backward
// keeps its per-direction partial sums in the continuum branch's columns, which it does not need.
enum { SC_BR = 0, SC_TAU = 0, SC_EPS = 1, SC_S = 2, SC_LD = 3, SC_B = 4, SC_JM = 5, SC_CE = 8, SC_CO = 11,
       SC_CL = 14, SC_H = 17, SC_PER_BR = 20, SC_LAM = 40, SC_RHS = 41, SC_IS = 42, SC_NARR = 45 };
static_assert(SC_NARR == SC_WS_ARRAYS, "scattering workspace size");

__device__ __forceinline__ Col sc_col(const StarDev& s, int id, int i) {
    return Col{s.sc + (size_t)id * s.D * s.Npad + i, (size_t)s.Npad};
}
__device__ __forceinline__ Col sc_bcol(const StarDev& s, int b, int k, int i) {
    return sc_col(s, SC_BR + SC_PER_BR * b + k, i);
}
__device__ __forceinline__ double sc_mu(int k) { return k == 0 ? kMu0 : (k == 1 ? kMu1 : kMu2); }
__device__ __forceinline__ double sc_hw(int k) { return k == 1 ? 0.5 * 8.0 / 18.0 : 0.5 * 5.0 / 18.0; }   // w_k / 2

// d(S_top)/d(tau_0), d(S_top)/d(tau_1) with S_top = S_0 - tau_0 (S_1 - S_0) / (tau_1 - tau_0)
__device__ __forceinline__ void sc_top_dtau(const Col& tau, const Col& S, double& d0, double& d1) {
    const double t0 = tau[0], dt = tau[1] - t0, sig = (S[1] - S[0]) / dt;
    d0 = -sig - t0 * sig / dt;
    d1 = t0 * sig / dt;
}

struct ScPixel {
    double kc, c1, c2, fs;   // continuum, Planck constants, sigma scale (lambda/lambda_ref)^sigma_alpha
};

__device__ __forceinline__ ScPixel sc_pixel(const StarDev& s, int i) {
    const double lnl = log(s.lam_first_nm) + (double)i * s.h;
    const double lam_cm = exp(lnl) * 1.0e-7;
    ScPixel p;
    p.kc = s.kappa0 * exp(s.alpha * (lnl - log(s.lam_ref_nm)));
    const double l2 = lam_cm * lam_cm;
    p.c1 = 2.0 * H_PLANCK * C_LIGHT * C_LIGHT / (l2 * l2 * lam_cm) * 1.0e-7;
    p.c2 = H_PLANCK * C_LIGHT / (lam_cm * K_BOLTZ);
    p.fs = exp(s.sigma_alpha * (lnl - log(s.lam_ref_nm)));
    return p;
}

// tau, eps and B of branch b; S starts at B
__device__ inline void sc_setup(const StarDev& s, int i, int b, const ScPixel& p) {
    const int D = s.D;
    const Col B = sc_bcol(s, b, SC_B, i), tau = sc_bcol(s, b, SC_TAU, i), eps = sc_bcol(s, b, SC_EPS, i),
              S = sc_bcol(s, b, SC_S, i);
    const float* kl = s.kappa + i;
    double chi_prev = 0.0, t = 0.0;
    for (int j = 0; j < D; ++j) {
        const double ka = p.kc + (b == 0 ? (double)kl[(size_t)j * s.Npad] : 0.0);
        const double chi = ka + s.sigma_c[j] * p.fs;
        t = (j == 0) ? chi * s.m[0] : t + 0.5 * (chi_prev + chi) * (s.m[j] - s.m[j - 1]);
        chi_prev = chi;
        tau[j] = t;
        eps[j] = ka / chi;
        const double Bj = p.c1 / expm1(p.c2 / s.T[j]);
        B[j] = Bj;
        S[j] = Bj;
    }
}

// Segment coefficients of direction m (see the workspace layout)
__device__ inline void sc_coeffs(int D, const Col& tau, int m, const Col& CE, const Col& CO, const Col& CL) {
    const double mu = sc_mu(m);
    double ta = 0.0;
    for (int j = 0; j < D; ++j) {
        const double tb = tau[j];
        const ExpTerms64 et = exp_terms64((tb - ta) / mu);
        CE[j] = et.e;
        CO[j] = et.om;
        CL[j] = et.lw;
        ta = tb;
    }
}

// Lambda*_jj for the depths j = m, m + 3, ... (the coefficient of S_j in J_j),
// from the coefficients of all three directions
__device__ inline void sc_lambda_diag_part(int D, const Col& tau, const Col& Ld, int m, const Col* CE, const Col* CO,
                                           const Col* CL) {
    const double t0 = tau[0], c = t0 / (tau[1] - t0), gD = 1.0 / (tau[D - 1] - tau[D - 2]);
    for (int j = m; j < D; j += 3) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double mu = sc_mu(k);
            double out, in;
            if (j == D - 1) {
                out = 1.0 + mu * gD;
            } else {
                out = CO[k][j + 1] - CL[k][j + 1];
                if (j == D - 2) out -= CE[k][j + 1] * mu * gD;
            }
            if (j == 0) {
                in = CO[k][0] + c * CL[k][0];
            } else {
                in = CO[k][j] - CL[k][j];
                if (j == 1) in -= CE[k][1] * c * CL[k][0];
            }
            acc += sc_hw(k) * (out + in);
        }
        Ld[j] = acc;
    }
}

// Jm = w_m/2 (I+ + I-) along direction m (one third of J = Lambda S)
__device__ inline void sc_lambda_mu(int D, const Col& tau, const Col& S, const Col& Jm, int m, const Col& CE,
                                    const Col& CO, const Col& CL) {
    const double mu = sc_mu(m), hw = sc_hw(m);
    double I;
    {
        const double t0 = tau[0], S0 = S[0];
        const double S_top = S0 - t0 * (S[1] - S0) / (tau[1] - t0);
        I = S0 * CO[0] + (S_top - S0) * CL[0];
        Jm[0] = hw * I;
    }
    double Sa = S[0];
    for (int j = 1; j < D; ++j) {
        const double Sb = S[j];
        I = I * CE[j] + Sb * CO[j] + (Sa - Sb) * CL[j];
        Jm[j] = hw * I;
        Sa = Sb;
    }
    const double SD = S[D - 1];
    I = SD + mu * (SD - S[D - 2]) / (tau[D - 1] - tau[D - 2]);
    Jm[D - 1] += hw * I;
    double Sb = SD;
    for (int j = D - 2; j >= 0; --j) {
        const double Sj = S[j];
        I = I * CE[j + 1] + Sj * CO[j + 1] + (Sb - Sj) * CL[j + 1];
        Jm[j] += hw * I;
        Sb = Sj;
    }
}

// 2 pi w_m mu_m I+(0, mu_m) of S
__device__ inline double sc_flux_mu(int D, const Col& tau, const Col& S, int m, const Col& CE, const Col& CO,
                                    const Col& CL) {
    const double mu = sc_mu(m);
    const double SD = S[D - 1];
    double I = SD + mu * (SD - S[D - 2]) / (tau[D - 1] - tau[D - 2]);
    double Sb = SD;
    for (int j = D - 2; j >= 0; --j) {
        const double Sj = S[j];
        I = I * CE[j + 1] + Sj * CO[j + 1] + (Sb - Sj) * CL[j + 1];
        Sb = Sj;
    }
    const double t0 = tau[0], S0 = S[0];
    const double S_top = S0 - t0 * (S[1] - S0) / (tau[1] - t0);
    return 2.0 * PI * 2.0 * sc_hw(m) * mu * (I * CE[0] + S_top * CO[0] + (S0 - S_top) * CL[0]);
}

// Ng's extrapolation of one pixel's S from x0 = S (iterate it) and the
// previous iterates x1, x2, x3 in H[(it - k) % 3]: with d0 = x0 - x1,
// d1 = x1 - x2, d2 = x2 - x3 and weights 1/x0^2, (a, b) minimise
// |d0 - a (d0 - d1) - b (d0 - d2)|^2 and S <- (1 - a - b) x0 + a x1 + b x2;
// the one-term form (b = 0) when d0 - d1 and d0 - d2 are nearly parallel.
// Called by every thread of the workgroup (it synchronises it); ng: the
// pixel is still iterating.  The depth sums are split over the three
// direction threads and added in a fixed order.
__device__ inline void sc_ng_step(int D, const Col& S, const Col* H, int it, bool ng, int m, int tx,
                                  double (*ngs)[3][64]) {
    const Col &h1 = H[(it - 1) % 3], &h2 = H[(it - 2) % 3], &h3 = H[(it - 3) % 3];
    double p[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (ng) {
        for (int j = m; j < D; j += 3) {
            const double x0 = S[j], x1 = h1[j], x2 = h2[j], x3 = h3[j];
            const double d0 = x0 - x1, u = d0 - (x1 - x2), v = d0 - (x2 - x3), w = 1.0 / (x0 * x0);
            p[0] += w * u * u;
            p[1] += w * u * v;
            p[2] += w * v * v;
            p[3] += w * d0 * u;
            p[4] += w * d0 * v;
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) ngs[k][m][tx] = p[k];
    __syncthreads();
    if (m == 0 && ng) {
        double q[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) q[k] = ngs[k][0][tx] + ngs[k][1][tx] + ngs[k][2][tx];
        const double det = q[0] * q[2] - q[1] * q[1];
        double a = 0.0, c = 0.0;
        if (det > 1e-10 * q[0] * q[2]) {
            a = (q[3] * q[2] - q[4] * q[1]) / det;
            c = (q[4] * q[0] - q[3] * q[1]) / det;
        } else if (q[0] > 0.0) {
            a = q[3] / q[0];
        }
        if (!(isfinite(a) && isfinite(c))) a = c = 0.0;
        ngs[0][0][tx] = a;
        ngs[1][0][tx] = c;
    }
    __syncthreads();
    if (ng) {
        const double a = ngs[0][0][tx], c = ngs[1][0][tx];
        for (int j = m; j < D; j += 3) S[j] = (1.0 - a - c) * S[j] + a * h1[j] + c * h2[j];
    }
    __syncthreads();
}

// Forward of one branch for 64 pixels: a workgroup of 64 x 3 threads,
// threadIdx.y = m the ray direction (called by every thread: it synchronises
// the workgroup).  Each iteration every direction sweeps into its part of J;
// then each thread updates the depths j = m (mod 3) of its pixel.  A pixel
// stops at max_j |dS_j / S_j| <= tol or the cap and its S is then frozen, so
// its result does not depend on the other pixels of the workgroup.
__device__ inline void dev_flux_scatter(const StarDev& s, int i, int b) {
    __shared__ double red[3][64];
    __shared__ double ngs[5][3][64];
    __shared__ int done[64];
    const int tx = threadIdx.x, m = threadIdx.y, D = s.D;
    const bool px = i < s.N;
    const Col tau = sc_bcol(s, b, SC_TAU, i), eps = sc_bcol(s, b, SC_EPS, i), S = sc_bcol(s, b, SC_S, i),
              Ld = sc_bcol(s, b, SC_LD, i), B = sc_bcol(s, b, SC_B, i);
    const Col Jm[3] = {sc_bcol(s, b, SC_JM, i), sc_bcol(s, b, SC_JM + 1, i), sc_bcol(s, b, SC_JM + 2, i)};
    const Col CE[3] = {sc_bcol(s, b, SC_CE, i), sc_bcol(s, b, SC_CE + 1, i), sc_bcol(s, b, SC_CE + 2, i)};
    const Col CO[3] = {sc_bcol(s, b, SC_CO, i), sc_bcol(s, b, SC_CO + 1, i), sc_bcol(s, b, SC_CO + 2, i)};
    const Col CL[3] = {sc_bcol(s, b, SC_CL, i), sc_bcol(s, b, SC_CL + 1, i), sc_bcol(s, b, SC_CL + 2, i)};
    const Col H[3] = {sc_bcol(s, b, SC_H, i), sc_bcol(s, b, SC_H + 1, i), sc_bcol(s, b, SC_H + 2, i)};
    if (px && m == 0) sc_setup(s, i, b, sc_pixel(s, i));
    if (m == 0) done[tx] = px ? 0 : 1;
    __syncthreads();
    if (px) sc_coeffs(D, tau, m, CE[m], CO[m], CL[m]);
    __syncthreads();
    if (px) sc_lambda_diag_part(D, tau, Ld, m, CE, CO, CL);
    int it = 0;
    for (;;) {
        const bool active = px && !done[tx];
        if (active) sc_lambda_mu(D, tau, S, Jm[m], m, CE[m], CO[m], CL[m]);
        __syncthreads();
        double dmax = 0.0;
        if (active) {
            const Col& Hs = H[it % 3];                // iterate `it` becomes history
            for (int j = m; j < D; j += 3) {
                const double e = eps[j], Sj = S[j];
                const double J = Jm[0][j] + Jm[1][j] + Jm[2][j];
                const double Sn = Sj + (e * B[j] + (1.0 - e) * J - Sj) / (1.0 - (1.0 - e) * Ld[j]);
                dmax = fmax(dmax, fabs(Sn - Sj) / fabs(Sn));
                Hs[j] = Sj;
                S[j] = Sn;
            }
        }
        red[m][tx] = dmax;
        ++it;
        __syncthreads();
        if (m == 0 && active) {
            const double d = fmax(red[0][tx], fmax(red[1][tx], red[2][tx]));
            if (d <= s.sc_tol || it >= s.sc_max_iter) {
                done[tx] = 1;
                if (s.sc_iters) s.sc_iters[b * s.Npad + i] = it;
            }
        }
        __syncthreads();
        if (it % 4 == 0) sc_ng_step(D, S, H, it, px && !done[tx], m, tx, ngs);
        if (!__syncthreads_or(!done[tx])) break;
    }
    const double f = px ? sc_flux_mu(D, tau, S, m, CE[m], CO[m], CL[m]) : 0.0;
    red[m][tx] = f;
    __syncthreads();
    if (px && m == 0) {
        float* out = b == 0 ? s.F : s.Fc;
        if (out) out[i] = (float)(red[0][tx] + red[1][tx] + red[2][tx]);
    }
}

// lw'(x) = e^-x - lw(x) / x of a segment of length x with coefficients e^-x and lw(x)
__device__ __forceinline__ double sc_dlw(double e, double lw, double x) { return e - lw / x; }

// I+_j along direction m into IS (bottom-up), from the segment tables
__device__ inline void sc_out_mu(int D, const Col& tau, const Col& S, int m, const Col& CE, const Col& CO,
                                 const Col& CL, const Col& IS) {
    const double SD = S[D - 1];
    double I = SD + sc_mu(m) * (SD - S[D - 2]) / (tau[D - 1] - tau[D - 2]);
    IS[D - 1] = I;
    double Sb = SD;
    for (int j = D - 2; j >= 0; --j) {
        const double Sj = S[j];
        I = I * CE[j + 1] + Sj * CO[j + 1] + (Sb - Sj) * CL[j + 1];
        IS[j] = I;
        Sb = Sj;
    }
}

// I-_j along direction m into IS (top-down)
__device__ inline void sc_in_mu(int D, const Col& tau, const Col& S, const Col& CE, const Col& CO, const Col& CL,
                                const Col& IS) {
    const double t0 = tau[0], S0 = S[0];
    const double S_top = S0 - t0 * (S[1] - S0) / (tau[1] - t0);
    double I = S0 * CO[0] + (S_top - S0) * CL[0];
    IS[0] = I;
    double Sa = S0;
    for (int j = 1; j < D; ++j) {
        const double Sb = S[j];
        I = I * CE[j] + Sb * CO[j] + (Sa - Sb) * CL[j];
        IS[j] = I;
        Sa = Sb;
    }
}

// Direction m's part of the flux VJP for the seed G = dL/dF: its dF/dS G into gS and its tau
// terms into gt (both overwritten); leaves I+ of S in IS.
__device__ inline void sc_flux_vjp_mu(int D, const Col& tau, const Col& S, double G, int m, const Col& CE,
                                      const Col& CO, const Col& CL, const Col& IS, const Col& gS, const Col& gt) {
    sc_out_mu(D, tau, S, m, CE, CO, CL, IS);
    for (int j = 2; j < D; ++j) {
        gS[j] = 0.0;
        gt[j] = 0.0;
    }
    const double mu = sc_mu(m);
    const double t0 = tau[0], S0 = S[0], dt01 = tau[1] - t0;
    const double S_top = S0 - t0 * (S[1] - S0) / dt01;
    double d0, d1;
    sc_top_dtau(tau, S, d0, d1);
    const double g0 = G * 2.0 * PI * 2.0 * sc_hw(m) * mu;           // dL/dI(0, mu_m)
    {
        const double e = CE[0], lw = CL[0], dlw = sc_dlw(e, lw, t0 / mu);
        const double gStop = g0 * (CO[0] - lw);
        gt[0] = g0 * (-IS[0] * e + S_top * e + (S0 - S_top) * dlw) / mu + gStop * d0;
        gt[1] = gStop * d1;
        gS[0] = g0 * lw + gStop * (1.0 + t0 / dt01);
        gS[1] = gStop * (-t0 / dt01);
    }
    double Gk = g0 * CE[0];                                           // dL/dI+(tau_0)
    for (int j = 0; j < D - 1; ++j) {
        const double Sj = S[j], Sn = S[j + 1];
        const double e = CE[j + 1], lw = CL[j + 1], dlw = sc_dlw(e, lw, (tau[j + 1] - tau[j]) / mu);
        const double gx = Gk * (-IS[j + 1] * e + Sj * e + (Sn - Sj) * dlw) / mu;
        gS[j] += Gk * (CO[j + 1] - lw);
        gS[j + 1] += Gk * lw;
        gt[j + 1] += gx;
        gt[j] -= gx;
        Gk *= e;
    }
    {
        const double dS = S[D - 1] - S[D - 2], dt = tau[D - 1] - tau[D - 2];
        gS[D - 1] += Gk * (1.0 + mu / dt);
        gS[D - 2] -= Gk * mu / dt;
        const double gd = Gk * (-mu * dS / (dt * dt));
        gt[D - 1] += gd;
        gt[D - 2] -= gd;
    }
}

// out = direction m's part of Lambda^T v (overwritten).  Each sweep carries the pending term of
// the next depth, so the first sweep writes every element once and the second adds once.
__device__ inline void sc_lambda_T_mu(int D, const Col& tau, const Col& v, const Col& out, int m, const Col& CE,
                                      const Col& CO, const Col& CL) {
    const double mu = sc_mu(m), hw = sc_hw(m);
    // transpose of the outward sweep, surface first
    double G = 0.0, carry = 0.0;
    for (int j = 0; j < D - 1; ++j) {
        G += hw * v[j];
        const double lw = CL[j + 1];
        out[j] = carry + G * (CO[j + 1] - lw);
        carry = G * lw;
        G *= CE[j + 1];
    }
    {
        const double g = mu / (tau[D - 1] - tau[D - 2]);
        G += hw * v[D - 1];
        out[D - 1] = carry + G * (1.0 + g);
        out[D - 2] -= G * g;
    }
    // transpose of the inward sweep, deepest first
    G = 0.0;
    carry = 0.0;
    for (int j = D - 1; j >= 1; --j) {
        G += hw * v[j];
        const double lw = CL[j];
        out[j] += carry + G * (CO[j] - lw);
        carry = G * lw;
        G *= CE[j];
    }
    {
        const double t0 = tau[0], c = t0 / (tau[1] - t0);
        G += hw * v[0];
        out[0] += carry + G * (CO[0] + c * CL[0]);
        out[1] -= G * c * CL[0];
    }
}

// Adds to gt direction m's tau terms of the VJP of J(S, tau) for the cotangent u.  IS holds I+ of
// S on entry and I- of S on exit.
__device__ inline void sc_lambda_tau_vjp_mu(int D, const Col& tau, const Col& S, const Col& u, int m, const Col& CE,
                                            const Col& CO, const Col& CL, const Col& IS, const Col& gt) {
    const double mu = sc_mu(m), hw = sc_hw(m);
    // outward: reverse sweep from the surface over the stored I+
    double G = 0.0;
    for (int j = 0; j < D - 1; ++j) {
        const double Sj = S[j], Sn = S[j + 1];
        G += hw * u[j];
        const double e = CE[j + 1], dlw = sc_dlw(e, CL[j + 1], (tau[j + 1] - tau[j]) / mu);
        const double gx = G * (-IS[j + 1] * e + Sj * e + (Sn - Sj) * dlw) / mu;
        G *= e;
        gt[j + 1] += gx;
        gt[j] -= gx;
    }
    {
        const double dS = S[D - 1] - S[D - 2], dt = tau[D - 1] - tau[D - 2];
        G += hw * u[D - 1];
        const double gd = G * (-mu * dS / (dt * dt));
        gt[D - 1] += gd;
        gt[D - 2] -= gd;
    }
    // inward: profiles, then the reverse sweep from the deepest layer
    sc_in_mu(D, tau, S, CE, CO, CL, IS);
    G = 0.0;
    for (int j = D - 1; j >= 1; --j) {
        const double Sj = S[j], Sp = S[j - 1];
        G += hw * u[j];
        const double e = CE[j], dlw = sc_dlw(e, CL[j], (tau[j] - tau[j - 1]) / mu);
        const double gx = G * (-IS[j - 1] * e + Sj * e + (Sp - Sj) * dlw) / mu;
        G *= e;
        gt[j] += gx;
        gt[j - 1] -= gx;
    }
    {
        const double t0 = tau[0], S0 = S[0];
        const double S_top = S0 - t0 * (S[1] - S0) / (tau[1] - t0);
        double d0, d1;
        sc_top_dtau(tau, S, d0, d1);
        G += hw * u[0];
        const double e = CE[0], lw = CL[0], dlw = sc_dlw(e, lw, t0 / mu);
        gt[0] += G * (S0 * e + (S_top - S0) * dlw) / mu + G * lw * d0;
        gt[1] += G * lw * d1;
    }
}

// Backward of the total branch for 64 pixels: a workgroup of 64 x 3 threads,
// threadIdx.y = m the ray direction (called by every thread: it synchronises
// the workgroup).  Needs the forward's tau, eps, S*, Lambda* and segment tables
// of the total branch; writes dL/dkappa_line into gk.  A pixel's adjoint
// iteration stops at max_j |d lambda_j| <= tol max_j |lambda_j| or the cap.
__device__ inline void dev_reverse_scatter(const StarDev& s, int i) {
    __shared__ double red[2][3][64];
    __shared__ int done[64];
    const int tx = threadIdx.x, m = threadIdx.y, D = s.D;
    const bool px = i < s.N;
    const Col B = sc_bcol(s, 0, SC_B, i), tau = sc_bcol(s, 0, SC_TAU, i), eps = sc_bcol(s, 0, SC_EPS, i),
              S = sc_bcol(s, 0, SC_S, i), Ld = sc_bcol(s, 0, SC_LD, i);
    const Col CE = sc_bcol(s, 0, SC_CE + m, i), CO = sc_bcol(s, 0, SC_CO + m, i), CL = sc_bcol(s, 0, SC_CL + m, i);
    const Col lam = sc_col(s, SC_LAM, i), rhs = sc_col(s, SC_RHS, i), IS = sc_col(s, SC_IS + m, i);
    // per-direction parts: Lambda^T (1 - eps) lambda, dF/dS G, tau terms (continuum-branch columns)
    // and J* (the total branch's own J parts)
    const Col U = sc_bcol(s, 1, SC_S, i);
    const Col Tm[3] = {sc_bcol(s, 1, SC_JM, i), sc_bcol(s, 1, SC_JM + 1, i), sc_bcol(s, 1, SC_JM + 2, i)};
    const Col gS[3] = {sc_bcol(s, 1, SC_CE, i), sc_bcol(s, 1, SC_CE + 1, i), sc_bcol(s, 1, SC_CE + 2, i)};
    const Col gt[3] = {sc_bcol(s, 1, SC_CO, i), sc_bcol(s, 1, SC_CO + 1, i), sc_bcol(s, 1, SC_CO + 2, i)};
    const Col Jm[3] = {sc_bcol(s, 0, SC_JM, i), sc_bcol(s, 0, SC_JM + 1, i), sc_bcol(s, 0, SC_JM + 2, i)};
    if (px) sc_flux_vjp_mu(D, tau, S, (double)s.dLdF[i], m, CE, CO, CL, IS, gS[m], gt[m]);
    if (m == 0) done[tx] = px ? 0 : 1;
    __syncthreads();
    if (px) {
        for (int j = m; j < D; j += 3) {
            const double r = gS[0][j] + gS[1][j] + gS[2][j];
            rhs[j] = r;
            lam[j] = r;
            U[j] = (1.0 - eps[j]) * r;
        }
    }
    __syncthreads();
    // adjoint fixed point: lambda = rhs + Lambda^T ((1 - eps) lambda)
    int it = 0;
    for (;;) {
        const bool active = px && !done[tx];
        if (active) sc_lambda_T_mu(D, tau, U, Tm[m], m, CE, CO, CL);
        __syncthreads();
        double dmax = 0.0, lmax = 0.0;
        if (active) {
            for (int j = m; j < D; j += 3) {
                const double e = eps[j], lj = lam[j];
                const double T = Tm[0][j] + Tm[1][j] + Tm[2][j];
                const double ln = lj + (rhs[j] + T - lj) / (1.0 - (1.0 - e) * Ld[j]);
                dmax = fmax(dmax, fabs(ln - lj));
                lmax = fmax(lmax, fabs(ln));
                lam[j] = ln;
                U[j] = (1.0 - e) * ln;
            }
        }
        red[0][m][tx] = dmax;
        red[1][m][tx] = lmax;
        ++it;
        __syncthreads();
        if (m == 0 && active) {
            const double d = fmax(red[0][0][tx], fmax(red[0][1][tx], red[0][2][tx]));
            const double l = fmax(red[1][0][tx], fmax(red[1][1][tx], red[1][2][tx]));
            if (d <= s.sc_tol * l || it >= s.sc_max_iter) {
                done[tx] = 1;
                if (s.sc_iters) s.sc_iters[2 * s.Npad + i] = it;
            }
        }
        __syncthreads();
        if (!__syncthreads_or(!done[tx])) break;
    }
    // J* and the tau terms of the fixed point, per direction
    if (px) {
        sc_lambda_mu(D, tau, S, Jm[m], m, CE, CO, CL);
        sc_lambda_tau_vjp_mu(D, tau, S, U, m, CE, CO, CL, IS, gt[m]);
    }
    __syncthreads();
    if (!px || m != 0) return;
    // dL/dchi by the trapezoid adjoint, then dL/dkappa_line
    const ScPixel p = sc_pixel(s, i);
    const float* kl = s.kappa + i;
    float* out = s.gk + i;
    double suffix = 0.0, gnext = 0.0;
    for (int j = D - 1; j >= 0; --j) {
        suffix += gt[0][j] + gt[1][j] + gt[2][j];
        double gchi = (j == D - 1) ? 0.0 : 0.5 * (s.m[j + 1] - s.m[j]) * gnext;
        gchi += (j == 0) ? s.m[0] * suffix : 0.5 * (s.m[j] - s.m[j - 1]) * suffix;
        gnext = suffix;
        const double sig = s.sigma_c[j] * p.fs;
        const double chi = p.kc + (double)kl[(size_t)j * s.Npad] + sig;
        const double geps = lam[j] * (B[j] - (Jm[0][j] + Jm[1][j] + Jm[2][j]));
        out[(size_t)j * s.Npad] = (float)(gchi + geps * sig / (chi * chi));
    }
}

}  // namespace pz
