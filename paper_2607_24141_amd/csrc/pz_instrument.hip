// Instrument operator of Eq. 31 (and Eq. 9) on the GPU: Gaussian broadening
// B(v_b) on the logarithmic synthesis grid, an optional rotational broadening
// R(v sin i) (Sec. 7 names a GPU-resident rotational kernel without defining
// it), Doppler shift S(v_r), and a Gaussian line-spread function sampled at
// the observed pixels (K), applied to both the total and the continuum flux
// before their ratio,
//     f_p = {K S R B F}_p / {K S R B F_c}_p ,
// with the vector-Jacobian product for F, F_c, v_r, v_b and v sin i.
//
// Discretisation (x = ln lambda, native x_i = x_0 + i h):
//   B: (B G)_i = sum_{|k|<=J} g_k G_{i-k} / Z_i, g_k = exp(-k^2 / (2 s^2)),
//      s = v_b / (c h) pixels, Z_i the sum of the g_k whose G_{i-k} exists;
//      J fixed at creation from the largest v_b.
//   R: (R G)_i = sum_{|k|<=JR} r_k G_{i-k} / ZR_i, r_k the integral over the
//      pixel cell [k - 1/2, k + 1/2] of the rotation profile of a linearly
//      limb-darkened disc (limb-darkening coefficient eps) scaled to the
//      half-width s = v sin i / (c h) pixels; the profile in y = u / s is
//      [2 (1 - eps) sqrt(1 - y^2) + (pi eps / 2)(1 - y^2)] / [pi (1 - eps/3)]
//      and its antiderivative is closed form, so r_k is a difference of two
//      antiderivative values (taken in FP64); JR fixed at creation from the
//      largest v sin i, ZR_i the sum of the r_k whose G_{i-k} exists.
//   S: (S G)_i = (1 - r) G_{i+m} + r G_{i+m+1}, i - t = i + m + r,
//      t = ln(1 + v_r/c) / h, m = floor(-t), indices clamped to the grid.
//   K: (K H)_p = sum_i w_pi H_i / W_p over the pixels within T LSF widths,
//      w_pi = exp(-(i - c_p)^2 a_p), a_p = h^2 / (2 sigma_p^2).
// The transposes are gathers (each output owned by one thread); the two
// velocity gradients are fixed-order two-level sums.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "pz_internal.h"

namespace pz {
int set_error(int code, const char* msg);
}

using namespace pz;

struct pz_inst {
    int N, P, J, JR, nblk;
    double h, eps;
    // per observed pixel: LSF support [lo, hi], centre c_p = lo + off, a_p
    int* lo;
    int* hi;
    float* off;
    float* ap;
    // per native pixel: observed pixels whose support holds it, [plo, phi]
    int* plo;
    int* phi;
    // workspace
    float* BF;     // [2][N] broadened total, continuum
    float* Z;      // [N]    broadening normalisers
    float* RBF;    // [2][N] rotated R B F, R B Fc (rotation only)
    float* ZR;     // [N]    rotation normalisers (rotation only)
    float* dR;     // [2][N] dL/d(R B F) (rotation only)
    float* KW;     // [P]    LSF weight sums
    float* dY;     // [2][P] dL/d(K S B F) / W_p, both branches
    float* dS;     // [2][N] dL/d(S B F)
    float* dB;     // [2][N] dL/d(B F)
    float* part;   // [3][nblk] partial sums of dL/dt, dL/ds and dL/ds_rot
    void* base;
};

namespace {

constexpr int TPB = 256;
constexpr double C_KMS = 2.99792458e5;
constexpr int MAX_J = 1024;

struct Vel {
    double t;        // shift in pixels
    int m;           // floor(-t)
    float r;         // -t - m, in [0, 1)
    float s;         // broadening width in pixels
    bool s_clamped;  // s held at its floor (identity broadening, zero gradient)
};

__device__ __forceinline__ Vel velocities(const float* vel, double h) {
    Vel v;
    v.t = log1p((double)vel[0] / C_KMS) / h;
    const double fm = floor(-v.t);
    v.m = (int)fm;
    v.r = (float)(-v.t - fm);
    const float s = (float)((double)vel[1] / (C_KMS * h));
    v.s_clamped = !(s > 1e-3f);
    v.s = v.s_clamped ? 1e-3f : s;
    return v;
}

__device__ __forceinline__ void load_taps(float* g, int J, float s) {
    const float c = -0.5f / (s * s);
    for (int k = threadIdx.x; k <= J; k += blockDim.x) g[k] = __expf(c * (float)(k * k));
    __syncthreads();
}

// B for both branches; also the normalisers Z.
__global__ __launch_bounds__(TPB) void k_broaden(int N, int J, double h, const float* vel, const float* F,
                                                 const float* Fc, float* BF, float* Z) {
    extern __shared__ float g[];
    const Vel v = velocities(vel, h);
    load_taps(g, J, v.s);
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= N) return;
    float a = 0.0f, b = 0.0f, z = 0.0f;
    const int k0 = max(-J, i - (N - 1)), k1 = min(J, i);       // 0 <= i - k < N
    for (int k = k0; k <= k1; ++k) {
        const float w = g[abs(k)];
        a = fmaf(w, F[i - k], a);
        b = fmaf(w, Fc[i - k], b);
        z += w;
    }
    const float iz = 1.0f / z;
    BF[i] = a * iz;
    BF[N + i] = b * iz;
    Z[i] = z;
}

// K S for both branches at observed pixel p; with dL_df also the scaled seeds.
__global__ __launch_bounds__(TPB) void k_lsf(int N, int P, double h, const float* vel, const int* lo, const int* hi,
                                             const float* off, const float* ap, const float* BF, float* KF, float* KFc,
                                             float* f, const float* dL_df, float* KW, float* dY) {
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= P) return;
    const Vel v = velocities(vel, h);
    const int l0 = lo[p], l1 = hi[p];
    const float o = off[p], a = ap[p];
    float sf = 0.0f, sc = 0.0f, W = 0.0f;
    for (int i = l0; i <= l1; ++i) {
        const float d = (float)(i - l0) - o;
        const float w = __expf(-d * d * a);
        const int k0 = min(max(i + v.m, 0), N - 1), k1 = min(max(i + v.m + 1, 0), N - 1);
        sf = fmaf(w, fmaf(v.r, BF[k1] - BF[k0], BF[k0]), sf);
        sc = fmaf(w, fmaf(v.r, BF[N + k1] - BF[N + k0], BF[N + k0]), sc);
        W += w;
    }
    const float kf = sf / W, kc = sc / W, fr = kf / kc;
    if (KF) KF[p] = kf;
    if (KFc) KFc[p] = kc;
    if (f) f[p] = fr;
    if (dL_df) {
        const float g = dL_df[p];
        KW[p] = W;
        dY[p] = g / kc / W;                 // dL/dKF_p / W_p
        dY[P + p] = -g * fr / kc / W;       // dL/dKFc_p / W_p
    }
}

// K^T: dS_i = sum_p w_pi dY_p over the observed pixels whose support holds i.
__global__ __launch_bounds__(TPB) void k_lsf_T(int N, int P, const int* lo, const float* off, const float* ap,
                                               const int* plo, const int* phi, const float* dY, float* dS) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= N) return;
    float a = 0.0f, b = 0.0f;
    for (int p = plo[i]; p <= phi[i]; ++p) {
        const float d = (float)(i - lo[p]) - off[p];
        const float w = __expf(-d * d * ap[p]);
        a = fmaf(w, dY[p], a);
        b = fmaf(w, dY[P + p], b);
    }
    dS[i] = a;
    dS[N + i] = b;
}

__device__ __forceinline__ float block_sum(float x, float* red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// Rotation profile of unit integral on |y| <= 1 and its antiderivative from -1.
__device__ __forceinline__ double rot_pdf(double y, double eps) {
    const double q = fmax(1.0 - y * y, 0.0);
    return (2.0 * (1.0 - eps) * sqrt(q) + 0.5 * M_PI * eps * q) / (M_PI * (1.0 - eps / 3.0));
}

__device__ __forceinline__ double rot_cdf(double y, double eps) {
    y = fmin(fmax(y, -1.0), 1.0);
    const double a = (1.0 - eps) * (y * sqrt(fmax(1.0 - y * y, 0.0)) + asin(y));
    const double b = 0.5 * M_PI * eps * (y - y * y * y / 3.0);
    return (a + b) / (M_PI * (1.0 - eps / 3.0)) + 0.5;
}

// Rotation half-width in pixels from vel[2] (not positive: the identity).
__device__ __forceinline__ double rot_width(const float* vel, double h) { return (double)vel[2] / (C_KMS * h); }

// Cell weights r_k and dr_k/ds for k = 0..JR into LDS (the profile is even, so
// r_{-k} = r_k).  A cell bound y = b/s moves as -y/s with s, unless clamped at +-1.
__device__ __forceinline__ void load_rot(float* r, float* dr, int JR, double s, double eps) {
    for (int k = threadIdx.x; k <= JR; k += blockDim.x) {
        if (!(s > 0.0)) {
            r[k] = k == 0 ? 1.0f : 0.0f;
            dr[k] = 0.0f;
            continue;
        }
        const double lo = (k - 0.5) / s, hi = (k + 0.5) / s;
        r[k] = (float)(rot_cdf(hi, eps) - rot_cdf(lo, eps));
        const double dhi = fabs(hi) < 1.0 ? rot_pdf(hi, eps) * (-hi / s) : 0.0;
        const double dlo = fabs(lo) < 1.0 ? rot_pdf(lo, eps) * (-lo / s) : 0.0;
        dr[k] = (float)(dhi - dlo);
    }
    __syncthreads();
}

// R for both branches; also the normalisers ZR.
__global__ __launch_bounds__(TPB) void k_rotate(int N, int JR, double h, double eps, const float* vel,
                                                const float* BF, float* RBF, float* ZR) {
    extern __shared__ float rw[];
    load_rot(rw, rw + JR + 1, JR, rot_width(vel, h), eps);
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= N) return;
    float a = 0.0f, b = 0.0f, z = 0.0f;
    const int k0 = max(-JR, i - (N - 1)), k1 = min(JR, i);     // 0 <= i - k < N
    for (int k = k0; k <= k1; ++k) {
        const float w = rw[abs(k)];
        a = fmaf(w, BF[i - k], a);
        b = fmaf(w, BF[N + i - k], b);
        z += w;
    }
    const float iz = 1.0f / z;
    RBF[i] = a * iz;
    RBF[N + i] = b * iz;
    ZR[i] = z;
}

// R^T: dB_j = sum_k r_k dR_{j+k} / ZR_{j+k}; and the per-block partial of
// dL/ds_rot = sum_i dR_i d(R G)_i/ds with d(R G)_i/ds = sum_k r'_k (G_{i-k} - (R G)_i) / ZR_i
// (the quotient rule with the normalised mean taken out of every tap first,
// which keeps float cancellation small where G is nearly flat).
__global__ __launch_bounds__(TPB) void k_rotate_T(int N, int JR, double h, double eps, const float* vel,
                                                  const float* BF, const float* RBF, const float* ZR,
                                                  const float* dR, float* dB, float* part) {
    extern __shared__ float rw[];
    __shared__ float red[TPB];
    const float* dr = rw + JR + 1;
    load_rot(rw, rw + JR + 1, JR, rot_width(vel, h), eps);
    const int j = blockIdx.x * TPB + threadIdx.x;
    float ds = 0.0f;
    if (j < N) {
        float a = 0.0f, b = 0.0f;
        const int k0 = max(-JR, -j), k1 = min(JR, N - 1 - j);        // 0 <= j + k < N
        for (int k = k0; k <= k1; ++k) {
            const float w = rw[abs(k)] / ZR[j + k];
            a = fmaf(w, dR[j + k], a);
            b = fmaf(w, dR[N + j + k], b);
        }
        dB[j] = a;
        dB[N + j] = b;
        const float m0 = RBF[j], m1 = RBF[N + j];
        float d0 = 0.0f, d1 = 0.0f;
        const int q0 = max(-JR, j - (N - 1)), q1 = min(JR, j);       // 0 <= j - k < N
        for (int k = q0; k <= q1; ++k) {
            const float w = dr[abs(k)];
            d0 = fmaf(w, BF[j - k] - m0, d0);
            d1 = fmaf(w, BF[N + j - k] - m1, d1);
        }
        ds = (dR[j] * d0 + dR[N + j] * d1) / ZR[j];
    }
    const float tot = block_sum(ds, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// S^T, and the per-block partial of dL/dt = sum_i dS_i d(S B F)_i/dt,
// d(S G)_i/dt = -(G_{i+m+1} - G_{i+m}) where neither index is clamped.
__global__ __launch_bounds__(TPB) void k_shift_T(int N, double h, const float* vel, const float* BF, const float* dS,
                                                 float* dB, float* part) {
    __shared__ float red[TPB];
    const Vel v = velocities(vel, h);
    const int j = blockIdx.x * TPB + threadIdx.x;
    float dt = 0.0f;
    if (j < N) {
        for (int br = 0; br < 2; ++br) {
            const float* s = dS + br * N;
            float acc = 0.0f;
            // the k0 tap reaches j from i with clamp(i + m) == j, the k1 tap with clamp(i + m + 1) == j
            for (int tap = 0; tap < 2; ++tap) {
                const float wt = tap == 0 ? 1.0f - v.r : v.r;
                const int off = v.m + tap;                 // index = clamp(i + off)
                int i0, i1;                                // i range mapping onto j
                if (j == 0) {
                    i0 = 0;
                    i1 = min(N - 1, -off);
                } else if (j == N - 1) {
                    i0 = max(0, N - 1 - off);
                    i1 = N - 1;
                } else {
                    i0 = i1 = j - off;
                }
                i0 = max(i0, 0);
                i1 = min(i1, N - 1);
                for (int i = i0; i <= i1; ++i) acc = fmaf(wt, s[i], acc);
            }
            dB[br * N + j] = acc;
            // dL/dt term of output pixel i = j
            const int k0 = j + v.m, k1 = k0 + 1;
            if (k0 >= 0 && k1 <= N - 1) dt = fmaf(s[j], -(BF[br * N + k1] - BF[br * N + k0]), dt);
        }
    }
    const float tot = block_sum(dt, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// B^T: dF_j = sum_k g_k dB_{j+k} / Z_{j+k}; and the per-block partial of
// dL/ds = sum_i dB_i d(B G)_i/ds, d(B G)_i/ds = (N'_i Z_i - N_i Z'_i) / Z_i^2,
// N_i = sum g_k G_{i-k}, g'_k = g_k k^2 / s^3.
__global__ __launch_bounds__(TPB) void k_broaden_T(int N, int J, double h, const float* vel, const float* F,
                                                   const float* Fc, const float* Z, const float* dB, float* dF,
                                                   float* dFc, float* part) {
    extern __shared__ float g[];
    __shared__ float red[TPB];
    const Vel v = velocities(vel, h);
    load_taps(g, J, v.s);
    const int j = blockIdx.x * TPB + threadIdx.x;
    float ds = 0.0f;
    if (j < N) {
        float a = 0.0f, b = 0.0f;
        const int k0 = max(-J, -j), k1 = min(J, N - 1 - j);          // 0 <= j + k < N
        for (int k = k0; k <= k1; ++k) {
            const float w = g[abs(k)] / Z[j + k];
            a = fmaf(w, dB[j + k], a);
            b = fmaf(w, dB[N + j + k], b);
        }
        if (dF) dF[j] = a;
        if (dFc) dFc[j] = b;
        if (!v.s_clamped) {
            const float is3 = 1.0f / (v.s * v.s * v.s);
            float n0 = 0.0f, n1 = 0.0f, dn0 = 0.0f, dn1 = 0.0f, dz = 0.0f;
            const int q0 = max(-J, j - (N - 1)), q1 = min(J, j);       // 0 <= j - k < N
            for (int k = q0; k <= q1; ++k) {
                const float w = g[abs(k)], dw = w * (float)(k * k) * is3;
                n0 = fmaf(w, F[j - k], n0);
                n1 = fmaf(w, Fc[j - k], n1);
                dn0 = fmaf(dw, F[j - k], dn0);
                dn1 = fmaf(dw, Fc[j - k], dn1);
                dz += dw;
            }
            const float z = Z[j], iz2 = 1.0f / (z * z);
            ds = dB[j] * (dn0 * z - n0 * dz) * iz2 + dB[N + j] * (dn1 * z - n1 * dz) * iz2;
        }
    }
    const float tot = block_sum(ds, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One workgroup: fixed-order sums of the partials -> dL/dv_r, dL/dv_b and,
// with rotation, dL/d(v sin i).
__global__ __launch_bounds__(TPB) void k_vel_final(int nblk, int rot, double h, const float* vel, const float* part,
                                                   float* g_vel) {
    __shared__ float red[TPB];
    const Vel v = velocities(vel, h);
    float a = 0.0f, b = 0.0f, c = 0.0f;
    for (int k = threadIdx.x; k < nblk; k += TPB) {
        a += part[k];
        b += part[nblk + k];
        if (rot) c += part[2 * nblk + k];
    }
    const float dt = block_sum(a, red);
    const float ds = block_sum(b, red);
    const float dsr = rot ? block_sum(c, red) : 0.0f;
    if (threadIdx.x == 0) {
        g_vel[0] = (float)((double)dt / (h * (C_KMS + (double)vel[0])));     // t = ln(1 + v_r/c) / h
        g_vel[1] = v.s_clamped ? 0.0f : (float)((double)ds / (C_KMS * h));  // s = v_b / (c h)
        if (rot) g_vel[2] = (float)((double)dsr / (C_KMS * h));             // s_rot = v sin i / (c h)
    }
}

int fail_hip(hipError_t e, const char* what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return set_error(PZ_E_HIP, buf);
}

#define INST_HIP(call)                                     \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return fail_hip(e_, #call);  \
    } while (0)

}  // namespace

extern "C" {

int pz_inst_create(const pz_grid* grid, const pz_inst_desc* d, pz_inst** out) {
    if (!out) return set_error(PZ_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !d || !d->lam_obs_nm || !d->lsf_sigma_ln)
        return set_error(PZ_E_INVALID_ARG, "grid, desc and its arrays are required");
    if (!(grid->lam_first_nm > 0.0) || !(grid->R > 0.0) || grid->N < 2 || !std::isfinite(grid->lam_first_nm) ||
        !std::isfinite(grid->R))
        return set_error(PZ_E_INVALID_ARG, "invalid grid");
    if (d->P < 1) return set_error(PZ_E_SHAPE, "P must be >= 1");
    const double T = d->lsf_trunc == 0.0 ? 4.0 : d->lsf_trunc;
    if (!(T > 0.0) || !std::isfinite(T)) return set_error(PZ_E_INVALID_ARG, "lsf_trunc must be finite and >= 0");
    if (!(d->vb_max_kms > 0.0) || !std::isfinite(d->vb_max_kms))
        return set_error(PZ_E_INVALID_ARG, "vb_max_kms must be finite and > 0");
    const int N = grid->N, P = d->P;
    const double h = std::log1p(1.0 / grid->R), x0 = std::log(grid->lam_first_nm);
    const double Jd = std::ceil(4.0 * d->vb_max_kms / C_KMS / h);
    if (Jd > MAX_J) return set_error(PZ_E_INVALID_ARG, "vb_max_kms gives a broadening support above 1024 pixels");
    const int J = (int)Jd;
    if (!(d->vrot_max_kms >= 0.0) || !std::isfinite(d->vrot_max_kms))
        return set_error(PZ_E_INVALID_ARG, "vrot_max_kms must be finite and >= 0");
    if (!(d->limb_eps >= 0.0 && d->limb_eps <= 1.0))
        return set_error(PZ_E_INVALID_ARG, "limb_eps must lie in [0, 1]");
    // rotation support: the cells [k - 1/2, k + 1/2] that reach |u| <= s_max
    const double JRd = d->vrot_max_kms > 0.0 ? std::ceil(d->vrot_max_kms / C_KMS / h + 0.5) : 0.0;
    if (JRd > MAX_J) return set_error(PZ_E_INVALID_ARG, "vrot_max_kms gives a rotation support above 1024 pixels");
    const int JR = (int)JRd;
    std::vector<int> lo(P), hi(P);
    std::vector<float> off(P), ap(P);
    for (int p = 0; p < P; ++p) {
        const double lam = d->lam_obs_nm[p], s = d->lsf_sigma_ln[p];
        if (!(lam > 0.0) || !std::isfinite(lam) || !(s > 0.0) || !std::isfinite(s))
            return set_error(PZ_E_INVALID_ARG, "observed pixels need finite lam_obs_nm > 0 and lsf_sigma_ln > 0");
        if (p > 0 && !(lam > d->lam_obs_nm[p - 1]))
            return set_error(PZ_E_INVALID_ARG, "lam_obs_nm must be strictly increasing");
        const double c = (std::log(lam) - x0) / h, half = T * s / h;
        const double a = std::ceil(c - half), b = std::floor(c + half);
        if (a < 0.0 || b > N - 1 || a > b)
            return set_error(PZ_E_INVALID_ARG, "an observed pixel's LSF support leaves the synthesis grid");
        lo[p] = (int)a;
        hi[p] = (int)b;
        off[p] = (float)(c - a);
        ap[p] = (float)(1.0 / (2.0 * (s / h) * (s / h)));      // per pixel^2
    }
    // native pixel -> observed pixels whose support holds it (supports are intervals with
    // non-decreasing ends, so each native pixel sees a contiguous range of p)
    std::vector<int> plo(N, 0), phi(N, -1);
    for (int p = P - 1; p >= 0; --p)
        for (int i = lo[p]; i <= hi[p]; ++i) plo[i] = p;
    for (int p = 0; p < P; ++p)
        for (int i = lo[p]; i <= hi[p]; ++i) phi[i] = p;
    for (int p = 1; p < P; ++p)
        if (lo[p] < lo[p - 1] || hi[p] < hi[p - 1])
            return set_error(PZ_E_INVALID_ARG, "LSF supports must not shrink backwards (sigma varies too fast)");
    const int nblk = (N + TPB - 1) / TPB;
    size_t offb = 0;
    auto take = [&](size_t bytes) {
        const size_t o = offb;
        offb = (offb + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_lo = take(P * 4), o_hi = take(P * 4), o_off = take(P * 4), o_ap = take(P * 4),
                 o_plo = take((size_t)N * 4), o_phi = take((size_t)N * 4), o_BF = take((size_t)2 * N * 4),
                 o_Z = take((size_t)N * 4), o_KW = take(P * 4), o_dY = take((size_t)2 * P * 4),
                 o_dS = take((size_t)2 * N * 4), o_dB = take((size_t)2 * N * 4), o_part = take((size_t)3 * nblk * 4),
                 o_RBF = take(JR ? (size_t)2 * N * 4 : 0), o_ZR = take(JR ? (size_t)N * 4 : 0),
                 o_dR = take(JR ? (size_t)2 * N * 4 : 0);
    pz_inst* in = new (std::nothrow) pz_inst();
    if (!in) return set_error(PZ_E_NOMEM, "host allocation failed");
    char* base = nullptr;
    if (hipMalloc((void**)&base, offb) != hipSuccess) {
        (void)hipGetLastError();
        delete in;
        return set_error(PZ_E_NOMEM, "hipMalloc failed for the instrument workspace");
    }
    in->N = N;
    in->P = P;
    in->J = J;
    in->JR = JR;
    in->nblk = nblk;
    in->h = h;
    in->eps = d->limb_eps;
    in->base = base;
    in->lo = (int*)(base + o_lo);
    in->hi = (int*)(base + o_hi);
    in->off = (float*)(base + o_off);
    in->ap = (float*)(base + o_ap);
    in->plo = (int*)(base + o_plo);
    in->phi = (int*)(base + o_phi);
    in->BF = (float*)(base + o_BF);
    in->Z = (float*)(base + o_Z);
    in->KW = (float*)(base + o_KW);
    in->dY = (float*)(base + o_dY);
    in->dS = (float*)(base + o_dS);
    in->dB = (float*)(base + o_dB);
    in->part = (float*)(base + o_part);
    in->RBF = JR ? (float*)(base + o_RBF) : nullptr;
    in->ZR = JR ? (float*)(base + o_ZR) : nullptr;
    in->dR = JR ? (float*)(base + o_dR) : nullptr;
    hipError_t e = hipMemcpy(in->lo, lo.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(in->hi, hi.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(in->off, off.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(in->ap, ap.data(), P * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(in->plo, plo.data(), (size_t)N * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(in->phi, phi.data(), (size_t)N * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete in;
        return fail_hip(e, "hipMemcpy");
    }
    *out = in;
    return PZ_OK;
}

void pz_inst_destroy(pz_inst* in) {
    if (!in) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(in->base);
    delete in;
}

int pz_inst_forward(const pz_inst* in, const float* F, const float* Fc, const float* vel, float* KF, float* KFc,
                    float* f, pz_stream stream) {
    if (!in || !F || !Fc || !vel) return set_error(PZ_E_INVALID_ARG, "inst, F, Fc and vel are required");
    if (!KF && !KFc && !f) return set_error(PZ_E_INVALID_ARG, "no output requested");
    hipStream_t st = (hipStream_t)stream;
    const int gN = (in->N + TPB - 1) / TPB;
    const size_t lds = (size_t)(in->J + 1) * 4;
    k_broaden<<<gN, TPB, lds, st>>>(in->N, in->J, in->h, vel, F, Fc, in->BF, in->Z);
    if (in->JR)
        k_rotate<<<gN, TPB, (size_t)2 * (in->JR + 1) * 4, st>>>(in->N, in->JR, in->h, in->eps, vel, in->BF, in->RBF,
                                                                in->ZR);
    const float* src = in->JR ? in->RBF : in->BF;
    k_lsf<<<(in->P + TPB - 1) / TPB, TPB, 0, st>>>(in->N, in->P, in->h, vel, in->lo, in->hi, in->off, in->ap, src, KF,
                                                   KFc, f, nullptr, nullptr, nullptr);
    INST_HIP(hipGetLastError());
    return PZ_OK;
}

int pz_inst_backward(const pz_inst* in, const float* F, const float* Fc, const float* vel, const float* dL_df,
                     float* dL_dF, float* dL_dFc, float* g_vel, pz_stream stream) {
    if (!in || !F || !Fc || !vel || !dL_df) return set_error(PZ_E_INVALID_ARG, "inst, F, Fc, vel and dL_df are required");
    if (!dL_dF && !dL_dFc && !g_vel) return set_error(PZ_E_INVALID_ARG, "no output requested");
    hipStream_t st = (hipStream_t)stream;
    const int gN = (in->N + TPB - 1) / TPB;
    const size_t lds = (size_t)(in->J + 1) * 4;
    const size_t ldsr = (size_t)2 * (in->JR + 1) * 4;
    k_broaden<<<gN, TPB, lds, st>>>(in->N, in->J, in->h, vel, F, Fc, in->BF, in->Z);
    if (in->JR) k_rotate<<<gN, TPB, ldsr, st>>>(in->N, in->JR, in->h, in->eps, vel, in->BF, in->RBF, in->ZR);
    const float* src = in->JR ? in->RBF : in->BF;
    k_lsf<<<(in->P + TPB - 1) / TPB, TPB, 0, st>>>(in->N, in->P, in->h, vel, in->lo, in->hi, in->off, in->ap, src,
                                                   nullptr, nullptr, nullptr, dL_df, in->KW, in->dY);
    k_lsf_T<<<gN, TPB, 0, st>>>(in->N, in->P, in->lo, in->off, in->ap, in->plo, in->phi, in->dY, in->dS);
    k_shift_T<<<gN, TPB, 0, st>>>(in->N, in->h, vel, src, in->dS, in->JR ? in->dR : in->dB, in->part);
    if (in->JR)
        k_rotate_T<<<gN, TPB, ldsr, st>>>(in->N, in->JR, in->h, in->eps, vel, in->BF, in->RBF, in->ZR, in->dR, in->dB,
                                          in->part + 2 * in->nblk);
    k_broaden_T<<<gN, TPB, lds, st>>>(in->N, in->J, in->h, vel, F, Fc, in->Z, in->dB, dL_dF, dL_dFc,
                                      in->part + in->nblk);
    if (g_vel) k_vel_final<<<1, TPB, 0, st>>>(in->nblk, in->JR ? 1 : 0, in->h, vel, in->part, g_vel);
    INST_HIP(hipGetLastError());
    return PZ_OK;
}

}  // extern "C"
