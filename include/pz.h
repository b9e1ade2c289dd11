/*
 * pz.h -- C ABI of the MI355X (gfx950) LTE spectral-synthesis library.
 *
 * The library computes, for one fixed 1-D model atmosphere and one line list,
 * the emergent flux on a log-uniform wavelength grid (Sec. 2.1 of the paper):
 *
 *   grid        lambda_i = lambda_first (1 + 1/R)^i, i = 0..N-1        (Eq. 1)
 *   populations two-stage Saha ionisation, no ionisation lowering      (Sec. 3, Eq. 11)
 *   line params Doppler width dv^2 = 2kT/m + xi^2, damping ratio
 *               a = Gamma / (4 pi dnu_D), Gamma = g_rad + g_S n_e + g_vdW n_pert (Eq. 5)
 *   opacity     kappa_line(i, j) = sum over lines with |lambda_i - lambda_l| <= W of
 *               (pi e^2 / m_e c) n/(rho U) gf e^{-E/kT} (1 - e^{-h nu_l/kT})
 *               H(a, v) / (sqrt(pi) dnu_D)                              (Eqs. 3-4)
 *   continuum   kappa_c = kappa0 (lambda / lambda_ref)^alpha, sigma_c = 0
 *   transfer    d tau = chi dm (trapezoid, tau_0 = chi_0 m_0), S = B_lambda(T),
 *               piecewise-linear S, diffusion lower boundary           (Eqs. 6-7)
 *   flux        F = 2 pi int_0^1 I(0, mu) mu dmu, 3-point Gauss-Legendre in mu,
 *               per nm, for the total and the continuum-only branch   (Eq. 8)
 *
 * plus the vector-Jacobian product for the four corrections of Eq. 30
 * (Sec. 6): per-line log gf, per-line damping scale, per-species abundance
 * (at fixed atmosphere) and microturbulence; and a batched launch over many
 * stars.
 *
 * Conventions
 *   - Units: wavelengths in nm (vacuum), energies in eV, masses in amu,
 *     densities in cm^-3, column mass in g cm^-2, rho in g cm^-3, damping
 *     constants as log10 (s^-1 for radiative, cm^3 s^-1 for Stark and van
 *     der Waals), microturbulence in km/s, flux in erg s^-1 cm^-2 nm^-1.
 *   - Memory: "host" pointers are read during the call only; "device"
 *     pointers are caller-owned device allocations that must stay valid until
 *     the work enqueued on the stream has finished.  The library never frees
 *     or reallocates caller memory.  A plan owns its own device buffers.
 *   - Streams: every synth_* call only enqueues work on the given stream and
 *     returns; no implicit device synchronisation (pz_plan_create is the one
 *     call that synchronises).
 *   - Errors: functions return PZ_OK (0) or a negative PZ_E_* code; a
 *     thread-local message is available from pz_last_error().  All argument
 *     validation happens before any device work is enqueued.
 *   - Determinism: no floating-point atomics; results are bitwise
 *     reproducible run to run, and synth_batch equals the per-star calls.
 *   - Limits: 2 <= D <= PZ_MAX_DEPTH depths, 1 <= S species, 0 <= L lines, L D < 2^31,
 *     and under 2^28 / D lines overlapping any one pixel tile (PZ_E_SHAPE).
 */
#ifndef PZ_H
#define PZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PZ_VERSION 6
#define PZ_MAX_DEPTH 80

#define PZ_OK 0
#define PZ_E_INVALID_ARG -1   /* null pointer, bad enum, non-positive size      */
#define PZ_E_SHAPE -2         /* sizes do not match the plan or a limit         */
#define PZ_E_NOMEM -3         /* device or host allocation failed               */
#define PZ_E_HIP -4           /* a HIP runtime call failed                      */
#define PZ_E_NONFINITE -5     /* NaN/Inf in an input that must be finite        */
#define PZ_E_UNSUPPORTED -6   /* a valid request this build does not implement  */

#define PZ_QUAD_GAUSS3 0      /* 3-point Gauss-Legendre in mu on [0, 1] (Eq. 8) */
#define PZ_QUAD_E2 1          /* F = 2 pi int S E2 dtau (exponential integral)  */
#define PZ_FLAG_DAMPING_FAMILIES 1  /* pz_options.flags: synth_backward writes g_damp as [3][L]
                                       (radiative, Stark, van der Waals: dL/d ddamp_family) */
#define PZ_FLAG_SCATTERING 2        /* pz_options.flags: allocate the workspace of the transfer with
                                       continuum scattering (atmospheres with sigma_c != NULL) */

#define PZ_MODE_FWD 1
#define PZ_MODE_FWD_BWD 2

typedef struct pz_plan pz_plan;     /* opaque */
typedef struct pz_batch pz_batch;   /* opaque */
typedef void* pz_stream;            /* a hipStream_t; NULL = the null stream */

/* Log-uniform synthesis grid (Eq. 1): lambda_i = lambda_first (1 + 1/R)^i. */
typedef struct {
    double lam_first_nm;   /* > 0 */
    double R;              /* R_grid > 0 (model sampling, not resolving power) */
    int32_t N;             /* number of samples, >= 2 */
} pz_grid;

/* Line list (Table 1 "Atomic line" and "Broadening" symbols), host arrays of
 * length L in the caller's order.  Copied into the plan. */
typedef struct {
    int32_t L;
    const double* lam0_nm;      /* line centre, vacuum nm                   */
    const double* loggf;        /* log10 gf                                  */
    const double* E_eV;         /* lower-level excitation energy             */
    const int32_t* species;     /* 0 <= species < S                          */
    const int32_t* ion;         /* 0 = neutral, 1 = singly ionised            */
    const double* log_grad;     /* log10 gamma_rad [s^-1]                     */
    const double* log_gstark;   /* log10 gamma_S per electron [cm^3 s^-1]     */
    const double* log_gvdw;     /* log10 gamma_vdW per perturber [cm^3 s^-1]  */
} pz_lines;

/* Plan options. Zero fields take defaults. */
typedef struct {
    double window_nm;           /* W: line l reaches pixel i iff |lambda_i - lambda_l| <= W (> 0) */
    int32_t quadrature;         /* PZ_QUAD_GAUSS3 (default, FP32) or PZ_QUAD_E2 (FP64) */
    int32_t tile_px;            /* opacity tile width in pixels: 0 = autotuned/default */
    int32_t lines_per_chunk;    /* lines staged in LDS per step: 0 = default          */
    int32_t flags;              /* PZ_FLAG_* bits; others must be 0                    */
    double center_eta;          /* continuum-referenced centre test (Sec. 2.2, Table 2): 0 = off
                                   (plain windowed sum); eta > 0 keeps a (line, depth) pair only
                                   if K H(a,0) >= eta kappa_c(lambda_l), and a kept pair deposits
                                   only where |v| <= max(sqrt(ln(R/eta)), sqrt(a R/(sqrt(pi) eta))),
                                   R = K / kappa_c(lambda_l); both decided in float64.  Gradients
                                   treat the mask as constant (it is piecewise constant).  Must be
                                   finite and >= 0. */
    int32_t scatter_max_iter;   /* scattering: iteration cap of the source-function (and adjoint)
                                   iteration per pixel; 0 = 500 */
    double scatter_tol;         /* scattering: stop when max_j |dS_j / S_j| <= tol; 0 = 1e-10 */
} pz_options;

/* One fixed 1-D atmosphere (device arrays, float64, caller-owned).  Depth
 * index j = 0 is the surface; column mass m is strictly increasing inward. */
typedef struct {
    int32_t D;                  /* depths, equals the plan's D                 */
    int32_t S;                  /* species, equals the plan's S                */
    const double* T;            /* [D] K                                       */
    const double* m;            /* [D] g cm^-2                                 */
    const double* ne;           /* [D] electron density                        */
    const double* npert;        /* [D] neutral perturber density (n_H)         */
    const double* rho;          /* [D] mass density                            */
    const double* n_species;    /* [S*D] total number density of each species  */
    const double* chi_ion_eV;   /* [S] ionisation energy I -> II; +inf = one stage */
    const double* U;            /* [S*2*D] partition functions U_{s,r,j}, r = 0, 1 */
    const double* mass_amu;     /* [S] absorber mass                           */
    double kappa0;              /* continuum: kappa0 (lambda/lambda_ref)^alpha, cm^2 g^-1 */
    double lam_ref_nm;
    double alpha;
    const double* sigma_c;      /* [D] or NULL: continuum scattering per unit mass at lambda_ref,
                                   sigma_c(lambda) = sigma_c (lambda/lambda_ref)^sigma_alpha (Eq. 3).
                                   Non-NULL: S = eps B + (1 - eps) J (Eq. 6), iterated per pixel to
                                   its fixed point in float64 (Gauss-3 only; the plan needs
                                   PZ_FLAG_SCATTERING); NULL: S = B */
    double sigma_alpha;
} pz_atmos;

/* Corrections of Eq. 30 (device float32 arrays; NULL means all zero).
 * gf' = gf 10^dgf, n_s' = n_s 10^dA, and the damping width
 * Gamma' = 10^ddamp (g_rad 10^d_rad + g_S n_e 10^d_S + g_vdW n_pert 10^d_vdW):
 * Eq. 30 corrects the three families separately (ddamp_family), ddamp
 * scales their sum.  xi_kms is a device pointer to one float
 * (microturbulence, km/s) and is required. */
typedef struct {
    const float* dgf;           /* [L] caller line order, dex */
    const float* ddamp;         /* [L] caller line order, dex */
    const float* dA;            /* [S] dex                    */
    const float* xi_kms;        /* [1]                        */
    const float* ddamp_family;  /* [3][L] caller line order, dex: radiative, Stark, van der Waals */
} pz_params;

/* Library version (PZ_VERSION). */
int pz_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char* pz_last_error(void);

/* Build a plan (Sec. 2.1 Eqs. 1-2: the log-uniform grid and its sample
 * count; Sec. 2.2: the window bounds prepared once per source window and kept
 * resident, the bounded wing spans): validates the grid and the line list,
 * sorts the lines by wavelength, computes each line's integer window
 * [i_lo, i_hi] in float64 from |lambda_i - lambda_l| <= W, bins lines into
 * wavelength tiles and uploads everything to the current device.  Lines whose
 * window misses the grid are kept (zero contribution, zero gradient).
 * Synchronises the device.  n_species = S and n_depth = D fix the atmosphere
 * shape the plan accepts.  Host arrays are read during the call only; the
 * plan owns its device memory until pz_plan_destroy.  Errors: PZ_E_INVALID_ARG
 * (null pointer, bad option, species or ion out of range), PZ_E_NONFINITE (a
 * non-finite line value), PZ_E_SHAPE (sizes beyond the limits above),
 * PZ_E_NOMEM, PZ_E_HIP. */
int pz_plan_create(const pz_grid* grid, const pz_lines* lines, int32_t n_species,
                   int32_t n_depth, const pz_options* opts, pz_plan** out);

/* Forget the workspace of the last forward pass, so the next synth_backward
 * recomputes the opacity. */
int pz_plan_invalidate(pz_plan* plan);

/* Release a plan (NULL is a no-op).  Synchronises the device. */
void pz_plan_destroy(pz_plan* plan);

/* Query plan sizes: N, L, S, D, tile_px and the number of Voigt evaluations
 * one forward pass performs (sum over lines of D * window pixels). */
int pz_plan_info(const pz_plan* plan, int32_t* N, int32_t* L, int32_t* S, int32_t* D,
                 int32_t* tile_px, int64_t* voigt_evals);

/* Forward synthesis (Secs. 2.1-2.2): writes F[N] and Fc[N] (device float32,
 * per nm) for the total and the continuum-only branch.  Leaves the line
 * opacity kappa_line[D][N] and the per-(line, depth) parameters in the plan's
 * workspace for a following synth_backward with the same inputs. */
int synth_forward(const pz_plan* plan, const pz_atmos* atm, const pz_params* par,
                  float* F, float* Fc, pz_stream stream);

/* Vector-Jacobian product (Sec. 6, Eq. 30): given dL/dF[N] (device), writes
 * dL/d dgf[L] and dL/d ddamp[L] (caller line order), dL/d dA[S] and
 * dL/d xi[1] (per km/s), all device float32.  dL_dFc may be NULL: the
 * continuum branch depends on none of the corrections, so it is ignored.
 * The line opacity of the most recent synth_forward on this plan is reused
 * when that call had the same atmosphere and correction descriptors (same
 * pointers) and the same stream, and no other call has written the plan's
 * workspace since; otherwise the forward opacity is recomputed first.  The
 * caller must not change the contents of those arrays in between, or must
 * call pz_plan_invalidate.  Any gradient pointer may be NULL to skip it. */
int synth_backward(const pz_plan* plan, const pz_atmos* atm, const pz_params* par,
                   const float* dL_dF, const float* dL_dFc,
                   float* g_loggf, float* g_damp, float* g_abund, float* g_xi,
                   pz_stream stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward synthesis as synth_forward, same kernels and bitwise the same F and
 * Fc, with its per-call workspace (populations, line factors, the
 * per-(line, depth) parameters, the line opacity kappa_line[D][Npad], the
 * opacity work-queue counter and the centre-test masks) in one static device
 * array of PZ_NOALLOC_SCRATCH_BYTES per GPU, which the library holds until the
 * process ends.  No allocation, no memset, no host synchronisation.
 *   - The plan must have been created on the current device.
 *   - Fails with PZ_E_SHAPE, before any launch, when the plan's workspace
 *     (about L D 16 + D Npad 4 bytes, plus L D 4 with the centre test) exceeds
 *     PZ_NOALLOC_SCRATCH_BYTES; PZ_E_UNSUPPORTED for an atmosphere with
 *     continuum scattering.
 *   - All calls on one GPU share that GPU's array, whatever the plan: calls
 *     that overlap in time on one GPU (other streams or threads) race and give
 *     wrong results.  Calls queued on one stream are ordered and safe.
 *   - It leaves the plan's own workspace untouched, so a following
 *     synth_backward does not reuse this call's opacity. */
#define PZ_NOALLOC_SCRATCH_BYTES (64ull << 20)
int synth_forward_noalloc(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, float* F, float* Fc,
                          pz_stream stream);

/* Largest number of iterations any pixel used in the last scattering forward
 * (total branch, continuum branch) and adjoint solve on this plan: iters[3]
 * (host).  Synchronises the device.  PZ_E_INVALID_ARG without the
 * scattering workspace. */
int pz_scatter_iterations(const pz_plan* plan, int32_t* iters);

/* Atmosphere-dependent line-selection keep test (Sec. 3, Eqs. 17-19): for
 * the plan's catalogue and one atmosphere, decides which lines can reach
 * eta_sel times the continuum at their centre in some layer.  In float64,
 * per line l of species s, ion r and frequency bin b:
 *   bins    width bin_ln in ln lambda from the first grid wavelength; b =
 *           floor(ln(lambda_l / lambda_first) / bin_ln) clamped to the bins
 *           covering the grid; nu_b at the bin's centre in ln lambda
 *   C_jb    = eta_sel kappa_c(nu_b) / (1 - exp(-h nu_b / k T_j))  (sigma_c = 0)
 *   Q_srb   = max_j (n_{s,r} / U_{s,r})_j / (rho_j (dv_{s,j} / c) C_jb)
 *   R_l     = C_0 gf_l Q_srb / nu_b,  C_0 = sqrt(pi) e^2 / (m_e c)
 *   keep    iff R_l >= 1 and R_l exp(-E_l / k T_deepest) >= 1
 * Populations, Doppler widths and gf include the corrections in par (dA,
 * xi, dgf), as in synth_forward.  Outputs (device, caller line order, any may
 * be NULL but not all): keep [L] (1 = keep), R [L] and R_deep [L] = R_l
 * exp(-E_l/kT_deepest) (float64), n_keep [1] (int32, the number kept).
 * Rewrites the plan's population workspace (a following synth_backward
 * recomputes the forward).  Enqueue-only.  Errors: PZ_E_INVALID_ARG (eta_sel
 * or bin_ln not finite and > 0, more than 2^30 bins, no output). */
int pz_select_lines(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, double eta_sel, double bin_ln,
                    uint8_t* keep, double* R, double* R_deep, int32_t* n_keep, pz_stream stream);

/* Loss seed of a chi^2 fit to a normalised spectrum: with f = F / Fc (Eq. 9,
 * identity instrument operator) and L = sum_i ((f_i - y_i) / sigma)^2 (the
 * chi^2 objective of Sec. 5), writes dL/dF[N], dL/dFc[N] and L[1] (device
 * float32; dL_dFc and loss may be NULL).  The sum runs in a fixed order. */
int pz_chi2_seed(int32_t N, const float* F, const float* Fc, const float* y, float sigma,
                 float* dL_dF, float* dL_dFc, float* loss, pz_stream stream);

/* Debug/test entry: line opacity only.  Writes kappa_line as [D][N] float32
 * (device) for the given atmosphere and corrections. */
int pz_line_opacity(const pz_plan* plan, const pz_atmos* atm, const pz_params* par,
                    float* kappa_line, pz_stream stream);

/* Debug/test entry: the reverse depth scan alone.  Writes dL/dkappa_line as
 * [D][N] float32 (device) for the seed dL/dF[N] (device), the quantity the
 * line-parallel gather of synth_backward consumes.  Reuses or recomputes the
 * forward opacity as synth_backward does. */
int pz_debug_opacity_adjoint(const pz_plan* plan, const pz_atmos* atm, const pz_params* par,
                             const float* dL_dF, float* g_kappa, pz_stream stream);

/* Debug/test entry: formal solution for a caller-given source function and
 * optical depth (Eqs. 7-8), both [D][n] float32 device arrays; writes F[n].
 * quadrature is PZ_QUAD_GAUSS3 or PZ_QUAD_E2 (anything else: PZ_E_INVALID).
 * Lets closed forms (linear S, Milne-Eddington) pin the transfer kernel. */
int pz_debug_formal_solve(int32_t D, int32_t n, const float* S, const float* tau,
                          int32_t quadrature, float* F, pz_stream stream);

/* Stage profiling.  While enabled, every kernel launch of this plan is
 * bracketed by hipEvents recorded on the launch stream (no host
 * synchronisation is added); pz_plan_profile_read synchronises on the recorded
 * events and returns, per stage, the summed duration in ms and the launch
 * count since profiling was enabled.  At most PZ_PROFILE_SLOTS launches per
 * stage are recorded; later ones are not timed (counted in *count only up to
 * the limit).  Stages: PZ_STAGE_*. */
#define PZ_STAGE_POPULATIONS 0
#define PZ_STAGE_LINE_PARAMS 1
#define PZ_STAGE_OPACITY 2
#define PZ_STAGE_FLUX 3
#define PZ_STAGE_REVERSE_SCAN 4
#define PZ_STAGE_GATHER 5
#define PZ_STAGE_REDUCE 6
#define PZ_N_STAGES 7
#define PZ_PROFILE_SLOTS 512
int pz_plan_profile(pz_plan* plan, int32_t enable);
int pz_plan_profile_read(pz_plan* plan, double* total_ms /*[PZ_N_STAGES]*/, int32_t* count /*[PZ_N_STAGES]*/);

/* One star of a batch (all pointers as in synth_forward/synth_backward). */
typedef struct {
    const pz_plan* plan;
    pz_atmos atm;
    pz_params par;
    float* F;                    /* [N]  */
    float* Fc;                   /* [N]  */
    const float* dL_dF;          /* [N], FWD_BWD seed when y is NULL */
    const float* y;              /* [N] or NULL: chi^2 target (pz_chi2_seed); the seed
                                    is then computed from this star's F and Fc */
    float sigma;                 /* chi^2 noise level (used with y) */
    float* loss;                 /* [1] or NULL: chi^2 value (used with y) */
    float* g_loggf;              /* [L], FWD_BWD only (may be NULL) */
    float* g_damp;               /* [L]  */
    float* g_abund;              /* [S]  */
    float* g_xi;                 /* [1]  */
} pz_star;

/* Prepare a batch of stars with different atmospheres, windows and line
 * counts (the stars are independent syntheses, Sec. 9): uploads a device
 * table of the stars' descriptors and builds the work lists (opacity tiles of
 * all stars ordered by decreasing cost).  Preparing these once is what lets
 * synth_batch be a pure enqueue that can be captured and replayed.  The
 * per-star plans and every buffer a star names must outlive the batch, and no
 * two stars may share a plan (each plan's workspace holds that star's
 * intermediate arrays).  A star whose atmosphere has continuum scattering
 * needs a plan built with PZ_FLAG_SCATTERING, as for synth_forward.
 * Synchronises the device.  Errors: PZ_E_INVALID_ARG (null arguments, shared
 * plans), the per-star checks of synth_forward, PZ_E_NOMEM, PZ_E_HIP. */
int pz_batch_create(int32_t n_star, const pz_star* stars, pz_batch** out);
void pz_batch_destroy(pz_batch* batch);

/* Batched synthesis of independent stars (Sec. 9; each star's forward and
 * backward as synth_forward and synth_backward define them, Secs. 2.1, 6)
 * (PZ_MODE_FWD or PZ_MODE_FWD_BWD): every stage runs as one
 * persistent launch whose workgroups take (star, item) work from a queue
 * spanning all stars; the transfer and reverse transfer of stars with
 * continuum scattering (Eq. 6) run in launches of their own after the
 * others'.  Enqueue-only: no host synchronisation, allocation or
 * memset, so the call may be captured in a hipGraph and replayed.  Results
 * are bitwise equal to per-star synth_forward / pz_chi2_seed /
 * synth_backward calls with the same plans. */
int synth_batch(const pz_batch* batch, int32_t mode, pz_stream stream);

/* Autotuner: times synth_forward for every supported (tile_px,
 * lines_per_chunk) pair on the given inputs and returns the fastest in
 * *best (other fields copied from *base).  Builds temporary plans and
 * synchronises the device; reps timed forward passes per candidate. */
int pz_autotune(const pz_grid* grid, const pz_lines* lines, int32_t n_species, int32_t n_depth,
                const pz_options* base, const pz_atmos* atm, const pz_params* par, int32_t reps,
                pz_options* best, float* best_ms);

/* ---------------------------------------------------------------- instrument
 * The instrument operator of Eq. 31 (Eq. 9): both native fluxes pass through
 * a Gaussian broadening B(v_b) on the logarithmic synthesis grid, optionally
 * a rotational broadening R(v sin i) (Sec. 7 mentions a GPU-resident
 * rotational kernel and leaves it undefined), a Doppler shift S(v_r) and a
 * Gaussian line-spread function sampled at observed pixels K before their
 * ratio, f_p = {K S R B F}_p / {K S R B F_c}_p.
 * Discretisation (x = ln lambda, native pixel spacing h = ln(1 + 1/R)):
 *   B: normalised Gaussian of sigma = v_b / (c h) pixels over a fixed support
 *      of +-J pixels, J = ceil(4 vb_max / (c h)), renormalised at the grid
 *      ends (v_b below 1e-3 c h acts as the identity, with zero gradient);
 *   R: (only when vrot_max_kms > 0) weights r_k = the integral over the pixel
 *      cell [k - 1/2, k + 1/2] of the classical rotation profile of a disc
 *      with linear limb darkening I(mu) = 1 - eps + eps mu, of half-width
 *      s = v sin i / (c h) pixels, over a fixed support of +-JR pixels,
 *      JR = ceil(vrot_max / (c h) + 1/2), renormalised at the grid ends;
 *      v sin i <= 0 is the identity; a v sin i above vrot_max is cut to the
 *      support and renormalised (it is read on the device, so not checked);
 *   S: value at fractional pixel i - ln(1 + v_r/c)/h by linear interpolation,
 *      the index clamped to the grid;
 *   K: normalised Gaussian of the pixel's LSF width in ln lambda over
 *      |x_i - x_p| <= lsf_trunc widths, sampled at the pixel centre. */
typedef struct pz_inst pz_inst;     /* opaque */

typedef struct {
    int32_t P;                  /* observed pixels, >= 1                                    */
    const double* lam_obs_nm;   /* [P] host: pixel centres (vacuum nm), strictly increasing */
    const double* lsf_sigma_ln; /* [P] host: Gaussian LSF width in ln lambda (> 0)           */
    double lsf_trunc;           /* LSF support half-width in widths; 0 = 4                   */
    double vb_max_kms;          /* > 0: the largest broadening used; sets B's support        */
    double vrot_max_kms;        /* >= 0: the largest v sin i used; 0 = no rotation stage     */
    double limb_eps;            /* linear limb-darkening coefficient in [0, 1] (rotation)    */
} pz_inst_desc;

/* Build an instrument for the synthesis grid: LSF supports (each must lie
 * inside the grid, and may not shrink from one pixel to the next), their
 * transposed index ranges, and one device workspace owned by the instrument.
 * Synchronises.  Errors: PZ_E_INVALID_ARG, PZ_E_SHAPE, PZ_E_NOMEM, PZ_E_HIP. */
int pz_inst_create(const pz_grid* grid, const pz_inst_desc* desc, pz_inst** out);

/* Release an instrument (NULL is a no-op).  Synchronises the device. */
void pz_inst_destroy(pz_inst* inst);

/* f = K S R B F / K S R B Fc.  F, Fc: [N] device float32 native fluxes; vel:
 * device float32 velocities in km/s, [2] (v_r, v_b), or [3] (v_r, v_b,
 * v sin i) for an instrument with a rotation stage; outputs [P] device
 * float32, any of KF (K S R B F), KFc, f may be NULL but not all.
 * Enqueue-only. */
int pz_inst_forward(const pz_inst* inst, const float* F, const float* Fc, const float* vel, float* KF, float* KFc,
                    float* f, pz_stream stream);

/* Vector-Jacobian product of the map above for the seed dL_df [P]: writes
 * dL_dF, dL_dFc [N] and g_vel = (dL/dv_r, dL/dv_b), and dL/d(v sin i) as a
 * third entry with a rotation stage (device float32; any may be NULL but
 * not all).  The velocity sums run in a fixed order.  Uses
 * the instrument's workspace: calls on one instrument must not overlap.
 * Enqueue-only; no allocation, so it may be captured in a hipGraph. */
int pz_inst_backward(const pz_inst* inst, const float* F, const float* Fc, const float* vel, const float* dL_df,
                     float* dL_dF, float* dL_dFc, float* g_vel, pz_stream stream);

/* ------------------------------------------------------- line calibration
 * Sec. 6 fits four logarithmic corrections per group of catalogue lines
 * (Eq. 30: log gf and the radiative, Stark and van der Waals damping
 * constants) to standard spectra; all lines of a group share its four values.
 * The calls below build the groups, expand group values to lines, gather
 * per-line gradients back into groups, and seed the weighted mean-square
 * objective on the observed pixels of one standard. */

/* Greedy correction groups (host arrays, host code, no device use).  Anchor
 * complexes come first: lines with anchor[l] >= 0 form one group per distinct
 * id (ascending id).  Then the remaining calibrated lines are visited by
 * decreasing loggf (ties: lower index first); each line not yet grouped seeds
 * a new group holding itself and every ungrouped calibrated line of the same
 * species and ion with |E - E_seed| <= dE_eV and |lambda0 - lambda0_seed| <=
 * dlam_nm (float64, both inclusive; measured from the seed, not chained).
 *   L                  lines (>= 0)
 *   lam0_nm, E_eV,     [L] line wavelength (nm), lower level energy (eV),
 *   species, ion,      species index, ionisation stage, log gf
 *   loggf
 *   active             [L] or NULL (all): nonzero marks a calibrated line;
 *                      other lines get group -1
 *   anchor             [L] or NULL: anchor complex id, or -1
 *   dE_eV, dlam_nm     tolerances (finite, >= 0); 2.0 cm^-1 = 2.4797e-4 eV
 *   group_of_line      [L] out: group index, or -1
 *   n_groups           out: number of groups G
 * Errors: PZ_E_INVALID_ARG, PZ_E_SHAPE, PZ_E_NONFINITE (non-finite values of
 * a calibrated line). */
int pz_correction_groups(int32_t L, const double* lam0_nm, const double* E_eV, const int32_t* species,
                         const int32_t* ion, const double* loggf, const uint8_t* active, const int32_t* anchor,
                         double dE_eV, double dlam_nm, int32_t* group_of_line, int32_t* n_groups);

typedef struct pz_groups pz_groups; /* opaque: a group map on the device */

/* Upload a group map: group_of_line [L] (host) with entries in [-1, G)
 * (-1: the line has no group).  Members of each group are kept in ascending
 * line order.  Synchronises.  Errors: PZ_E_SHAPE (L or G < 1),
 * PZ_E_INVALID_ARG (an entry out of range), PZ_E_NOMEM, PZ_E_HIP. */
int pz_groups_create(int32_t L, int32_t G, const int32_t* group_of_line, pz_groups** out);

/* Release a group map (NULL is a no-op).  Synchronises the device. */
void pz_groups_destroy(pz_groups* groups);

/* Sizes of a group map. */
int pz_groups_info(const pz_groups* groups, int32_t* L, int32_t* G);

/* x_line[r][l] = x_group[r][group_of_line[l]], or 0 for a line without a
 * group, for rows r < R (1 <= R <= 64).  Device float32: x_group [R][G],
 * x_line [R][L].  With R = 4 and rows (log gf, radiative, Stark, van der
 * Waals) this yields pz_params.dgf (row 0) and pz_params.ddamp_family (rows
 * 1-3).  Enqueue-only. */
int pz_groups_expand(const pz_groups* groups, int32_t R, const float* x_group, float* x_line, pz_stream stream);

/* The transpose: x_group[r][g] = (accumulate ? x_group[r][g] : 0) + a, where
 * a is the sum of x_line[r][l] over the lines of group g, added one by one in
 * ascending line order from 0 (bitwise reproducible).  Device float32, shapes
 * as above.  With synth_backward under PZ_FLAG_DAMPING_FAMILIES writing g_loggf
 * and g_damp into rows 0 and 1-3 of one [4][L] array, this gives the gradient
 * of the group corrections.  Enqueue-only. */
int pz_groups_reduce(const pz_groups* groups, int32_t R, const float* x_line, float* x_group, int32_t accumulate,
                     pz_stream stream);

/* Weighted mean-square objective of one standard on its observed pixels
 * (Sec. 6: telluric weights w), L = c sum_p w_p (f_p - y_p)^2.  f, y: [P]
 * device float32; w: [P] or NULL (all 1); c: the standard's weight (finite).
 * Writes dL_df [P] = 2 c w (f - y) (may be NULL) and loss [1] (may be NULL,
 * not both): loss = c * (fixed-order float32 sum), or added to loss[0] when
 * accumulate is nonzero.  Enqueue-only. */
int pz_wmse_seed(int32_t P, const float* f, const float* y, const float* w, double c, float* dL_df, float* loss,
                 int32_t accumulate, pz_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* PZ_H */
