// Internal structures shared by the library's host code and kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pz.h"

namespace pz {

// CODATA 2018, CGS
static constexpr double C_LIGHT = 2.99792458e10;
static constexpr double H_PLANCK = 6.62607015e-27;
static constexpr double K_BOLTZ = 1.380649e-16;
static constexpr double E_CHARGE = 4.803204712570263e-10;
static constexpr double M_ELECTRON = 9.1093837015e-28;
static constexpr double AMU_G = 1.66053906660e-24;
static constexpr double EV_ERG = 1.602176634e-12;
static constexpr double PI = 3.14159265358979323846;
static constexpr double LN10 = 2.30258509299404568402;

static constexpr int MAXD = PZ_MAX_DEPTH;
static constexpr int NPAD = 256;          // row padding of [D][Npad] workspaces

// Per-line data of a plan, in wavelength-sorted order (device SoA).
struct LineArrays {
    double* lam_cm;      // line centre, cm
    double* loggf;
    double* E_eV;
    double* lgr;         // log10 gamma_rad
    double* lgs;         // log10 gamma_S
    double* lgw;         // log10 gamma_vdW
    int* spion;          // species * 2 + ion
    int* ic;             // anchor pixel: nearest grid index to the line centre
    float* delta;        // ln(lambda_l / lambda_ic), |delta| <= h/2
    int* ilo;            // window [ilo, ihi] (empty: ilo > ihi)
    int* ihi;
    int* perm;           // sorted index -> caller index
};

// Everything a kernel needs about one star (plan + atmosphere + corrections +
// outputs + workspaces).  Passed by value or stored in the batch table.
struct StarDev {
    // grid
    int N, Npad, L, S, D, tile_px, n_tiles, chunk, quad;
    double lam_first_nm, h;      // h = ln(1 + 1/R)
    float h_hi, h_lo;            // h split for float32 offsets
    LineArrays ln;
    const int* tile_first;       // [n_tiles]
    const int* tile_last;        // [n_tiles]
    const int* sp_off;           // [S+1] species CSR over sorted lines
    const int* sp_idx;           // [L]
    // atmosphere (caller device memory, float64)
    const double* T;
    const double* m;
    const double* ne;
    const double* npert;
    const double* rho;
    const double* n_species;
    const double* chi_ion;
    const double* U;
    const double* mass;
    double kappa0, lam_ref_nm, alpha;
    const double* sigma_c;       // [D] continuum scattering at lambda_ref, or null (S = B)
    double sigma_alpha;
    bool scatter;
    int sc_max_iter;
    double sc_tol;
    double* sc;                  // scattering workspace, [SC_NARR][D][Npad] float64
    int* sc_iters;               // [3][Npad] iterations used (forward total, continuum, adjoint)
    // corrections (caller device memory; may be null except xi)
    const float* dgf;
    const float* ddamp;
    const float* ddamp_family;   // [3][L] caller order, or null
    const float* dA;
    const float* xi;
    // outputs
    float* F;
    float* Fc;
    const float* dLdF;
    float* g_loggf;
    float* g_damp;
    float* g_abund;
    float* g_xi;
    // plan workspaces
    double* pop;                 // [S][2][D] n/(rho U) including 10^dA
    double* inv_dv;              // [S][D] 1 / Doppler velocity width dv (s/cm)
    double4* lc;                 // [L] per-line factors of K and a (see dev_line_consts)
    float* zmax;                 // [L][D] centre test: kept pairs deposit where v^2 + a^2 <= zmax (-1: dropped)
    float* xlim;                 // [L] centre test: largest |x| any depth of the line reaches (0: none)
    int* wide_a;                 // [L] 1 if the line's damping ratio spans the near and far wing tiers
    int* wide_any;               // [1] nonzero if any line is flagged (reset by the populations stage)
    double* inv_kcl;             // [L] centre test: 1 / kappa_c at the line centre
    double center_eta;           // centre-test threshold (0: plain windowed sum)
    bool center;
    bool fam;                    // backward writes per-family damping gradients [3][L]
    float4* lp;                  // [L][D] (c/dv, a^2, K, K a)
    float* kappa;                // [D][Npad]
    float* gk;                   // [D][Npad] dL/dkappa_line
    float* gline;                // [5][L] per-line sums (sorted order): gf, damping (or radiative), xi, Stark, vdW
    float* partial;              // [S+1][n_rchunk] reduction partials
    int n_rchunk;
    const int* tile_order;       // opacity work queue (decreasing cost)
    int* qctr;
    int grid_opacity;
};

static constexpr int RCHUNK = 2048;      // lines per reduction partial
static constexpr int SC_WS_ARRAYS = 45;  // [D][Npad] float64 arrays of the scattering workspace
static constexpr int MAX_CHUNK = 16;     // most lines per LDS chunk of the opacity tile

// Kernel launchers (pz_kernels.hip).  Each enqueues on the stream and returns
// the hipError_t of the launch.
int opacity_grid(int tile_px, bool center);   // persistent opacity workgroups for this device
hipError_t launch_populations(const StarDev& s, hipStream_t st);
hipError_t launch_line_params(const StarDev& s, hipStream_t st);
hipError_t launch_select(const StarDev& s, double eta, double bin_ln, int B, unsigned char* keep, double* R,
                         double* Rd, int* n_keep, hipStream_t st);
hipError_t launch_opacity(const StarDev& s, int chunk, hipStream_t st);
hipError_t launch_flux(const StarDev& s, hipStream_t st);
hipError_t launch_reverse_scan(const StarDev& s, hipStream_t st);
hipError_t launch_gather(const StarDev& s, hipStream_t st);
hipError_t launch_reduce(const StarDev& s, hipStream_t st);
hipError_t launch_chi2_seed(int N, const float* F, const float* Fc, const float* y, float sigma, float* gF,
                            float* gFc, float* loss, hipStream_t st);
hipError_t launch_debug_formal(int D, int n, const float* S, const float* tau, int quad, float* F,
                               hipStream_t st);

}  // namespace pz

struct pz_plan {
    int device;
    int N, Npad, L, S, D, tile_px, chunk, quadrature;
    int n_tiles;
    double lam_first_nm, R, h, window_nm;
    int64_t voigt_evals;
    pz::LineArrays ln;
    int* tile_first;
    int* tile_last;
    int* sp_off;
    int* sp_idx;
    double* pop;
    double* inv_dv;
    double4* lc;
    float* zmax;
    float* xlim;
    int* wide_a;
    int* wide_any;
    double* inv_kcl;
    double center_eta;
    bool families;
    float4* lp;
    float* kappa;
    float* gk;
    float* gline;
    float* partial;
    int n_rchunk;
    float* seed;         // [Npad] loss seed written by the batched chi^2 stage
    int* tile_order;     // [n_tiles] tiles by decreasing cost (opacity work queue)
    int* qctr;           // [1] opacity work-queue counter
    int grid_opacity;    // persistent opacity workgroups (CUs x occupancy)
    int64_t* tile_cost;  // host [n_tiles]: Voigt evaluations per opacity tile
    void* base;          // single device allocation holding everything above
    // stage profiling (see pz_plan_profile)
    bool prof;
    int prof_n[PZ_N_STAGES];
    hipEvent_t* prof_ev;  // [PZ_N_STAGES][PZ_PROFILE_SLOTS][2], created on first enable
    // transfer with scattering (PZ_FLAG_SCATTERING)
    bool scatter_ws;
    double* sc;
    int* sc_iters;
    int sc_max_iter;
    double sc_tol;
    bool sc_ok;          // the scattering source functions match the recorded workspace
    // who last wrote kappa / lp (see synth_backward)
    bool ws_valid;
    pz_atmos ws_atm;
    pz_params ws_par;
    hipStream_t ws_stream;
};
