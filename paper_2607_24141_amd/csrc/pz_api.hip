// C ABI of the synthesis library: argument validation, plan construction
// (sort, integer windows, tile binning, species lists) and the entry points
// that enqueue the kernels.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "pz_internal.h"

using namespace pz;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(PZ_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define PZ_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

bool finite_all(const double* x, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// Integer window of one line: all i in [0, N) with |lambda_i - lambda_l| <= W,
// evaluated in float64 exactly as the definition reads, lambda_i =
// lambda_first (1 + 1/R)^i.  The pixel set is an interval; the log-space
// estimate is corrected by direct tests.
struct Window {
    int lo, hi;   // lo in [0, N], hi in [-1, N-1]; empty iff lo > hi
};

Window line_window(double lam_l, double lf, double r1, double h, int N, double W) {
    auto lam = [&](long i) { return lf * std::pow(r1, (double)i); };
    auto in = [&](long i) { return std::fabs(lam(i) - lam_l) <= W; };
    double e = std::log(lam_l / lf) / h;
    e = std::min(std::max(e, -1.0), (double)N);
    long c = std::lround(e);
    c = std::min(std::max(c, 0L), (long)N - 1);
    long seed = -1;
    for (long k = std::max(0L, c - 1); k <= std::min((long)N - 1, c + 1); ++k)
        if (in(k)) {
            seed = k;
            break;
        }
    if (seed < 0) {
        // no pixel within W; keep the bounds monotone in lambda for binning
        if (lam_l < lf) return {0, -1};
        if (lam_l > lam(N - 1)) return {N, N - 1};
        return {(int)c + 1, (int)c};
    }
    long lo, hi;
    double el = (lam_l - W > 0.0) ? std::ceil(std::log((lam_l - W) / lf) / h) : 0.0;
    lo = (long)std::min(std::max(el, 0.0), (double)seed);
    while (lo > 0 && in(lo - 1)) --lo;
    while (!in(lo)) ++lo;
    double eh = std::floor(std::log((lam_l + W) / lf) / h);
    hi = (long)std::min(std::max(eh, (double)seed), (double)(N - 1));
    while (hi < N - 1 && in(hi + 1)) ++hi;
    while (!in(hi)) --hi;
    return {(int)lo, (int)hi};
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int pz_version(void) { return PZ_VERSION; }

const char* pz_last_error(void) { return g_err.c_str(); }

int pz_plan_create(const pz_grid* grid, const pz_lines* lines, int32_t n_species, int32_t n_depth,
                   const pz_options* opts, pz_plan** out) {
    g_err.clear();
    if (!out) return fail(PZ_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !lines || !opts) return fail(PZ_E_INVALID_ARG, "grid, lines and opts are required");
    if (!(grid->lam_first_nm > 0.0) || !std::isfinite(grid->lam_first_nm))
        return fail(PZ_E_INVALID_ARG, "lam_first_nm must be finite and > 0");
    if (!(grid->R > 0.0) || !std::isfinite(grid->R)) return fail(PZ_E_INVALID_ARG, "R must be finite and > 0");
    if (grid->N < 2) return fail(PZ_E_SHAPE, "N must be >= 2 (got %d)", grid->N);
    if (n_species < 1) return fail(PZ_E_SHAPE, "n_species must be >= 1");
    if (n_depth < 2 || n_depth > PZ_MAX_DEPTH)
        return fail(PZ_E_SHAPE, "n_depth must be in [2, %d] (got %d)", PZ_MAX_DEPTH, n_depth);
    if (lines->L < 0) return fail(PZ_E_SHAPE, "L must be >= 0");
    if ((long long)lines->L * n_depth >= (1LL << 31))
        return fail(PZ_E_SHAPE, "L x n_depth must be below 2^31 (got %lld)", (long long)lines->L * n_depth);
    if (!(opts->window_nm > 0.0) || !std::isfinite(opts->window_nm))
        return fail(PZ_E_INVALID_ARG, "window_nm must be finite and > 0");
    if (opts->quadrature != PZ_QUAD_GAUSS3 && opts->quadrature != PZ_QUAD_E2)
        return fail(PZ_E_INVALID_ARG, "unknown quadrature %d", opts->quadrature);
    int tile_px = opts->tile_px ? opts->tile_px : 64;
    if (tile_px != 32 && tile_px != 64 && tile_px != 128)
        return fail(PZ_E_INVALID_ARG, "tile_px must be 0, 32, 64 or 128 (got %d)", opts->tile_px);
    int chunk = opts->lines_per_chunk ? opts->lines_per_chunk : 16;
    if (chunk < 1 || chunk > MAX_CHUNK) return fail(PZ_E_INVALID_ARG, "lines_per_chunk must be in [0, %d]", MAX_CHUNK);
    if (opts->flags & ~(PZ_FLAG_DAMPING_FAMILIES | PZ_FLAG_SCATTERING))
        return fail(PZ_E_INVALID_ARG, "unknown bits in flags");
    if (opts->scatter_max_iter < 0 || opts->scatter_max_iter > 100000)
        return fail(PZ_E_INVALID_ARG, "scatter_max_iter must be in [0, 100000]");
    if (!(opts->scatter_tol >= 0.0) || !std::isfinite(opts->scatter_tol))
        return fail(PZ_E_INVALID_ARG, "scatter_tol must be finite and >= 0");
    if ((opts->flags & PZ_FLAG_SCATTERING) && opts->quadrature != PZ_QUAD_GAUSS3)
        return fail(PZ_E_UNSUPPORTED, "scattering is implemented with the Gauss-3 quadrature only");
    if (!(opts->center_eta >= 0.0) || !std::isfinite(opts->center_eta))
        return fail(PZ_E_INVALID_ARG, "center_eta must be finite and >= 0");
    const int L = lines->L, N = grid->N, S = n_species, D = n_depth;
    if (L > 0) {
        if (!lines->lam0_nm || !lines->loggf || !lines->E_eV || !lines->species || !lines->ion ||
            !lines->log_grad || !lines->log_gstark || !lines->log_gvdw)
            return fail(PZ_E_INVALID_ARG, "a line array is NULL");
        if (!finite_all(lines->lam0_nm, L) || !finite_all(lines->loggf, L) || !finite_all(lines->E_eV, L) ||
            !finite_all(lines->log_grad, L) || !finite_all(lines->log_gstark, L) ||
            !finite_all(lines->log_gvdw, L))
            return fail(PZ_E_NONFINITE, "non-finite value in the line list");
        for (int l = 0; l < L; ++l) {
            if (!(lines->lam0_nm[l] > 0.0)) return fail(PZ_E_INVALID_ARG, "line %d: lam0_nm must be > 0", l);
            if (lines->species[l] < 0 || lines->species[l] >= S)
                return fail(PZ_E_INVALID_ARG, "line %d: species %d outside [0, %d)", l, lines->species[l], S);
            if (lines->ion[l] != 0 && lines->ion[l] != 1)
                return fail(PZ_E_INVALID_ARG, "line %d: ion stage must be 0 or 1", l);
        }
    }

    // ---- host plan
    const double lf = grid->lam_first_nm, R = grid->R;
    const double r1 = 1.0 + 1.0 / R;
    const double h = std::log1p(1.0 / R);
    std::vector<int> order(L);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return lines->lam0_nm[a] < lines->lam0_nm[b]; });
    std::vector<double> lam_cm(L), loggf(L), E(L), lgr(L), lgs(L), lgw(L);
    std::vector<int> spion(L), ic(L), ilo(L), ihi(L), perm(L);
    std::vector<float> delta(L);
    int64_t evals = 0;
    for (int k = 0; k < L; ++k) {
        const int l = order[k];
        const double lam = lines->lam0_nm[l];
        perm[k] = l;
        lam_cm[k] = lam * 1.0e-7;
        loggf[k] = lines->loggf[l];
        E[k] = lines->E_eV[l];
        lgr[k] = lines->log_grad[l];
        lgs[k] = lines->log_gstark[l];
        lgw[k] = lines->log_gvdw[l];
        spion[k] = lines->species[l] * 2 + lines->ion[l];
        const Window w = line_window(lam, lf, r1, h, N, opts->window_nm);
        ilo[k] = w.lo;
        ihi[k] = w.hi;
        if (w.hi >= w.lo) evals += (int64_t)(w.hi - w.lo + 1) * D;
        const double lnr = std::log(lam / lf);
        double e = std::min(std::max(lnr / h, -1.0e9), 1.0e9);
        const long a = std::lround(e);
        ic[k] = (int)a;
        delta[k] = (float)(lnr - (double)a * h);
    }
    // tiles: lines overlapping [t*TP, t*TP+TP-1] form a contiguous range
    const int n_tiles = (N + tile_px - 1) / tile_px;
    std::vector<int> pmax_hi(L), smin_lo(L);
    for (int k = 0; k < L; ++k) pmax_hi[k] = k ? std::max(pmax_hi[k - 1], ihi[k]) : ihi[k];
    for (int k = L - 1; k >= 0; --k) smin_lo[k] = (k < L - 1) ? std::min(smin_lo[k + 1], ilo[k]) : ilo[k];
    std::vector<int> tfirst(n_tiles), tlast(n_tiles);
    for (int t = 0; t < n_tiles; ++t) {
        const int start = t * tile_px, end = std::min(N - 1, start + tile_px - 1);
        const int f = (int)(std::lower_bound(pmax_hi.begin(), pmax_hi.end(), start) - pmax_hi.begin());
        const int g = (int)(std::upper_bound(smin_lo.begin(), smin_lo.end(), end) - smin_lo.begin());
        tfirst[t] = f;
        tlast[t] = std::max(f, g);
        // the opacity kernel addresses a tile's parameter rows with 32-bit byte offsets
        if ((long long)(tlast[t] - tfirst[t]) * D >= (1LL << 28))
            return fail(PZ_E_SHAPE, "%d lines overlap pixel tile %d: lines x n_depth per tile must be below 2^28",
                        tlast[t] - tfirst[t], t);
    }
    // species lists over sorted lines (ascending sorted index)
    std::vector<int> sp_off(S + 1, 0), sp_idx(L);
    for (int k = 0; k < L; ++k) sp_off[(spion[k] >> 1) + 1]++;
    for (int s = 0; s < S; ++s) sp_off[s + 1] += sp_off[s];
    {
        std::vector<int> fill(sp_off.begin(), sp_off.end() - 1);
        for (int k = 0; k < L; ++k) sp_idx[fill[spion[k] >> 1]++] = k;
    }

    // ---- device layout (one allocation)
    const int Npad = ((N + NPAD - 1) / NPAD) * NPAD;
    const size_t Ls = (size_t)std::max(L, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t o_lam = take(Ls * 8), o_gf = take(Ls * 8), o_E = take(Ls * 8), o_lgr = take(Ls * 8),
                 o_lgs = take(Ls * 8), o_lgw = take(Ls * 8), o_spion = take(Ls * 4), o_ic = take(Ls * 4),
                 o_delta = take(Ls * 4), o_ilo = take(Ls * 4), o_ihi = take(Ls * 4), o_perm = take(Ls * 4),
                 o_tf = take((size_t)n_tiles * 4), o_tl = take((size_t)n_tiles * 4),
                 o_spo = take((size_t)(S + 1) * 4), o_spi = take(Ls * 4), o_pop = take((size_t)S * 2 * D * 8),
                 o_idv = take((size_t)S * D * 8), o_lc = take(Ls * 32), o_zmax = take(Ls * D * 4),
                 o_xlim = take(Ls * 4), o_wide = take(Ls * 4), o_ikc = take(Ls * 8),
                 o_lp = take(Ls * D * 16), o_kap = take((size_t)D * Npad * 4), o_gk = take((size_t)D * Npad * 4),
                 o_gl = take(Ls * 5 * 4);
    const int n_rchunk = (int)((Ls + RCHUNK - 1) / RCHUNK);
    const size_t o_part = take((size_t)(S + 1) * n_rchunk * 4);
    const size_t o_seed = take((size_t)Npad * 4);
    const size_t o_order = take((size_t)n_tiles * 4), o_qctr = take(4), o_wany = take(4);
    const bool scatter_ws = (opts->flags & PZ_FLAG_SCATTERING) != 0;
    const size_t o_sc = scatter_ws ? take((size_t)SC_WS_ARRAYS * D * Npad * 8) : 0;
    const size_t o_sci = scatter_ws ? take((size_t)3 * Npad * 4) : 0;
    // Voigt evaluations per tile (orders the batched opacity work)
    std::vector<int64_t> tcost(n_tiles, 0);
    for (int k = 0; k < L; ++k) {
        if (ihi[k] < ilo[k]) continue;
        for (int t = ilo[k] / tile_px; t <= ihi[k] / tile_px; ++t) {
            const int a0 = std::max(ilo[k], t * tile_px), a1 = std::min(ihi[k], t * tile_px + tile_px - 1);
            tcost[t] += (int64_t)(a1 - a0 + 1) * D;
        }
    }
    pz_plan* p = new (std::nothrow) pz_plan();
    if (!p) return fail(PZ_E_NOMEM, "host allocation failed");
    std::memset(p, 0, sizeof *p);
    p->tile_cost = new (std::nothrow) int64_t[n_tiles];
    if (!p->tile_cost) {
        delete p;
        return fail(PZ_E_NOMEM, "host allocation failed");
    }
    std::copy(tcost.begin(), tcost.end(), p->tile_cost);
    PZ_HIP(hipGetDevice(&p->device));
    char* base = nullptr;
    hipError_t e = hipMalloc((void**)&base, off);
    if (e != hipSuccess) {
        delete[] p->tile_cost;
        delete p;
        (void)hipGetLastError();
        return fail(PZ_E_NOMEM, "hipMalloc of %zu bytes failed: %s", off, hipGetErrorString(e));
    }
    p->base = base;
    p->N = N;
    p->Npad = Npad;
    p->L = L;
    p->S = S;
    p->D = D;
    p->tile_px = tile_px;
    p->chunk = chunk;
    p->quadrature = opts->quadrature;
    p->n_tiles = n_tiles;
    p->lam_first_nm = lf;
    p->R = R;
    p->h = h;
    p->window_nm = opts->window_nm;
    p->voigt_evals = evals;
    p->ln.lam_cm = (double*)(base + o_lam);
    p->ln.loggf = (double*)(base + o_gf);
    p->ln.E_eV = (double*)(base + o_E);
    p->ln.lgr = (double*)(base + o_lgr);
    p->ln.lgs = (double*)(base + o_lgs);
    p->ln.lgw = (double*)(base + o_lgw);
    p->ln.spion = (int*)(base + o_spion);
    p->ln.ic = (int*)(base + o_ic);
    p->ln.delta = (float*)(base + o_delta);
    p->ln.ilo = (int*)(base + o_ilo);
    p->ln.ihi = (int*)(base + o_ihi);
    p->ln.perm = (int*)(base + o_perm);
    p->tile_first = (int*)(base + o_tf);
    p->tile_last = (int*)(base + o_tl);
    p->sp_off = (int*)(base + o_spo);
    p->sp_idx = (int*)(base + o_spi);
    p->pop = (double*)(base + o_pop);
    p->inv_dv = (double*)(base + o_idv);
    p->lc = (double4*)(base + o_lc);
    p->zmax = (float*)(base + o_zmax);
    p->xlim = (float*)(base + o_xlim);
    p->wide_a = (int*)(base + o_wide);
    p->wide_any = (int*)(base + o_wany);
    p->inv_kcl = (double*)(base + o_ikc);
    p->center_eta = opts->center_eta;
    p->families = (opts->flags & PZ_FLAG_DAMPING_FAMILIES) != 0;
    p->scatter_ws = scatter_ws;
    p->sc = scatter_ws ? (double*)(base + o_sc) : nullptr;
    p->sc_iters = scatter_ws ? (int*)(base + o_sci) : nullptr;
    p->sc_max_iter = opts->scatter_max_iter ? opts->scatter_max_iter : 500;
    p->sc_tol = opts->scatter_tol > 0.0 ? opts->scatter_tol : 1e-10;
    p->lp = (float4*)(base + o_lp);
    p->kappa = (float*)(base + o_kap);
    p->gk = (float*)(base + o_gk);
    p->gline = (float*)(base + o_gl);
    p->partial = (float*)(base + o_part);
    p->n_rchunk = n_rchunk;
    p->seed = (float*)(base + o_seed);
    p->tile_order = (int*)(base + o_order);
    p->qctr = (int*)(base + o_qctr);
    std::vector<int> torder(n_tiles);
    std::iota(torder.begin(), torder.end(), 0);
    std::stable_sort(torder.begin(), torder.end(), [&](int a, int b) { return tcost[a] > tcost[b]; });
    p->grid_opacity = opacity_grid(tile_px, opts->center_eta > 0.0);
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t ue = hipSuccess;
    if (L > 0) {
        const hipError_t r[] = {
            up(p->ln.lam_cm, lam_cm.data(), (size_t)L * 8), up(p->ln.loggf, loggf.data(), (size_t)L * 8),
            up(p->ln.E_eV, E.data(), (size_t)L * 8),        up(p->ln.lgr, lgr.data(), (size_t)L * 8),
            up(p->ln.lgs, lgs.data(), (size_t)L * 8),       up(p->ln.lgw, lgw.data(), (size_t)L * 8),
            up(p->ln.spion, spion.data(), (size_t)L * 4),   up(p->ln.ic, ic.data(), (size_t)L * 4),
            up(p->ln.delta, delta.data(), (size_t)L * 4),   up(p->ln.ilo, ilo.data(), (size_t)L * 4),
            up(p->ln.ihi, ihi.data(), (size_t)L * 4),       up(p->ln.perm, perm.data(), (size_t)L * 4),
            up(p->sp_idx, sp_idx.data(), (size_t)L * 4)};
        for (hipError_t x : r)
            if (x != hipSuccess) ue = x;
    }
    if (ue == hipSuccess) ue = up(p->tile_first, tfirst.data(), (size_t)n_tiles * 4);
    if (ue == hipSuccess) ue = up(p->tile_last, tlast.data(), (size_t)n_tiles * 4);
    if (ue == hipSuccess) ue = up(p->sp_off, sp_off.data(), (size_t)(S + 1) * 4);
    if (ue == hipSuccess) ue = up(p->tile_order, torder.data(), (size_t)n_tiles * 4);
    // workspaces start defined (pixels beyond N in the padded rows stay zero)
    if (ue == hipSuccess) ue = hipMemset(p->kappa, 0, (size_t)D * Npad * 4);
    if (ue == hipSuccess) ue = hipMemset(p->gk, 0, (size_t)D * Npad * 4);
    if (ue == hipSuccess) ue = hipMemset(p->gline, 0, Ls * 3 * 4);
    if (ue == hipSuccess) ue = hipDeviceSynchronize();
    if (ue == hipSuccess) ue = hipMemset(p->seed, 0, (size_t)Npad * 4);
    if (ue != hipSuccess) {
        (void)hipFree(base);
        delete[] p->tile_cost;
        delete p;
        return hip_fail(ue, "plan upload");
    }
    *out = p;
    return PZ_OK;
}

void pz_plan_destroy(pz_plan* plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    if (plan->prof_ev) {
        for (int k = 0; k < PZ_N_STAGES * PZ_PROFILE_SLOTS * 2; ++k) (void)hipEventDestroy(plan->prof_ev[k]);
        delete[] plan->prof_ev;
    }
    (void)hipFree(plan->base);
    delete[] plan->tile_cost;
    delete plan;
}

int pz_plan_invalidate(pz_plan* plan) {
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    plan->ws_valid = false;
    return PZ_OK;
}

int pz_plan_profile(pz_plan* plan, int32_t enable) {
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    if (enable && !plan->prof_ev) {
        const int n = PZ_N_STAGES * PZ_PROFILE_SLOTS * 2;
        plan->prof_ev = new (std::nothrow) hipEvent_t[n];
        if (!plan->prof_ev) return fail(PZ_E_NOMEM, "host allocation failed");
        for (int k = 0; k < n; ++k) {
            hipError_t e = hipEventCreate(&plan->prof_ev[k]);
            if (e != hipSuccess) {
                for (int q = 0; q < k; ++q) (void)hipEventDestroy(plan->prof_ev[q]);
                delete[] plan->prof_ev;
                plan->prof_ev = nullptr;
                return hip_fail(e, "hipEventCreate");
            }
        }
    }
    plan->prof = enable != 0;
    if (enable)
        for (int k = 0; k < PZ_N_STAGES; ++k) plan->prof_n[k] = 0;
    return PZ_OK;
}

int pz_plan_profile_read(pz_plan* plan, double* total_ms, int32_t* count) {
    if (!plan || !total_ms || !count) return fail(PZ_E_INVALID_ARG, "plan, total_ms and count are required");
    for (int k = 0; k < PZ_N_STAGES; ++k) {
        total_ms[k] = 0.0;
        count[k] = plan->prof_ev ? plan->prof_n[k] : 0;
        for (int q = 0; q < count[k]; ++q) {
            hipEvent_t a = plan->prof_ev[(k * PZ_PROFILE_SLOTS + q) * 2];
            hipEvent_t b = plan->prof_ev[(k * PZ_PROFILE_SLOTS + q) * 2 + 1];
            PZ_HIP(hipEventSynchronize(b));
            float ms = 0.0f;
            PZ_HIP(hipEventElapsedTime(&ms, a, b));
            total_ms[k] += ms;
        }
    }
    return PZ_OK;
}

int pz_plan_info(const pz_plan* plan, int32_t* N, int32_t* L, int32_t* S, int32_t* D, int32_t* tile_px,
                 int64_t* voigt_evals) {
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    if (N) *N = plan->N;
    if (L) *L = plan->L;
    if (S) *S = plan->S;
    if (D) *D = plan->D;
    if (tile_px) *tile_px = plan->tile_px;
    if (voigt_evals) *voigt_evals = plan->voigt_evals;
    return PZ_OK;
}

}  // extern "C"

namespace pz {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int clear_error() {
    g_err.clear();
    return PZ_OK;
}

int check_atmos(const pz_plan* plan, const pz_atmos* atm) {
    if (!atm) return fail(PZ_E_INVALID_ARG, "atmosphere is NULL");
    if (atm->D != plan->D) return fail(PZ_E_SHAPE, "atmosphere has D=%d, plan expects %d", atm->D, plan->D);
    if (atm->S != plan->S) return fail(PZ_E_SHAPE, "atmosphere has S=%d, plan expects %d", atm->S, plan->S);
    if (!atm->T || !atm->m || !atm->ne || !atm->npert || !atm->rho || !atm->n_species || !atm->chi_ion_eV ||
        !atm->U || !atm->mass_amu)
        return fail(PZ_E_INVALID_ARG, "an atmosphere array is NULL");
    if (!std::isfinite(atm->kappa0) || !std::isfinite(atm->lam_ref_nm) || !std::isfinite(atm->alpha) ||
        !(atm->lam_ref_nm > 0.0))
        return fail(PZ_E_NONFINITE, "continuum parameters must be finite (lam_ref_nm > 0)");
    if (atm->sigma_c) {
        if (!plan->scatter_ws)
            return fail(PZ_E_INVALID_ARG, "atmosphere has sigma_c but the plan was built without PZ_FLAG_SCATTERING");
        if (!std::isfinite(atm->sigma_alpha)) return fail(PZ_E_NONFINITE, "sigma_alpha must be finite");
    }
    return PZ_OK;
}

int check_params(const pz_params* par) {
    if (!par) return fail(PZ_E_INVALID_ARG, "params is NULL");
    if (!par->xi_kms) return fail(PZ_E_INVALID_ARG, "params.xi_kms (device pointer) is required");
    return PZ_OK;
}

StarDev make_star(const pz_plan* p, const pz_atmos* atm, const pz_params* par) {
    StarDev s;
    std::memset(&s, 0, sizeof s);
    s.N = p->N;
    s.Npad = p->Npad;
    s.L = p->L;
    s.S = p->S;
    s.D = p->D;
    s.tile_px = p->tile_px;
    s.n_tiles = p->n_tiles;
    s.chunk = p->chunk;
    s.quad = p->quadrature;
    s.lam_first_nm = p->lam_first_nm;
    s.h = p->h;
    s.h_hi = (float)p->h;
    s.h_lo = (float)(p->h - (double)s.h_hi);
    s.ln = p->ln;
    s.tile_first = p->tile_first;
    s.tile_last = p->tile_last;
    s.sp_off = p->sp_off;
    s.sp_idx = p->sp_idx;
    s.T = atm->T;
    s.m = atm->m;
    s.ne = atm->ne;
    s.npert = atm->npert;
    s.rho = atm->rho;
    s.n_species = atm->n_species;
    s.chi_ion = atm->chi_ion_eV;
    s.U = atm->U;
    s.mass = atm->mass_amu;
    s.kappa0 = atm->kappa0;
    s.lam_ref_nm = atm->lam_ref_nm;
    s.alpha = atm->alpha;
    s.sigma_c = atm->sigma_c;
    s.sigma_alpha = atm->sigma_alpha;
    s.scatter = atm->sigma_c != nullptr;
    s.sc_max_iter = p->sc_max_iter;
    s.sc_tol = p->sc_tol;
    s.sc = p->sc;
    s.sc_iters = p->sc_iters;
    s.dgf = par->dgf;
    s.ddamp = par->ddamp;
    s.ddamp_family = par->ddamp_family;
    s.dA = par->dA;
    s.xi = par->xi_kms;
    s.pop = p->pop;
    s.inv_dv = p->inv_dv;
    s.lc = p->lc;
    s.zmax = p->zmax;
    s.xlim = p->xlim;
    s.wide_a = p->wide_a;
    s.wide_any = p->wide_any;
    s.inv_kcl = p->inv_kcl;
    s.center_eta = p->center_eta;
    s.center = p->center_eta > 0.0;
    s.fam = p->families;
    s.lp = p->lp;
    s.kappa = p->kappa;
    s.gk = p->gk;
    s.gline = p->gline;
    s.partial = p->partial;
    s.n_rchunk = p->n_rchunk;
    s.tile_order = p->tile_order;
    s.qctr = p->qctr;
    s.grid_opacity = p->grid_opacity;
    return s;
}

// Bracket one stage launch with profiling events when enabled.
struct StageTimer {
    pz_plan* p;
    int stage, slot;
    hipStream_t st;
    StageTimer(const pz_plan* plan, int stage_, hipStream_t st_)
        : p(const_cast<pz_plan*>(plan)), stage(stage_), slot(-1), st(st_) {
        if (p->prof && p->prof_n[stage] < PZ_PROFILE_SLOTS) {
            slot = p->prof_n[stage]++;
            (void)hipEventRecord(p->prof_ev[(stage * PZ_PROFILE_SLOTS + slot) * 2], st);
        }
    }
    ~StageTimer() {
        if (slot >= 0) (void)hipEventRecord(p->prof_ev[(stage * PZ_PROFILE_SLOTS + slot) * 2 + 1], st);
    }
};

void record_workspace(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, hipStream_t st) {
    pz_plan* p = const_cast<pz_plan*>(plan);
    p->ws_valid = true;
    p->sc_ok = false;                    // set by a forward flux stage that solves the scattering
    p->ws_atm = *atm;
    p->ws_par = *par;
    p->ws_stream = st;
}

bool workspace_matches(const pz_plan* p, const pz_atmos* atm, const pz_params* par, hipStream_t st) {
    return p->ws_valid && p->ws_stream == st && std::memcmp(&p->ws_atm, atm, sizeof *atm) == 0 &&
           std::memcmp(&p->ws_par, par, sizeof *par) == 0;
}

int enqueue_opacity(const pz_plan* p, const StarDev& s, hipStream_t st) {
    {
        StageTimer t(p, PZ_STAGE_POPULATIONS, st);
        PZ_HIP(launch_populations(s, st));
    }
    {
        StageTimer t(p, PZ_STAGE_LINE_PARAMS, st);
        PZ_HIP(launch_line_params(s, st));
    }
    {
        StageTimer t(p, PZ_STAGE_OPACITY, st);
        PZ_HIP(launch_opacity(s, p->chunk, st));
    }
    return PZ_OK;
}

// The scattering backward needs the forward's converged source functions: solve
// them again (no flux output) unless the last forward on this workspace did.
int ensure_scatter_forward(const pz_plan* p, const StarDev& s, hipStream_t st) {
    if (!s.scatter || p->sc_ok) return PZ_OK;
    StarDev f = s;
    f.F = nullptr;
    f.Fc = nullptr;
    PZ_HIP(launch_flux(f, st));
    const_cast<pz_plan*>(p)->sc_ok = true;
    return PZ_OK;
}

}  // namespace pz

extern "C" {

int pz_scatter_iterations(const pz_plan* plan, int32_t* iters) {
    g_err.clear();
    if (!plan || !iters) return fail(PZ_E_INVALID_ARG, "plan and iters are required");
    if (!plan->scatter_ws) return fail(PZ_E_INVALID_ARG, "the plan has no scattering workspace");
    std::vector<int32_t> h((size_t)3 * plan->Npad);
    PZ_HIP(hipDeviceSynchronize());
    PZ_HIP(hipMemcpy(h.data(), plan->sc_iters, h.size() * 4, hipMemcpyDeviceToHost));
    for (int r = 0; r < 3; ++r) {
        int32_t mx = 0;
        for (int i = 0; i < plan->N; ++i) mx = std::max(mx, h[(size_t)r * plan->Npad + i]);
        iters[r] = mx;
    }
    return PZ_OK;
}

int synth_forward(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, float* F, float* Fc,
                  pz_stream stream) {
    g_err.clear();
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    int rc = check_atmos(plan, atm);
    if (rc) return rc;
    if ((rc = check_params(par))) return rc;
    if (!F || !Fc) return fail(PZ_E_INVALID_ARG, "F and Fc are required");
    StarDev s = make_star(plan, atm, par);
    s.F = F;
    s.Fc = Fc;
    hipStream_t st = (hipStream_t)stream;
    const_cast<pz_plan*>(plan)->ws_valid = false;
    if ((rc = enqueue_opacity(plan, s, st))) return rc;
    record_workspace(plan, atm, par, st);
    StageTimer t(plan, PZ_STAGE_FLUX, st);
    PZ_HIP(launch_flux(s, st));
    const_cast<pz_plan*>(plan)->sc_ok = s.scatter;
    return PZ_OK;
}

int pz_select_lines(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, double eta_sel, double bin_ln,
                    uint8_t* keep, double* R, double* R_deep, int32_t* n_keep, pz_stream stream) {
    g_err.clear();
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    int rc = check_atmos(plan, atm);
    if (rc) return rc;
    if ((rc = check_params(par))) return rc;
    if (!(eta_sel > 0.0) || !std::isfinite(eta_sel)) return fail(PZ_E_INVALID_ARG, "eta_sel must be finite and > 0");
    if (!(bin_ln > 0.0) || !std::isfinite(bin_ln)) return fail(PZ_E_INVALID_ARG, "bin_ln must be finite and > 0");
    if (!keep && !R && !R_deep && !n_keep) return fail(PZ_E_INVALID_ARG, "no output requested");
    const double span = plan->h * (plan->N - 1);                        // ln(lambda_last / lambda_first)
    const double Bd = std::floor(span / bin_ln) + 1.0;
    if (Bd > (double)(1 << 30)) return fail(PZ_E_INVALID_ARG, "bin_ln gives more than 2^30 bins");
    StarDev s = make_star(plan, atm, par);
    hipStream_t st = (hipStream_t)stream;
    const_cast<pz_plan*>(plan)->ws_valid = false;                       // populations are rewritten
    PZ_HIP(launch_populations(s, st));
    PZ_HIP(launch_select(s, eta_sel, bin_ln, (int)Bd, keep, R, R_deep, n_keep, st));
    return PZ_OK;
}

int synth_backward(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, const float* dL_dF,
                   const float* dL_dFc, float* g_loggf, float* g_damp, float* g_abund, float* g_xi,
                   pz_stream stream) {
    (void)dL_dFc;
    g_err.clear();
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    int rc = check_atmos(plan, atm);
    if (rc) return rc;
    if ((rc = check_params(par))) return rc;
    if (!dL_dF) return fail(PZ_E_INVALID_ARG, "dL_dF is required");
    StarDev s = make_star(plan, atm, par);
    s.dLdF = dL_dF;
    s.g_loggf = g_loggf;
    s.g_damp = g_damp;
    s.g_abund = g_abund;
    s.g_xi = g_xi;
    hipStream_t st = (hipStream_t)stream;
    if (!workspace_matches(plan, atm, par, st)) {
        const_cast<pz_plan*>(plan)->ws_valid = false;
        if ((rc = enqueue_opacity(plan, s, st))) return rc;
        record_workspace(plan, atm, par, st);
    }
    if ((rc = ensure_scatter_forward(plan, s, st))) return rc;
    {
        StageTimer t(plan, PZ_STAGE_REVERSE_SCAN, st);
        PZ_HIP(launch_reverse_scan(s, st));
    }
    {
        StageTimer t(plan, PZ_STAGE_GATHER, st);
        PZ_HIP(launch_gather(s, st));
    }
    StageTimer t(plan, PZ_STAGE_REDUCE, st);
    PZ_HIP(launch_reduce(s, st));
    return PZ_OK;
}

int pz_debug_opacity_adjoint(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, const float* dL_dF,
                             float* g_kappa, pz_stream stream) {
    g_err.clear();
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    int rc = check_atmos(plan, atm);
    if (rc) return rc;
    if ((rc = check_params(par))) return rc;
    if (!dL_dF || !g_kappa) return fail(PZ_E_INVALID_ARG, "dL_dF and g_kappa are required");
    StarDev s = make_star(plan, atm, par);
    s.dLdF = dL_dF;
    hipStream_t st = (hipStream_t)stream;
    if (!workspace_matches(plan, atm, par, st)) {
        const_cast<pz_plan*>(plan)->ws_valid = false;
        if ((rc = enqueue_opacity(plan, s, st))) return rc;
        record_workspace(plan, atm, par, st);
    }
    if ((rc = ensure_scatter_forward(plan, s, st))) return rc;
    PZ_HIP(launch_reverse_scan(s, st));
    PZ_HIP(hipMemcpy2DAsync(g_kappa, (size_t)plan->N * 4, plan->gk, (size_t)plan->Npad * 4, (size_t)plan->N * 4,
                            plan->D, hipMemcpyDeviceToDevice, st));
    return PZ_OK;
}

int pz_line_opacity(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, float* kappa_line,
                    pz_stream stream) {
    g_err.clear();
    if (!plan) return fail(PZ_E_INVALID_ARG, "plan is NULL");
    int rc = check_atmos(plan, atm);
    if (rc) return rc;
    if ((rc = check_params(par))) return rc;
    if (!kappa_line) return fail(PZ_E_INVALID_ARG, "kappa_line is required");
    StarDev s = make_star(plan, atm, par);
    hipStream_t st = (hipStream_t)stream;
    const_cast<pz_plan*>(plan)->ws_valid = false;
    if ((rc = enqueue_opacity(plan, s, st))) return rc;
    record_workspace(plan, atm, par, st);
    PZ_HIP(hipMemcpy2DAsync(kappa_line, (size_t)plan->N * 4, plan->kappa, (size_t)plan->Npad * 4,
                            (size_t)plan->N * 4, plan->D, hipMemcpyDeviceToDevice, st));
    return PZ_OK;
}

int pz_chi2_seed(int32_t N, const float* F, const float* Fc, const float* y, float sigma, float* dL_dF,
                 float* dL_dFc, float* loss, pz_stream stream) {
    g_err.clear();
    if (N < 1) return fail(PZ_E_SHAPE, "N must be >= 1");
    if (!F || !Fc || !y || !dL_dF) return fail(PZ_E_INVALID_ARG, "F, Fc, y and dL_dF are required");
    if (!(sigma > 0.0f) || !std::isfinite(sigma)) return fail(PZ_E_INVALID_ARG, "sigma must be finite and > 0");
    PZ_HIP(launch_chi2_seed(N, F, Fc, y, sigma, dL_dF, dL_dFc, loss, (hipStream_t)stream));
    return PZ_OK;
}

int pz_debug_formal_solve(int32_t D, int32_t n, const float* S, const float* tau, int32_t quadrature, float* F,
                          pz_stream stream) {
    g_err.clear();
    if (D < 2 || D > PZ_MAX_DEPTH) return fail(PZ_E_SHAPE, "D must be in [2, %d]", PZ_MAX_DEPTH);
    if (n < 0) return fail(PZ_E_SHAPE, "n must be >= 0");
    if (!S || !tau || !F) return fail(PZ_E_INVALID_ARG, "S, tau and F are required");
    if (quadrature != PZ_QUAD_GAUSS3 && quadrature != PZ_QUAD_E2)
        return fail(PZ_E_INVALID_ARG, "unknown quadrature %d", quadrature);
    if (n == 0) return PZ_OK;
    PZ_HIP(launch_debug_formal(D, n, S, tau, quadrature, F, (hipStream_t)stream));
    return PZ_OK;
}

}  // extern "C"
