// Line-list calibration support (Sec. 6, Eq. 30).  The calibration fits four
// logarithmic corrections per group of catalogue lines (oscillator strength
// and the radiative, Stark and van der Waals damping constants) to standard
// spectra; every line of a group takes its group's values.  This file holds
//   - the greedy strength-ordered grouping (host code, run once per catalogue):
//     anchor complexes first, then each unassigned line, strongest first,
//     seeds a group with the unassigned lines of its species and ion stage
//     within dE and dlam of it;
//   - the group -> line expansion (a gather) and its transpose, a fixed-order
//     reduction of per-line gradients into groups (one thread per group and
//     row, members added in ascending line order: bitwise reproducible);
//   - the weighted mean-square loss of one standard on its observed pixels,
//     L = c sum_p w_p (f_p - y_p)^2, with its seed dL/df.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "pz_internal.h"

namespace pz {
int set_error(int code, const char* msg);
}

using namespace pz;

struct pz_groups {
    int L, G;
    int* q;      // [L]   group of each line, -1 = none
    int* off;    // [G+1] CSR offsets
    int* idx;    // [off[G]] member lines, ascending within a group
    void* base;
};

namespace {

constexpr int TPB = 256;
constexpr int MAX_ROWS = 64;

__global__ __launch_bounds__(TPB) void k_groups_expand(int L, int G, int R, const int* __restrict__ q,
                                                       const float* __restrict__ xg, float* __restrict__ xl) {
    const long t = (long)blockIdx.x * TPB + threadIdx.x;
    if (t >= (long)R * L) return;
    const int r = (int)(t / L), l = (int)(t - (long)r * L);
    const int g = q[l];
    xl[t] = g >= 0 ? xg[(long)r * G + g] : 0.0f;
}

__global__ __launch_bounds__(TPB) void k_groups_reduce(int L, int G, int R, const int* __restrict__ off,
                                                       const int* __restrict__ idx, const float* __restrict__ xl,
                                                       float* __restrict__ xg, int accumulate) {
    const long t = (long)blockIdx.x * TPB + threadIdx.x;
    if (t >= (long)R * G) return;
    const int r = (int)(t / G), g = (int)(t - (long)r * G);
    const float* row = xl + (long)r * L;
    float a = 0.0f;
    for (int k = off[g], e = off[g + 1]; k < e; ++k) a += row[idx[k]];
    xg[t] = accumulate ? xg[t] + a : a;
}

__global__ __launch_bounds__(TPB) void k_wmse_seed(int P, const float* __restrict__ f, const float* __restrict__ y,
                                                   const float* __restrict__ w, float two_c,
                                                   float* __restrict__ g) {
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= P) return;
    const float d = f[p] - y[p];
    g[p] = two_c * (w ? w[p] : 1.0f) * d;
}

// One workgroup: each thread sums a strided slice, then a fixed tree.
__global__ __launch_bounds__(1024) void k_wmse_loss(int P, const float* __restrict__ f, const float* __restrict__ y,
                                                    const float* __restrict__ w, float c, float* loss,
                                                    int accumulate) {
    __shared__ float red[1024];
    float acc = 0.0f;
    for (int p = threadIdx.x; p < P; p += 1024) {
        const float d = f[p] - y[p];
        acc = fmaf((w ? w[p] : 1.0f) * d, d, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = accumulate ? loss[0] + c * red[0] : c * red[0];
}

bool finite_all(const double* a, int32_t L, const uint8_t* active) {
    for (int32_t l = 0; l < L; ++l)
        if ((!active || active[l]) && !std::isfinite(a[l])) return false;
    return true;
}

}  // namespace

extern "C" {

int pz_correction_groups(int32_t L, const double* lam0_nm, const double* E_eV, const int32_t* species,
                         const int32_t* ion, const double* loggf, const uint8_t* active, const int32_t* anchor,
                         double dE_eV, double dlam_nm, int32_t* group_of_line, int32_t* n_groups) {
    if (!n_groups) return set_error(PZ_E_INVALID_ARG, "n_groups is NULL");
    *n_groups = 0;
    if (L < 0) return set_error(PZ_E_SHAPE, "L must be >= 0");
    if (L > 0 && (!lam0_nm || !E_eV || !species || !ion || !loggf || !group_of_line))
        return set_error(PZ_E_INVALID_ARG, "lam0_nm, E_eV, species, ion, loggf and group_of_line are required");
    if (!(dE_eV >= 0.0) || !(dlam_nm >= 0.0) || !std::isfinite(dE_eV) || !std::isfinite(dlam_nm))
        return set_error(PZ_E_INVALID_ARG, "dE_eV and dlam_nm must be finite and >= 0");
    if (!finite_all(lam0_nm, L, active) || !finite_all(E_eV, L, active) || !finite_all(loggf, L, active))
        return set_error(PZ_E_NONFINITE, "lam0_nm, E_eV and loggf must be finite for calibrated lines");
    std::vector<int32_t> q(L, -1);
    auto is_active = [&](int32_t l) { return !active || active[l] != 0; };
    int32_t G = 0;
    // anchor complexes: one group per distinct id, ascending
    if (anchor) {
        std::vector<int32_t> ids;
        for (int32_t l = 0; l < L; ++l)
            if (is_active(l) && anchor[l] >= 0) ids.push_back(anchor[l]);
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        for (int32_t l = 0; l < L; ++l)
            if (is_active(l) && anchor[l] >= 0)
                q[l] = (int32_t)(std::lower_bound(ids.begin(), ids.end(), anchor[l]) - ids.begin());
        G = (int32_t)ids.size();
    }
    // free lines sorted by (species, ion, lambda, index): each (species, ion)
    // bucket is a contiguous run ordered by wavelength
    std::vector<int32_t> byl;
    for (int32_t l = 0; l < L; ++l)
        if (is_active(l) && q[l] < 0) byl.push_back(l);
    std::sort(byl.begin(), byl.end(), [&](int32_t a, int32_t b) {
        if (species[a] != species[b]) return species[a] < species[b];
        if (ion[a] != ion[b]) return ion[a] < ion[b];
        if (lam0_nm[a] != lam0_nm[b]) return lam0_nm[a] < lam0_nm[b];
        return a < b;
    });
    const size_t n = byl.size();
    std::vector<int32_t> pos(L, -1), run_lo(n), run_hi(n);
    for (size_t k = 0; k < n; ++k) pos[byl[k]] = (int32_t)k;
    for (size_t k = 0; k < n;) {
        size_t e = k + 1;
        while (e < n && species[byl[e]] == species[byl[k]] && ion[byl[e]] == ion[byl[k]]) ++e;
        for (size_t j = k; j < e; ++j) {
            run_lo[j] = (int32_t)k;
            run_hi[j] = (int32_t)e;
        }
        k = e;
    }
    // visiting order: strongest first, ties by index
    std::vector<int32_t> order(byl);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (loggf[a] != loggf[b]) return loggf[a] > loggf[b];
        return a < b;
    });
    for (int32_t s : order) {
        if (q[s] >= 0) continue;
        const int32_t g = G++;
        const double ls = lam0_nm[s], es = E_eV[s];
        // candidates: a superset of the wavelength window, then the exact test
        const double pad = 2.0 * dlam_nm + 1e-9 * std::fabs(ls);
        const int32_t k0 = run_lo[pos[s]], k1 = run_hi[pos[s]];
        auto first = std::lower_bound(byl.begin() + k0, byl.begin() + k1, ls - pad,
                                      [&](int32_t m, double v) { return lam0_nm[m] < v; });
        for (auto it = first; it != byl.begin() + k1 && lam0_nm[*it] <= ls + pad; ++it) {
            const int32_t m = *it;
            if (q[m] < 0 && std::fabs(E_eV[m] - es) <= dE_eV && std::fabs(lam0_nm[m] - ls) <= dlam_nm) q[m] = g;
        }
    }
    std::copy(q.begin(), q.end(), group_of_line);
    *n_groups = G;
    return PZ_OK;
}

int pz_groups_create(int32_t L, int32_t G, const int32_t* group_of_line, pz_groups** out) {
    if (!out) return set_error(PZ_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (L < 1 || G < 1) return set_error(PZ_E_SHAPE, "L and G must be >= 1");
    if (!group_of_line) return set_error(PZ_E_INVALID_ARG, "group_of_line is required");
    std::vector<int32_t> off(G + 1, 0);
    for (int32_t l = 0; l < L; ++l) {
        const int32_t g = group_of_line[l];
        if (g < -1 || g >= G) return set_error(PZ_E_INVALID_ARG, "group_of_line entries must lie in [-1, G)");
        if (g >= 0) ++off[g + 1];
    }
    for (int32_t g = 0; g < G; ++g) off[g + 1] += off[g];
    std::vector<int32_t> fill(off.begin(), off.end() - 1), idx(std::max(off[G], 1));
    for (int32_t l = 0; l < L; ++l)
        if (group_of_line[l] >= 0) idx[fill[group_of_line[l]]++] = l;
    const size_t bq = ((size_t)L * 4 + 255) & ~(size_t)255, bo = ((size_t)(G + 1) * 4 + 255) & ~(size_t)255,
                 bi = (idx.size() * 4 + 255) & ~(size_t)255;
    pz_groups* h = new (std::nothrow) pz_groups();
    if (!h) return set_error(PZ_E_NOMEM, "host allocation failed");
    char* base = nullptr;
    if (hipMalloc((void**)&base, bq + bo + bi) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return set_error(PZ_E_NOMEM, "device allocation failed");
    }
    h->L = L;
    h->G = G;
    h->base = base;
    h->q = (int*)base;
    h->off = (int*)(base + bq);
    h->idx = (int*)(base + bq + bo);
    if (hipMemcpy(h->q, group_of_line, (size_t)L * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->off, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(base);
        delete h;
        return set_error(PZ_E_HIP, "upload of the group map failed");
    }
    *out = h;
    return PZ_OK;
}

void pz_groups_destroy(pz_groups* h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(h->base);
    delete h;
}

int pz_groups_info(const pz_groups* h, int32_t* L, int32_t* G) {
    if (!h) return set_error(PZ_E_INVALID_ARG, "groups is NULL");
    if (L) *L = h->L;
    if (G) *G = h->G;
    return PZ_OK;
}

int pz_groups_expand(const pz_groups* h, int32_t R, const float* x_group, float* x_line, pz_stream stream) {
    if (!h || !x_group || !x_line) return set_error(PZ_E_INVALID_ARG, "groups, x_group and x_line are required");
    if (R < 1 || R > MAX_ROWS) return set_error(PZ_E_SHAPE, "R must be in [1, 64]");
    const long n = (long)R * h->L;
    k_groups_expand<<<(unsigned)((n + TPB - 1) / TPB), TPB, 0, (hipStream_t)stream>>>(h->L, h->G, R, h->q, x_group,
                                                                                      x_line);
    if (hipGetLastError() != hipSuccess) return set_error(PZ_E_HIP, "k_groups_expand launch failed");
    return PZ_OK;
}

int pz_groups_reduce(const pz_groups* h, int32_t R, const float* x_line, float* x_group, int32_t accumulate,
                     pz_stream stream) {
    if (!h || !x_group || !x_line) return set_error(PZ_E_INVALID_ARG, "groups, x_line and x_group are required");
    if (R < 1 || R > MAX_ROWS) return set_error(PZ_E_SHAPE, "R must be in [1, 64]");
    const long n = (long)R * h->G;
    k_groups_reduce<<<(unsigned)((n + TPB - 1) / TPB), TPB, 0, (hipStream_t)stream>>>(
        h->L, h->G, R, h->off, h->idx, x_line, x_group, accumulate ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return set_error(PZ_E_HIP, "k_groups_reduce launch failed");
    return PZ_OK;
}

int pz_wmse_seed(int32_t P, const float* f, const float* y, const float* w, double c, float* dL_df, float* loss,
                 int32_t accumulate, pz_stream stream) {
    if (P < 1) return set_error(PZ_E_SHAPE, "P must be >= 1");
    if (!f || !y) return set_error(PZ_E_INVALID_ARG, "f and y are required");
    if (!dL_df && !loss) return set_error(PZ_E_INVALID_ARG, "dL_df or loss is required");
    if (!std::isfinite(c)) return set_error(PZ_E_NONFINITE, "c must be finite");
    hipStream_t st = (hipStream_t)stream;
    if (dL_df) k_wmse_seed<<<(P + TPB - 1) / TPB, TPB, 0, st>>>(P, f, y, w, (float)(2.0 * c), dL_df);
    if (loss) k_wmse_loss<<<1, 1024, 0, st>>>(P, f, y, w, (float)c, loss, accumulate ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return set_error(PZ_E_HIP, "wmse launch failed");
    return PZ_OK;
}

}  // extern "C"
