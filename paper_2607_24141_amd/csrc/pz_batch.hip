// Batched synthesis over many stars: every stage is one persistent launch
// whose workgroups take (star, item) work from a list spanning all stars.
// The opacity stage (dominant and skewed: stars differ in window length,
// line count and line density) pulls items from an atomic queue ordered by
// decreasing cost; the cheap, uniform stages stride over their lists.  The
// stage bodies are those of the per-star kernels (pz_stages.h), so each star
// gets bitwise the per-star result.  The host also hosts the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "pz_stages.h"

namespace pz {
int set_error(int code, const char* msg);
int check_atmos(const pz_plan* plan, const pz_atmos* atm);
int check_params(const pz_params* par);
StarDev make_star(const pz_plan* p, const pz_atmos* atm, const pz_params* par);
}  // namespace pz

using namespace pz;

namespace {

enum Phase {
    PH_POP,        // (star, 512 (species, depth) pairs)
    PH_LINES,      // (star, 512 lines): per-line factors
    PH_PARAMS,     // (star, PARAM_ITEM (line, depth) pairs)
    PH_OP32,       // (star, tile) of stars with 32-pixel tiles, decreasing cost, atomic queue
    PH_OP64,       // ... 64-pixel tiles
    PH_OP128,      // ... 128-pixel tiles
    PH_FLUX,       // (star, 512 pixels)
    PH_SEED,       // (star, 512 pixels): chi^2 seed for stars with a target
    PH_LOSS,       // (star): chi^2 value, one 1024-thread workgroup
    PH_REVERSE,    // (star, 64 pixels), 64-thread workgroups
    PH_GATHER,     // (star, GATHER_ITEM lines), atomic queue
    PH_SCATTER,    // (star, 512 lines)
    PH_PARTIAL,    // (star, list b * n_rchunk + c)
    PH_FINAL,      // (star, list b)
    N_PHASE
};

constexpr int PARAM_ITEM = 512 * 32;
constexpr int N_COUNTER = 4;             // queues: opacity x 3 tile widths, gather
constexpr int GATHER_ITEM = 64;

// Next item of an atomic queue for the whole workgroup (wavefront-uniform).
__device__ __forceinline__ int next_item(int* ctr, int* s_it) {
    if (threadIdx.x == 0) *s_it = atomicAdd(ctr, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*s_it);
    __syncthreads();
    return it;
}

// The item of a workgroup, made wavefront-uniform so the star descriptor is
// read with scalar loads.
__device__ __forceinline__ int2 uniform_item(const int2* __restrict__ items, int it) {
    const int2 w = items[it];
    return make_int2(__builtin_amdgcn_readfirstlane(w.x), __builtin_amdgcn_readfirstlane(w.y));
}

__global__ void kb_reset(int* ctr, int n) {
    if ((int)threadIdx.x < n) ctr[threadIdx.x] = 0;
}

__global__ __launch_bounds__(512) void kb_pop(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        dev_populations(stars[w.x], w.y * 512 + threadIdx.x);
    }
}

__global__ __launch_bounds__(512) void kb_lines(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    __shared__ double red[3 * 512];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const double3 bnd = damp_bounds(stars[w.x], red);
        dev_line_consts(stars[w.x], w.y * 512 + threadIdx.x, bnd);
    }
}

__global__ __launch_bounds__(512) void kb_params(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        const long base = (long)w.y * PARAM_ITEM;
        for (int k = threadIdx.x; k < PARAM_ITEM; k += 512) dev_line_params(s, base + k);
    }
}

// ANYCT: some star of the batch uses the centre test (the LDS holds its rows);
// G: depth-group slots (at least D / (64 / WPX) for every star); FG: exactly
// D / (64 / WPX) for every star.
template <int WPX, bool ANYCT, int G, bool FG>
__global__ __launch_bounds__(512) PZ_OPACITY_WAVES(WPX) void kb_opacity(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n, int* ctr) {
    PZ_OPACITY_LDS(WPX, ANYCT, sm);
    __shared__ int s_it;
    load_pw_table(sm.pw, false);                       // visible after the first item fetch's barrier
    for (;;) {
        const int it = next_item(ctr, &s_it);
        if (it >= n) return;
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        dev_opacity_tile<WPX, false, ANYCT, G, false, FG>(s, w.y, s.chunk, sm);
    }
}

// Adds the lines flagged wide_a (usually none) to every (star, tile) item.
template <int WPX, bool ANYCT>
__global__ __launch_bounds__(512) PZ_OPACITY_WAVES(WPX) void kb_opacity_wide(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    PZ_OPACITY_LDS(WPX, ANYCT, sm);
    load_pw_table(sm.pw, false);
    __syncthreads();
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        dev_opacity_tile<WPX, true, ANYCT, opacity_max_groups<WPX>(), false>(s, w.y, s.chunk, sm);
    }
}

__global__ __launch_bounds__(512) void kb_flux(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        const int i = w.y * 512 + threadIdx.x;
        if (s.quad == PZ_QUAD_E2)
            dev_flux_e2<true, true>(s, i, GlobalKCol{s.kappa + i, (size_t)s.Npad});
        else
            dev_flux<true, true>(s, i, GlobalKCol{s.kappa + i, (size_t)s.Npad});
    }
}

__global__ __launch_bounds__(512) void kb_seed(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n, const float* inv_s2,
                                               const float* const* ys) {
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        dev_chi2_seed(s.N, s.F, s.Fc, ys[w.x], inv_s2[w.x], const_cast<float*>(s.dLdF), nullptr,
                      w.y * 512 + threadIdx.x);
    }
}

__global__ __launch_bounds__(1024) void kb_loss(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n, const float* inv_s2,
                                                const float* const* ys, float* const* losses) {
    __shared__ float red[1024];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        dev_chi2_loss(s.N, s.F, s.Fc, ys[w.x], inv_s2[w.x], losses[w.x], red);
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void kb_reverse(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    __shared__ double col[MAXD * WAVE];               // each thread's own column
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        const int i = w.y * 64 + threadIdx.x;
        if (s.quad == PZ_QUAD_E2) {
            if (i < s.N) stage_kappa_column64(s, i, col + threadIdx.x);
            dev_reverse_scan_e2(s, i, col + threadIdx.x);
        } else {
            if (i < s.N) stage_kappa_column64(s, i, col + threadIdx.x);
            dev_reverse_scan(s, i, col + threadIdx.x);
        }
    }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8))) void kb_gather(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n, int* ctr) {
    __shared__ int s_it;
    __shared__ float4 pw[2 * PZ_PW_LDS];
    __shared__ float4 lq[512 / WAVE][2 * MAXD];
    load_pw_table(pw, true);                           // visible after the first item fetch's barrier
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    for (;;) {
        const int it = next_item(ctr, &s_it);
        if (it >= n) return;
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        for (int q = wave; q < GATHER_ITEM; q += 512 / WAVE) {
            const int l = __builtin_amdgcn_readfirstlane(w.y * GATHER_ITEM + q);
            // the row is private to this wavefront: order its writes before the
            // reads and the previous line's reads before the writes
            __builtin_amdgcn_wave_barrier();
            stage_line_params(s, l, lane, lq[wave]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            dev_gather(s, l, lane, pw, lq[wave]);
        }
    }
}

__global__ __launch_bounds__(512) void kb_scatter(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        dev_scatter(stars[w.x], w.y * 512 + threadIdx.x);
    }
}

__global__ __launch_bounds__(256) void kb_partial(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    __shared__ float red[256];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        const StarDev& s = stars[w.x];
        dev_reduce_partial(s, w.y % s.n_rchunk, w.y / s.n_rchunk, red);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void kb_final(const StarDev* __restrict__ stars, const int2* __restrict__ items, int n) {
    __shared__ float red[256];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = uniform_item(items, it);
        dev_reduce_final(stars[w.x], w.y, red);
        __syncthreads();
    }
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

template <bool ANYCT>
static hipError_t batch_opacity_occupancy(int* occ) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], kb_opacity<4, ANYCT, 4, true>, 512, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[1], kb_opacity<8, ANYCT, 9, true>, 512, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[2], kb_opacity<16, ANYCT, 19, false>, 512, 0);
    return e;
}

struct pz_batch {
    int n_star;
    int device;
    bool has_target;
    bool any_center;      // some star uses the centre test
    int max_d;            // largest depth count of the stars
    int min_d;            // smallest depth count of the stars
    std::vector<StarDev> sc_stars;   // stars with continuum scattering (their own flux and reverse launches)
    std::vector<const pz_plan*> plans;
    int n_items[N_PHASE];
    int2* items[N_PHASE];
    StarDev* stars;
    float* inv_s2;
    const float** ys;
    float** losses;
    int* ctr;             // [N_COUNTER] queue counters: opacity (32, 64, 128), gather
    int grid512, grid256, grid1024, grid_op[3], grid_gather, grid_rev;
    void* base;
};

// One phase's opacity launches: the main pass with the fewest depth-group
// slots that hold every star's D / (64 / WPX) groups (with no empty slot when
// every star has the same group count), then the wide pass.
template <int WPX, bool ANYCT>
static void batch_opacity_wpx(const pz_batch* bt, int n, const int2* items, int* ctr, int grid, hipStream_t st) {
    constexpr int GB = opacity_max_groups<WPX>();
    const int ng = bt->max_d / (64 / WPX);             // <= GB: D <= MAXD
    const bool same = bt->min_d / (64 / WPX) == ng;
    if (ng == GB)
        same ? kb_opacity<WPX, ANYCT, GB, true><<<grid, 512, 0, st>>>(bt->stars, items, n, ctr)
             : kb_opacity<WPX, ANYCT, GB, false><<<grid, 512, 0, st>>>(bt->stars, items, n, ctr);
    else if (ng == GB - 1 && same)
        kb_opacity<WPX, ANYCT, GB - 1, true><<<grid, 512, 0, st>>>(bt->stars, items, n, ctr);
    else
        kb_opacity<WPX, ANYCT, GB - 1, false><<<grid, 512, 0, st>>>(bt->stars, items, n, ctr);
    kb_opacity_wide<WPX, ANYCT><<<grid, 512, 0, st>>>(bt->stars, items, n);
}

template <bool ANYCT>
static void batch_opacity(const pz_batch* bt, hipStream_t st) {
    auto grid = [](int want, int n) { return std::max(1, std::min(want, n)); };
    const int* n = bt->n_items;
    int2* const* it = bt->items;
    if (n[PH_OP32]) batch_opacity_wpx<4, ANYCT>(bt, n[PH_OP32], it[PH_OP32], bt->ctr, grid(bt->grid_op[0], n[PH_OP32]), st);
    if (n[PH_OP64])
        batch_opacity_wpx<8, ANYCT>(bt, n[PH_OP64], it[PH_OP64], bt->ctr + 1, grid(bt->grid_op[1], n[PH_OP64]), st);
    if (n[PH_OP128])
        batch_opacity_wpx<16, ANYCT>(bt, n[PH_OP128], it[PH_OP128], bt->ctr + 2, grid(bt->grid_op[2], n[PH_OP128]), st);
}

extern "C" {

int pz_batch_create(int32_t n_star, const pz_star* stars, pz_batch** out) {
    if (!out) return set_error(PZ_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_star < 1 || !stars) return set_error(PZ_E_INVALID_ARG, "need n_star >= 1 stars");
    std::vector<StarDev> sd(n_star);
    std::vector<float> inv_s2(n_star, 0.0f);
    std::vector<const float*> ys(n_star, nullptr);
    std::vector<float*> losses(n_star, nullptr);
    std::vector<std::vector<int2>> items(N_PHASE);
    bool has_target = false;
    for (int b = 0; b < n_star; ++b) {
        const pz_star& st = stars[b];
        if (!st.plan) return set_error(PZ_E_INVALID_ARG, "star without a plan");
        for (int c = 0; c < b; ++c)
            if (stars[c].plan == st.plan) return set_error(PZ_E_INVALID_ARG, "two stars share a plan");
        int rc = check_atmos(st.plan, &st.atm);
        if (rc) return rc;
        if ((rc = check_params(&st.par))) return rc;
        if (st.atm.sigma_c && !st.plan->scatter_ws)
            return set_error(PZ_E_INVALID_ARG,
                             "a star has sigma_c but its plan was built without PZ_FLAG_SCATTERING");
        if (!st.F || !st.Fc) return set_error(PZ_E_INVALID_ARG, "every star needs F and Fc");
        if (st.y && !(st.sigma > 0.0f)) return set_error(PZ_E_INVALID_ARG, "sigma must be > 0 with a target y");
        const pz_plan* p = st.plan;
        StarDev s = make_star(p, &st.atm, &st.par);
        s.F = st.F;
        s.Fc = st.Fc;
        s.dLdF = st.y ? p->seed : st.dL_dF;
        s.g_loggf = st.g_loggf;
        s.g_damp = st.g_damp;
        s.g_abund = st.g_abund;
        s.g_xi = st.g_xi;
        sd[b] = s;
        if (st.y) {
            has_target = true;
            inv_s2[b] = 1.0f / (st.sigma * st.sigma);
            ys[b] = st.y;
            losses[b] = st.loss;
        }
        const long nld = (long)s.L * s.D;
        for (int k = 0; k < (s.S * s.D + 511) / 512; ++k) items[PH_POP].push_back({b, k});
        for (int k = 0; k < (s.L + 511) / 512; ++k) items[PH_LINES].push_back({b, k});
        for (long k = 0; k < (nld + PARAM_ITEM - 1) / PARAM_ITEM; ++k) items[PH_PARAMS].push_back({b, (int)k});
        const int ph_op = s.tile_px == 32 ? PH_OP32 : (s.tile_px == 64 ? PH_OP64 : PH_OP128);
        for (int t = 0; t < s.n_tiles; ++t) items[ph_op].push_back({b, t});
        // a star with scattering runs its transfer and reverse transfer in launches of its own
        for (int k = 0; k < (s.N + 511) / 512; ++k) {
            if (!s.scatter) items[PH_FLUX].push_back({b, k});
            if (st.y) items[PH_SEED].push_back({b, k});
        }
        if (!s.scatter)
            for (int k = 0; k < (s.N + 63) / 64; ++k) items[PH_REVERSE].push_back({b, k});
        if (st.y && st.loss) items[PH_LOSS].push_back({b, 0});
        for (int k = 0; k < (s.L + GATHER_ITEM - 1) / GATHER_ITEM; ++k) items[PH_GATHER].push_back({b, k});
        for (int k = 0; k < (s.L + 511) / 512; ++k) items[PH_SCATTER].push_back({b, k});
        for (int k = 0; k < (s.S + 1) * s.n_rchunk; ++k) items[PH_PARTIAL].push_back({b, k});
        for (int k = 0; k < s.S + 1; ++k) items[PH_FINAL].push_back({b, k});
    }
    // opacity work: most expensive tiles first (longest-processing-time order)
    for (int ph : {PH_OP32, PH_OP64, PH_OP128})
        std::stable_sort(items[ph].begin(), items[ph].end(), [&](const int2& x, const int2& y) {
            return stars[x.x].plan->tile_cost[x.y] > stars[y.x].plan->tile_cost[y.y];
        });

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    size_t o_items[N_PHASE];
    for (int ph = 0; ph < N_PHASE; ++ph) o_items[ph] = take(std::max<size_t>(items[ph].size(), 1) * sizeof(int2));
    const size_t o_st = take(n_star * sizeof(StarDev)), o_is = take(n_star * 4), o_ys = take(n_star * 8),
                 o_ls = take(n_star * 8), o_ctr = take(N_COUNTER * 4);
    pz_batch* bt = new (std::nothrow) pz_batch();
    if (!bt) return set_error(PZ_E_NOMEM, "host allocation failed");
    char* base = nullptr;
    if (hipGetDevice(&bt->device) != hipSuccess || hipMalloc((void**)&base, off) != hipSuccess) {
        (void)hipGetLastError();
        delete bt;
        return set_error(PZ_E_NOMEM, "device allocation for the batch failed");
    }
    bt->base = base;
    bt->n_star = n_star;
    bt->has_target = has_target;
    hipError_t e = hipSuccess;
    for (int ph = 0; ph < N_PHASE; ++ph) {
        bt->items[ph] = (int2*)(base + o_items[ph]);
        bt->n_items[ph] = (int)items[ph].size();
        if (e == hipSuccess && !items[ph].empty())
            e = hipMemcpy(bt->items[ph], items[ph].data(), items[ph].size() * sizeof(int2), hipMemcpyHostToDevice);
    }
    bt->stars = (StarDev*)(base + o_st);
    bt->inv_s2 = (float*)(base + o_is);
    bt->ys = (const float**)(base + o_ys);
    bt->losses = (float**)(base + o_ls);
    bt->ctr = (int*)(base + o_ctr);
    if (e == hipSuccess) e = hipMemcpy(bt->stars, sd.data(), n_star * sizeof(StarDev), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->inv_s2, inv_s2.data(), n_star * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->ys, ys.data(), n_star * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bt->losses, losses.data(), n_star * 8, hipMemcpyHostToDevice);
    int n_cu = 0, occ_op[3] = {0, 0, 0}, occ_g = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, bt->device);
    bt->any_center = false;
    bt->max_d = 0;
    bt->min_d = MAXD;
    for (int b = 0; b < n_star; ++b) {
        bt->any_center = bt->any_center || sd[b].center;
        bt->max_d = std::max(bt->max_d, sd[b].D);
        bt->min_d = std::min(bt->min_d, sd[b].D);
    }
    if (e == hipSuccess)
        e = bt->any_center ? batch_opacity_occupancy<true>(occ_op) : batch_opacity_occupancy<false>(occ_op);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_g, kb_gather, 512, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete bt;
        return set_error(PZ_E_HIP, hipGetErrorString(e));
    }
    for (int k = 0; k < 3; ++k) bt->grid_op[k] = std::max(1, n_cu * std::max(occ_op[k], 1));
    bt->grid_gather = std::max(1, n_cu * std::max(occ_g, 1));
    bt->grid512 = std::max(1, n_cu * 4);
    bt->grid256 = std::max(1, n_cu * 8);
    bt->grid1024 = std::max(1, n_cu * 2);
    bt->grid_rev = std::max(1, n_cu * 16);
    bt->plans.reserve(n_star);
    for (int b = 0; b < n_star; ++b) bt->plans.push_back(stars[b].plan);
    for (int b = 0; b < n_star; ++b)
        if (sd[b].scatter) bt->sc_stars.push_back(sd[b]);
    *out = bt;
    return PZ_OK;
}

void pz_batch_destroy(pz_batch* batch) {
    if (!batch) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(batch->base);
    delete batch;
}

int synth_batch(const pz_batch* bt, int32_t mode, pz_stream stream) {
    if (!bt) return set_error(PZ_E_INVALID_ARG, "batch is NULL");
    if (mode != PZ_MODE_FWD && mode != PZ_MODE_FWD_BWD) return set_error(PZ_E_INVALID_ARG, "unknown mode");
    hipStream_t st = (hipStream_t)stream;
    auto grid = [](int want, int n) { return std::max(1, std::min(want, n)); };
    const int* n = bt->n_items;
    int2* const* it = bt->items;
    kb_reset<<<1, 64, 0, st>>>(bt->ctr, N_COUNTER);
    kb_pop<<<grid(bt->grid512, n[PH_POP]), 512, 0, st>>>(bt->stars, it[PH_POP], n[PH_POP]);
    if (n[PH_LINES]) kb_lines<<<grid(bt->grid512, n[PH_LINES]), 512, 0, st>>>(bt->stars, it[PH_LINES], n[PH_LINES]);
    kb_params<<<grid(bt->grid512, n[PH_PARAMS]), 512, 0, st>>>(bt->stars, it[PH_PARAMS], n[PH_PARAMS]);
    if (bt->any_center)
        batch_opacity<true>(bt, st);
    else
        batch_opacity<false>(bt, st);
    if (n[PH_FLUX]) kb_flux<<<grid(bt->grid512, n[PH_FLUX]), 512, 0, st>>>(bt->stars, it[PH_FLUX], n[PH_FLUX]);
    for (const StarDev& s : bt->sc_stars) {
        const hipError_t e = launch_flux(s, st);
        if (e != hipSuccess) return set_error(PZ_E_HIP, hipGetErrorString(e));
    }
    if (n[PH_SEED])
        kb_seed<<<grid(bt->grid512, n[PH_SEED]), 512, 0, st>>>(bt->stars, it[PH_SEED], n[PH_SEED], bt->inv_s2, bt->ys);
    if (n[PH_LOSS])
        kb_loss<<<grid(bt->grid1024, n[PH_LOSS]), 1024, 0, st>>>(bt->stars, it[PH_LOSS], n[PH_LOSS], bt->inv_s2,
                                                                 bt->ys, bt->losses);
    if (mode == PZ_MODE_FWD_BWD) {
        if (n[PH_REVERSE])
            kb_reverse<<<grid(bt->grid_rev, n[PH_REVERSE]), 64, 0, st>>>(bt->stars, it[PH_REVERSE], n[PH_REVERSE]);
        for (const StarDev& s : bt->sc_stars) {
            const hipError_t e = launch_reverse_scan(s, st);
            if (e != hipSuccess) return set_error(PZ_E_HIP, hipGetErrorString(e));
        }
        kb_gather<<<grid(bt->grid_gather, n[PH_GATHER]), 512, 0, st>>>(bt->stars, it[PH_GATHER], n[PH_GATHER],
                                                                        bt->ctr + 3);
        kb_scatter<<<grid(bt->grid512, n[PH_SCATTER]), 512, 0, st>>>(bt->stars, it[PH_SCATTER], n[PH_SCATTER]);
        kb_partial<<<grid(bt->grid256, n[PH_PARTIAL]), 256, 0, st>>>(bt->stars, it[PH_PARTIAL], n[PH_PARTIAL]);
        kb_final<<<grid(bt->grid256, n[PH_FINAL]), 256, 0, st>>>(bt->stars, it[PH_FINAL], n[PH_FINAL]);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(PZ_E_HIP, hipGetErrorString(e));
    for (const pz_plan* p : bt->plans) {
        const_cast<pz_plan*>(p)->ws_valid = false;
        const_cast<pz_plan*>(p)->sc_ok = false;
    }
    return PZ_OK;
}

int pz_autotune(const pz_grid* grid, const pz_lines* lines, int32_t n_species, int32_t n_depth,
                const pz_options* base, const pz_atmos* atm, const pz_params* par, int32_t reps, pz_options* best,
                float* best_ms) {
    if (!grid || !lines || !base || !atm || !par || !best) return set_error(PZ_E_INVALID_ARG, "null argument");
    if (reps < 1) return set_error(PZ_E_INVALID_ARG, "reps must be >= 1");
    const int tiles[3] = {32, 64, 128};
    const int chunks[2] = {8, 16};
    float* F = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float bms = 1e30f;
    pz_options bo = *base;
    int rc = PZ_OK;
    if (hipMalloc((void**)&F, (size_t)2 * std::max(grid->N, 1) * 4) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = set_error(PZ_E_NOMEM, "autotune buffers");
    }
    for (int ti = 0; ti < 3 && rc == PZ_OK; ++ti) {
        for (int ci = 0; ci < 2 && rc == PZ_OK; ++ci) {
            pz_options o = *base;
            o.tile_px = tiles[ti];
            o.lines_per_chunk = chunks[ci];
            pz_plan* p = nullptr;
            if ((rc = pz_plan_create(grid, lines, n_species, n_depth, &o, &p))) break;
            if ((rc = synth_forward(p, atm, par, F, F + grid->N, nullptr)) == PZ_OK) {
                (void)hipEventRecord(e0, nullptr);
                for (int r = 0; r < reps && rc == PZ_OK; ++r) rc = synth_forward(p, atm, par, F, F + grid->N, nullptr);
                (void)hipEventRecord(e1, nullptr);
                float ms = 0.0f;
                if (rc == PZ_OK && hipEventSynchronize(e1) == hipSuccess &&
                    hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
                    ms /= reps;
                    if (ms < bms) {
                        bms = ms;
                        bo = o;
                    }
                }
            }
            pz_plan_destroy(p);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (F) (void)hipFree(F);
    if (rc) return rc;
    *best = bo;
    if (best_ms) *best_ms = bms;
    return PZ_OK;
}

}  // extern "C"
