// Per-star HIP kernels (gfx950): thin wrappers that map the grid onto the
// stage bodies of pz_stages.h, plus their launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pz_stages.h"
#include "pz_scatter.h"

namespace pz {

__global__ __launch_bounds__(256) void k_populations(StarDev s) {
    dev_populations(s, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_line_consts(StarDev s) {
    __shared__ double red[3 * 256];
    const double3 bnd = damp_bounds(s, red);
    dev_line_consts(s, blockIdx.x * blockDim.x + threadIdx.x, bnd);
}

__global__ __launch_bounds__(256) void k_line_params(StarDev s) {
    dev_line_params(s, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// Persistent workgroups take tiles from a queue ordered by decreasing cost
// (longest-processing-time first): tiles differ several-fold in line count
// (band clusters), and a one-shot grid of ~N/TPX workgroups leaves a long
// tail of heavy tiles.
// CT: the plan uses the centre test (its LDS holds the zmax rows); G: depth-group
// slots per lane (at least D / (64 / WPX)); FG: exactly D / (64 / WPX).
template <int WPX, bool CT, int G, bool FG>
__global__ __launch_bounds__(512) PZ_OPACITY_WAVES(WPX) void k_opacity(StarDev s, int chunk) {
    PZ_OPACITY_LDS(WPX, CT, sm);
    __shared__ int s_it;
    load_pw_table(sm.pw, false);                       // visible after the first item fetch's barrier
    for (;;) {
        if (threadIdx.x == 0) s_it = atomicAdd(s.qctr, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_it);
        __syncthreads();
        if (it >= s.n_tiles) return;
        dev_opacity_tile<WPX, false, CT, G, true, FG>(s, s.tile_order[it], chunk, sm);
    }
}

// Adds the lines flagged wide_a (usually none) to the tiles they overlap.
template <int WPX, bool CT>
__global__ __launch_bounds__(512) PZ_OPACITY_WAVES(WPX) void k_opacity_wide(StarDev s, int chunk) {
    PZ_OPACITY_LDS(WPX, CT, sm);
    if (s.wide_any[0] == 0) return;                   // the usual case: no flagged line
    load_pw_table(sm.pw, false);
    __syncthreads();
    for (int t = blockIdx.x; t < s.n_tiles; t += gridDim.x)
        dev_opacity_tile<WPX, true, CT, opacity_max_groups<WPX>(), true>(s, t, chunk, sm);
}

__global__ void k_reset_queue(int* ctr) { ctr[0] = 0; }

__global__ __launch_bounds__(256) void k_select(StarDev s, double eta, double bin_ln, int B, unsigned char* keep,
                                                double* R, double* Rd, int* n_keep) {
    dev_select(s, blockIdx.x * blockDim.x + threadIdx.x, eta, bin_ln, B, keep, R, Rd, n_keep);
}

template <bool CT>
static hipError_t opacity_occupancy(int tile_px, int* occ) {
    switch (tile_px) {
        case 32: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_opacity<4, CT, 4, true>, 512, 0);
        case 64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_opacity<8, CT, 9, true>, 512, 0);
        default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_opacity<16, CT, 19, false>, 512, 0);
    }
}

int opacity_grid(int tile_px, bool center) {
    int dev = 0, n_cu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1024;
    const hipError_t e = center ? opacity_occupancy<true>(tile_px, &occ) : opacity_occupancy<false>(tile_px, &occ);
    if (e != hipSuccess || occ < 1) occ = 1;
    return n_cu * occ;
}

// blockIdx.y = 0: the total branch, from an LDS copy of the pixel's
// kappa_line column; blockIdx.y = 1: the continuum branch (reads no kappa_line).
__global__ __launch_bounds__(64) void k_flux(StarDev s) {
    __shared__ float kst[MAXD * WAVE];
    const int i = blockIdx.x * WAVE + threadIdx.x;
    if (blockIdx.y == 0) {
        if (i < s.N) stage_kappa_column(s, i, kst + threadIdx.x);
        dev_flux<true, false>(s, i, LdsKCol{kst + threadIdx.x});
    } else {
        dev_flux<false, true>(s, i, GlobalKCol{s.kappa + i, (size_t)s.Npad});
    }
}

// As k_flux, with the exact E2 angle integral in float64.
__global__ __launch_bounds__(64) void k_flux_e2(StarDev s) {
    __shared__ float kst[MAXD * WAVE];
    const int i = blockIdx.x * WAVE + threadIdx.x;
    if (blockIdx.y == 0) {
        if (i < s.N) stage_kappa_column(s, i, kst + threadIdx.x);
        dev_flux_e2<true, false>(s, i, LdsKCol{kst + threadIdx.x});
    } else {
        dev_flux_e2<false, true>(s, i, GlobalKCol{s.kappa + i, (size_t)s.Npad});
    }
}

__global__ __launch_bounds__(192) void k_flux_scatter(StarDev s) {
    dev_flux_scatter(s, blockIdx.x * 64 + threadIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(192) void k_reverse_scatter(StarDev s) {
    dev_reverse_scatter(s, blockIdx.x * 64 + threadIdx.x);
}

__global__ void k_debug_formal(int D, int n, const float* S, const float* tau, int quad, float* F) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (quad == PZ_QUAD_E2) {
        RayE2 r;
        r.start();
        const double S0 = S[i], S1 = S[n + i], t0 = tau[i], t1 = tau[n + i];
        r.seg(S0 - t0 * (S1 - S0) / (t1 - t0), S0, 0.0, t0);
        double Sa = S0, Sb = S1, ta = t0, tb = t1;
        for (int j = 1; j < D; ++j) {
            if (j > 1) {
                Sa = Sb;
                ta = tb;
                Sb = S[(size_t)j * n + i];
                tb = tau[(size_t)j * n + i];
            }
            r.seg(Sa, Sb, ta, tb);
        }
        F[i] = (float)r.bottom(Sa, Sb, ta, tb);
        return;
    }
    Ray3 r;
    r.top(S[i], S[n + i], tau[i], tau[n + i]);
    float Sa = S[i], Sb = S[n + i], ta = tau[i], tb = tau[n + i];
    for (int j = 1; j < D; ++j) {
        if (j > 1) {
            Sa = Sb;
            ta = tb;
            Sb = S[(size_t)j * n + i];
            tb = tau[(size_t)j * n + i];
        }
        r.seg(Sa, Sb, ta, tb);
    }
    F[i] = r.bottom(Sa, Sb, ta, tb);
}

// One thread per pixel; its float64 column in LDS holds kappa_line, then dL/dtau.
__global__ __launch_bounds__(64) void k_reverse_scan(StarDev s) {
    __shared__ double col[MAXD * WAVE];
    const int i = blockIdx.x * WAVE + threadIdx.x;
    if (i < s.N) stage_kappa_column64(s, i, col + threadIdx.x);
    dev_reverse_scan(s, i, col + threadIdx.x);
}

__global__ __launch_bounds__(64) void k_reverse_scan_e2(StarDev s) {
    __shared__ double col[MAXD * WAVE];
    const int i = blockIdx.x * WAVE + threadIdx.x;
    if (i < s.N) stage_kappa_column64(s, i, col + threadIdx.x);
    dev_reverse_scan_e2(s, i, col + threadIdx.x);
}

// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b mod 8).
// Renumbering them so that each XCD takes one contiguous range of blocks puts
// neighbouring lines, whose windows read the same dL/dkappa columns, on the
// same XCD and so in the same L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_contiguous_block(int b, int nb) {
    const int x = b % 8, p = b / 8, q = nb / 8, r = nb % 8;
    return x * q + min(x, r) + p;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_gather(StarDev s) {
    __shared__ float4 pw[2 * PZ_PW_LDS];
    __shared__ float4 lq[256 / WAVE][2 * MAXD];
    load_pw_table(pw, true);
    const int w = threadIdx.x / WAVE;
    const int blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int l = __builtin_amdgcn_readfirstlane(blk * (256 / WAVE) + w);
    stage_line_params(s, l, threadIdx.x % WAVE, lq[w]);
    __syncthreads();
    dev_gather(s, l, threadIdx.x % WAVE, pw, lq[w]);
}

__global__ __launch_bounds__(256) void k_scatter_lines(StarDev s) { dev_scatter(s, blockIdx.x * blockDim.x + threadIdx.x); }

__global__ __launch_bounds__(256) void k_reduce_partials(StarDev s) {
    __shared__ float red[256];
    dev_reduce_partial(s, blockIdx.x, blockIdx.y, red);
}

__global__ __launch_bounds__(256) void k_reduce_final(StarDev s) {
    __shared__ float red[256];
    dev_reduce_final(s, blockIdx.x, red);
}

__global__ __launch_bounds__(256) void k_chi2_seed(int N, const float* F, const float* Fc, const float* y, float inv_s2,
                                                   float* gF, float* gFc) {
    dev_chi2_seed(N, F, Fc, y, inv_s2, gF, gFc, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(1024) void k_chi2_loss(int N, const float* F, const float* Fc, const float* y,
                                                    float inv_s2, float* loss) {
    __shared__ float red[1024];
    dev_chi2_loss(N, F, Fc, y, inv_s2, loss, red);
}

// ------------------------------------------------------------- launchers
hipError_t launch_populations(const StarDev& s, hipStream_t st) {
    const int n = s.S * s.D;
    k_populations<<<(n + 255) / 256, 256, 0, st>>>(s);
    return hipGetLastError();
}

hipError_t launch_select(const StarDev& s, double eta, double bin_ln, int B, unsigned char* keep, double* R,
                         double* Rd, int* n_keep, hipStream_t st) {
    if (n_keep) k_reset_queue<<<1, 1, 0, st>>>(n_keep);
    if (s.L > 0) k_select<<<(s.L + 255) / 256, 256, 0, st>>>(s, eta, bin_ln, B, keep, R, Rd, n_keep);
    return hipGetLastError();
}

hipError_t launch_line_params(const StarDev& s, hipStream_t st) {
    const long n = (long)s.L * s.D;
    if (n == 0) return hipSuccess;
    k_line_consts<<<(s.L + 255) / 256, 256, 0, st>>>(s);
    k_line_params<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(s);
    return hipGetLastError();
}

// The main pass with the fewest depth-group slots that hold D / (64 / WPX)
// groups (with no empty slot where the depths allow), then the wide pass.
template <int WPX, bool CT>
static void launch_opacity_wpx(const StarDev& s, int chunk, int grid, hipStream_t st) {
    constexpr int GB = opacity_max_groups<WPX>();
    const int ng = s.D / (64 / WPX);                   // <= GB: D <= MAXD
    if (ng == GB)
        k_opacity<WPX, CT, GB, true><<<grid, 512, 0, st>>>(s, chunk);
    else if (ng == GB - 1)
        k_opacity<WPX, CT, GB - 1, true><<<grid, 512, 0, st>>>(s, chunk);
    else
        k_opacity<WPX, CT, GB - 1, false><<<grid, 512, 0, st>>>(s, chunk);
    k_opacity_wide<WPX, CT><<<grid, 512, 0, st>>>(s, chunk);
}

template <bool CT>
static hipError_t launch_opacity_tiles(const StarDev& s, int chunk, int grid, hipStream_t st) {
    switch (s.tile_px) {
        case 32: launch_opacity_wpx<4, CT>(s, chunk, grid, st); break;
        case 64: launch_opacity_wpx<8, CT>(s, chunk, grid, st); break;
        case 128: launch_opacity_wpx<16, CT>(s, chunk, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_opacity(const StarDev& s, int chunk, hipStream_t st) {
    if (s.n_tiles == 0) return hipSuccess;
    const int grid = std::max(1, std::min(s.grid_opacity, s.n_tiles));
    k_reset_queue<<<1, 1, 0, st>>>(s.qctr);
    return s.center ? launch_opacity_tiles<true>(s, chunk, grid, st) : launch_opacity_tiles<false>(s, chunk, grid, st);
}

hipError_t launch_flux(const StarDev& s, hipStream_t st) {
    if (s.scatter)
        k_flux_scatter<<<dim3((s.N + 63) / 64, 2), dim3(64, 3), 0, st>>>(s);
    else if (s.quad == PZ_QUAD_E2)
        k_flux_e2<<<dim3((s.N + WAVE - 1) / WAVE, 2), WAVE, 0, st>>>(s);
    else
        k_flux<<<dim3((s.N + WAVE - 1) / WAVE, 2), WAVE, 0, st>>>(s);
    return hipGetLastError();
}

hipError_t launch_reverse_scan(const StarDev& s, hipStream_t st) {
    if (s.scatter)
        k_reverse_scatter<<<(s.N + 63) / 64, dim3(64, 3), 0, st>>>(s);
    else if (s.quad == PZ_QUAD_E2)
        k_reverse_scan_e2<<<(s.N + 63) / 64, 64, 0, st>>>(s);
    else
        k_reverse_scan<<<(s.N + 63) / 64, 64, 0, st>>>(s);
    return hipGetLastError();
}

hipError_t launch_gather(const StarDev& s, hipStream_t st) {
    if (s.L == 0) return hipSuccess;
    k_gather<<<(s.L + 3) / 4, 256, 0, st>>>(s);
    return hipGetLastError();
}

hipError_t launch_reduce(const StarDev& s, hipStream_t st) {
    if (s.L > 0) k_scatter_lines<<<(s.L + 255) / 256, 256, 0, st>>>(s);
    k_reduce_partials<<<dim3(s.n_rchunk, s.S + 1), 256, 0, st>>>(s);
    k_reduce_final<<<s.S + 1, 256, 0, st>>>(s);
    return hipGetLastError();
}

hipError_t launch_chi2_seed(int N, const float* F, const float* Fc, const float* y, float sigma, float* gF,
                            float* gFc, float* loss, hipStream_t st) {
    const float inv_s2 = 1.0f / (sigma * sigma);
    k_chi2_seed<<<(N + 255) / 256, 256, 0, st>>>(N, F, Fc, y, inv_s2, gF, gFc);
    if (loss) k_chi2_loss<<<1, 1024, 0, st>>>(N, F, Fc, y, inv_s2, loss);
    return hipGetLastError();
}

hipError_t launch_debug_formal(int D, int n, const float* S, const float* tau, int quad, float* F, hipStream_t st) {
    k_debug_formal<<<(n + 255) / 256, 256, 0, st>>>(D, n, S, tau, quad, F);
    return hipGetLastError();
}

}  // namespace pz
