// Windowed Voigt line opacity (Sec. 2.1 Eqs. 4-5; the bounded wing spans of
// Sec. 2.2): the tile kernel body that sums K H(a, v) over the lines
// overlapping a tile of pixels, for every depth, into kappa_line[D][Npad].
#pragma once

#include "pz_internal.h"
#include "pz_voigt.h"

namespace pz {

// x = lambda_l / lambda_i - 1 = expm1(delta - k h), k = i - ic: the
// detuning from an integer pixel offset and a float64-derived sub-pixel
// offset, so no large frequencies are subtracted in float32.
__device__ __forceinline__ float detuning(int k, float delta, float h_hi, float h_lo) {
    const float kf = (float)k;
    const float t = fmaf(-kf, h_lo, fmaf(-kf, h_hi, delta));
    return t * fmaf(t, fmaf(t, fmaf(t, 1.0f / 24.0f, 1.0f / 6.0f), 0.5f), 1.0f);
}

// -------------------------------------------------------------- opacity
// A workgroup of 8 wavefronts owns TPX = 8 WPX consecutive pixels x all
// depths.  The lines overlapping the tile are a contiguous range of the
// sorted list; per chunk of lines, their per-depth parameters and the
// detuning x of every (line, tile pixel) are staged in LDS (x = kNoLine
// outside the line's window; real detunings satisfy |x| < 1e-2).
//
// Depths split as D = nfull NDG + r, NDG = 64/WPX.  Main part: wavefront w
// covers pixels w WPX .. w WPX + WPX-1 of the tile, lane (px, dg) depths
// j = d NDG + dg, d < nfull -- nearby detunings, so little divergence between
// Voigt regions.  Tail: the TPX x r remaining (pixel, depth) pairs are dealt
// to the first wavefronts 64 at a time (pixel t / r, depth nfull NDG + t % r),
// so no lane idles on a partial depth group.  No atomics: every
// (pixel, depth) sum is owned by one thread and runs in sorted-line order.
static constexpr int MAX_CHUNK = 16;
static constexpr float kNoLine = 2.0f;

// The opacity loop is VALU-issue bound, so resident wavefronts matter more
// than the few spills a register cap costs (they fall in the per-tile and
// per-chunk code, not the evaluation loop): 8 waves per SIMD for 4-pixel
// wavefronts, 6 for the wider ones.
#define PZ_OPACITY_WAVES(WPX) __attribute__((amdgpu_waves_per_eu((WPX) == 4 ? 8 : 6)))

template <int WPX>
struct OpacityLds {
    float4 lp[MAX_CHUNK * MAXD];
    float zmax[MAX_CHUNK * MAXD];                     // centre test only
    float x[MAX_CHUNK * 8 * WPX];
    float4 pw[PZ_PW_N * 4];                           // piecewise core table
};

// With the centre test (CT) a pixel's detuning is marked kNoLine beyond the
// line's largest span, and a (pixel, depth) lane evaluates only where
// v^2 + a^2 <= zmax of its (line, depth).
template <int WPX, bool CT, bool WIDE>
__device__ __forceinline__ void opacity_tile_body(const StarDev& s, int tile, int chunk, OpacityLds<WPX>& sm) {
    constexpr int NDG = 64 / WPX;
    constexpr int DPT = MAXD / NDG;                    // most full depth groups
    constexpr int TPX = 8 * WPX;
    const int tid = threadIdx.x;
    const int lane = tid % 64;
    const int wave = tid / 64;
    const int px = wave * WPX + lane % WPX;           // main pixel within the tile
    const int dg = lane / WPX;
    const int D = s.D;
    const int nfull = D / NDG, r = D - nfull * NDG;
    const int t = tid;                                 // tail slot
    const bool tail = t < TPX * r;
    const int tpx = tail ? t / r : 0;
    const int tj = nfull * NDG + (tail ? t - tpx * r : 0);
    const int p0 = tile * TPX;
    const int l0 = s.tile_first[tile], l1 = s.tile_last[tile];
    const bool any_wide = s.wide_any[0] != 0;
    if (WIDE && !any_wide) return;
    if (WIDE) {                                        // nothing to add unless a line of the tile is flagged
        int any = 0;
        for (int l = l0 + tid; l < l1; l += 512) any |= s.wide_a[l];
        if (!__syncthreads_or(any)) return;
    }
    float acc[DPT], acc_t = 0.0f;
#pragma unroll
    for (int d = 0; d < DPT; ++d) acc[d] = 0.0f;

    for (int c0 = l0; c0 < l1; c0 += chunk) {
        const int nc = min(chunk, l1 - c0);
        const float4* src = s.lp + (size_t)c0 * D;
        for (int k = tid; k < nc * D; k += 512) {
            const int q = k / D;
            sm.lp[q * MAXD + (k - q * D)] = src[k];
            if (CT) sm.zmax[q * MAXD + (k - q * D)] = s.zmax[(size_t)c0 * D + k];
        }
        for (int k = tid; k < nc * TPX; k += 512) {
            const int q = k / TPX, i = p0 + (k - q * TPX);
            const int l = c0 + q;
            float x = kNoLine;
            if (i >= s.ln.ilo[l] && i <= s.ln.ihi[l] && (any_wide && s.wide_a[l] != 0) == WIDE)
                x = detuning(i - s.ln.ic[l], s.ln.delta[l], s.h_hi, s.h_lo);
            // the slack keeps every lane the per-depth test would accept
            if (CT && !(fabsf(x) <= s.xlim[l] * (1.0f + 1e-5f))) x = kNoLine;
            sm.x[k] = x;
        }
        __syncthreads();
        for (int q = 0; q < nc; ++q) {
            const float4* row = sm.lp + q * MAXD;
            const float* zrow = sm.zmax + q * MAXD;
            const float x = sm.x[q * TPX + px];
            if (x < 1.0f) {
#pragma unroll
                for (int d = 0; d < DPT; ++d) {
                    if (d < nfull) {
                        const float4 p = row[d * NDG + dg];
                        acc[d] = voigt_acc<CT, WIDE>(acc[d], p.y, p.z, p.w, x * p.x, sm.pw,
                                                     CT ? zrow[d * NDG + dg] : 0.0f);
                    }
                }
            }
            if (tail) {
                const float xt = sm.x[q * TPX + tpx];
                if (xt < 1.0f) {
                    const float4 p = row[tj];
                    acc_t = voigt_acc<CT, WIDE>(acc_t, p.y, p.z, p.w, xt * p.x, sm.pw, CT ? zrow[tj] : 0.0f);
                }
            }
        }
        __syncthreads();
    }
    const int i = p0 + px;
    if (i < s.N) {
#pragma unroll
        for (int d = 0; d < DPT; ++d)
            if (d < nfull) {
                float* k = s.kappa + (size_t)(d * NDG + dg) * s.Npad + i;
                *k = WIDE ? *k + acc[d] : acc[d];
            }
    }
    if (tail && p0 + tpx < s.N) {
        float* k = s.kappa + (size_t)tj * s.Npad + p0 + tpx;
        *k = WIDE ? *k + acc_t : acc_t;
    }
}

// Called by all 512 threads of a workgroup (it synchronises the workgroup);
// sm.pw must hold the piecewise core table.  The main pass (WIDE = false)
// writes the tile's opacity from every line not flagged wide_a; the wide
// pass then adds the flagged lines (whose damping ratio spans both near and
// far wing tiers across depths) with the evaluator that keeps each lane on
// its own tier, so the main pass's code stays as lean as before.
template <int WPX, bool WIDE>
__device__ __forceinline__ void dev_opacity_tile(const StarDev& s, int tile, int chunk, OpacityLds<WPX>& sm) {
    if (s.center)
        opacity_tile_body<WPX, true, WIDE>(s, tile, chunk, sm);
    else
        opacity_tile_body<WPX, false, WIDE>(s, tile, chunk, sm);
}

}  // namespace pz
