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
// depths.  The lines overlapping the tile are a contiguous range [l0, l1) of
// the sorted list, taken in chunks of at most MAX_CHUNK lines; chunk c holds
// the lines l0 + c + q nch (q = 0, 1, ...; nch chunks), so every chunk spans
// the tile's whole line range and the wavefronts' shares of a chunk are
// alike (a chunk of neighbouring lines would leave the wavefronts beyond its
// windows idle at the barrier).  Per chunk, the lines' per-depth parameters
// and the detuning x of every (line, tile pixel) are staged in LDS (x =
// kNoLine outside the line's window; real detunings satisfy |x| < 1e-2).
// For the plain sum two LDS buffers alternate: the parameters of chunk c + 1
// are copied from global memory straight into LDS while chunk c is summed,
// and its detunings are written after, so each chunk costs one barrier.  A
// workgroup that can meet the centre test stages one buffer and then sums it.
//
// Depths split as D = nfull NDG + r, NDG = 64/WPX.  Main part: wavefront w
// covers pixels w WPX .. w WPX + WPX-1 of the tile, lane (px, dg) depths
// j = d NDG + dg, d < nfull -- nearby detunings, so little divergence between
// Voigt regions.  Tail: the TPX x r remaining (pixel, depth) pairs are dealt
// to the first wavefronts 64 at a time (pixel t / r, depth nfull NDG + t % r).
// No atomics: every (pixel, depth) sum is owned by one thread and runs in a
// fixed line order (chunk by chunk).
static constexpr float kNoLine = 2.0f;

// Resident wavefronts per SIMD.  Six for 4-pixel wavefronts: the 80 VGPRs
// keep the straight-line wing sums of all depth groups in registers, and
// three workgroups per CU still overlap one another's barriers.
#define PZ_OPACITY_WAVES(WPX) __attribute__((amdgpu_waves_per_eu(6)))

// LDS of one workgroup: chunk buffers of parameter rows (rows of D) and
// detunings -- two, alternating, for the plain sum; one with the centre
// test (CT), whose zmax rows take the room of the second and which so keeps
// three workgroups per CU -- and the piecewise core table.  Each is an
// array of its own (PZ_OPACITY_LDS declares them in the kernel): the
// compiler then knows that reading one buffer cannot touch the copies in
// flight into the other, and does not wait for them.
template <int WPX, bool CT>
struct OpacityLds {
    static constexpr int NB = CT ? 1 : 2;
    float4* lp0;
    float4* lp1;
    float* x0;
    float* x1;
    int* f0;                     // window fields of a chunk's lines, [NFIELD][MAX_CHUNK]
    int* f1;
    float* zmax;
    float4* pw;
};

// Window fields staged per line: ilo, ihi, ic, the bits of delta, wide_a.
static constexpr int NFIELD = 5;

#define PZ_OPACITY_LDS(WPX, CT, sm)                                                        \
    __shared__ float4 sm##_lp0[MAX_CHUNK * MAXD];                                          \
    __shared__ float4 sm##_lp1[(CT) ? 1 : MAX_CHUNK * MAXD];                               \
    __shared__ float sm##_x0[MAX_CHUNK * 8 * (WPX)];                                       \
    __shared__ float sm##_x1[(CT) ? 1 : MAX_CHUNK * 8 * (WPX)];                            \
    __shared__ int sm##_f0[(CT) ? 1 : NFIELD * MAX_CHUNK];                                 \
    __shared__ int sm##_f1[(CT) ? 1 : NFIELD * MAX_CHUNK];                                 \
    __shared__ float sm##_zmax[(CT) ? MAX_CHUNK * MAXD : 1];                               \
    __shared__ float4 sm##_pw[PZ_PW_LDS];                                                \
    const OpacityLds<WPX, CT> sm { sm##_lp0, sm##_lp1, sm##_x0, sm##_x1, sm##_f0, sm##_f1, sm##_zmax, sm##_pw }

// A wavefront-uniform pointer the compiler treats as opaque, held in scalar
// registers: per-lane addresses are then this base plus a 32-bit offset,
// not 64-bit induction variables kept across the chunk loop.
__device__ __forceinline__ const char* scalar_base(const void* p) {
    // the builtin returns int: both halves go through unsigned, so the low
    // word is zero-extended (a sign-extended low word would corrupt the high)
    const unsigned long long u = (unsigned long long)p;
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((unsigned)u);
    unsigned long long v = ((unsigned long long)hi << 32) | lo;
    asm volatile("" : "+s"(v));
    return (const char*)v;
}

// A wavefront-uniform integer, opaque to the compiler (so nothing computed
// from it is hoisted out of the caller's loop).
__device__ __forceinline__ int scalar_opaque(int x) {
    x = __builtin_amdgcn_readfirstlane(x);
    asm volatile("" : "+s"(x));
    return x;
}

// Copies of chunk c's parameter rows (and, CT, zmax rows) into dst: LDS
// element k = q D + j of the chunk is row l0 + c + q nch, depth j.  Each
// wavefront instruction moves 64 elements from global memory straight into
// consecutive LDS slots; they are complete once the issuing wavefront's load
// counter drains.  The per-lane byte offsets fit 32 bits: the plan keeps
// every tile's rows under 2^28 elements.
template <int WPX, bool CT, class Lds>
__device__ __forceinline__ void stage_rows(const StarDev& s, int l0, int c, int nch, int nc, float4* dst,
                                           const Lds& sm) {
    constexpr int LPT = (MAX_CHUNK * MAXD + 511) / 512;
    const size_t row0 = (size_t)(l0 + c) * s.D;
    // offsets are recomputed per chunk, never hoisted
    const int D = scalar_opaque(s.D), stride = scalar_opaque((nch - 1) * s.D);
    const int n = nc * D;
    const int lane = threadIdx.x % WAVE;
    const float inv_d = __builtin_amdgcn_rcpf((float)D);   // to 1 ulp: ample for the split below
    const char* lp = scalar_base(s.lp + row0);
    const char* zm = CT ? scalar_base(s.zmax + row0) : nullptr;
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
        const int k0 = u * 512 + (threadIdx.x & ~(WAVE - 1));   // wavefront-uniform
        const int k = k0 + lane;
        if (k0 < n && k < n) {
            // k / D: (k + 1/2) / D lies at least 1/(2D) from an integer
            const int q = (int)(((float)k + 0.5f) * inv_d);
            const unsigned e = (unsigned)(k + q * stride);     // element offset from row0, < (l1 - l0) D
            __builtin_amdgcn_global_load_lds((const void*)(lp + e * 16u),
                                             (__attribute__((address_space(3))) void*)(dst + k0), 16, 0, 0);
            if (CT)
                __builtin_amdgcn_global_load_lds((const void*)(zm + e * 4u),
                                                 (__attribute__((address_space(3))) void*)(sm.zmax + k0), 4, 0, 0);
        }
    }
}

// Copies of the window fields of chunk c's lines into dst[NFIELD][MAX_CHUNK]
// by wavefront 0 (lane j: line l0 + c + j nch).
__device__ __forceinline__ void stage_fields(const StarDev& s, int l0, int c, int nch, int nc, int* dst) {
    if (threadIdx.x >= WAVE) return;
    const int step = scalar_opaque(nch);
    const int j = threadIdx.x;
    if (j >= nc) return;
    const unsigned off = (unsigned)(j * step) * 4u;
    auto copy = [&](const void* field, int f) {
        __builtin_amdgcn_global_load_lds((const void*)(scalar_base((const int*)field + l0 + c) + off),
                                         (__attribute__((address_space(3))) void*)(dst + f * MAX_CHUNK), 4, 0, 0);
    };
    copy(s.ln.ilo, 0);
    copy(s.ln.ihi, 1);
    copy(s.ln.ic, 2);
    copy(s.ln.delta, 3);
    copy(s.wide_a, 4);
}

// The window fields of a thread's staged (line, pixel) pairs, loaded before
// a chunk is summed and turned into detunings after.
template <int WPX>
struct XFields {
    static constexpr int XPT = (MAX_CHUNK * 8 * WPX + 511) / 512;
    int lo[XPT], hi[XPT], ic[XPT], wide[XPT];
    float dl[XPT];
};

template <int WPX>
__device__ __forceinline__ void load_xfields(const StarDev& s, int l0, int c, int nch, int nc, bool any_wide,
                                             XFields<WPX>& f) {
    constexpr int TPX = 8 * WPX;
#pragma unroll
    for (int u = 0; u < XFields<WPX>::XPT; ++u) {
        const int k = threadIdx.x + u * 512;
        const int l = l0 + c + min(k / TPX, nc - 1) * nch;
        f.lo[u] = s.ln.ilo[l];
        f.hi[u] = s.ln.ihi[l];
        f.ic[u] = s.ln.ic[l];
        f.dl[u] = s.ln.delta[l];
        f.wide[u] = any_wide ? s.wide_a[l] : 0;
    }
}

// A line the pass does not take (WIDE: the lines flagged wide_a; else the
// others) gets kNoLine at every pixel.
template <int WPX, bool WIDE>
__device__ __forceinline__ void write_x_lds(const StarDev& s, int nc, int p0, bool any_wide, const int* fl,
                                            float* dst) {
    constexpr int TPX = 8 * WPX;
#pragma unroll
    for (int u = 0; u < XFields<WPX>::XPT; ++u) {
        const int k = threadIdx.x + u * 512;
        if (k < nc * TPX) {
            const int q = k / TPX, i = p0 + (k - q * TPX);
            const int lo = fl[q], hi = fl[MAX_CHUNK + q], ic = fl[2 * MAX_CHUNK + q];
            const float dl = __int_as_float(fl[3 * MAX_CHUNK + q]);
            const bool wide = any_wide && fl[4 * MAX_CHUNK + q] != 0;
            float x = kNoLine;
            if (wide == WIDE && i >= lo && i <= hi) x = detuning(i - ic, dl, s.h_hi, s.h_lo);
            dst[k] = x;
        }
    }
}

template <int WPX, bool CT, bool WIDE>
__device__ __forceinline__ void write_x(const StarDev& s, int l0, int c, int nch, int nc, int p0, float* dst,
                                        const XFields<WPX>& f) {
    constexpr int TPX = 8 * WPX;
#pragma unroll
    for (int u = 0; u < XFields<WPX>::XPT; ++u) {
        const int k = threadIdx.x + u * 512;
        if (k < nc * TPX) {
            const int q = k / TPX, i = p0 + (k - q * TPX);
            float x = kNoLine;
            if ((f.wide[u] != 0) == WIDE && i >= f.lo[u] && i <= f.hi[u])
                x = detuning(i - f.ic[u], f.dl[u], s.h_hi, s.h_lo);
            // the slack keeps every lane the per-depth test would accept
            if (CT && !(fabsf(x) <= s.xlim[l0 + c + q * nch] * (1.0f + 1e-5f))) x = kNoLine;
            dst[k] = x;
        }
    }
}

// The wing sums of one line over a lane's depth groups d < nfull, all with
// the NP-pair quadrature; CT keeps only the pairs with z2 <= zmax.
template <int NP, bool CT, int DPT, int NDG>
__device__ __forceinline__ void wing_sums(float* acc, const float4* pd, const float* z2, const float* zrow, int dg,
                                          int nfull, const float* T2, const float* W) {
#pragma unroll
    for (int d = 0; d < DPT; ++d)
        if (d < nfull) {
            const bool keep = !CT || z2[d] <= zrow[d * NDG + dg];
            if (CT && !__any(keep)) continue;          // the whole wavefront drops this group
            const float a = fmaf(pd[d].w, wing_S<NP>(pd[d].y, z2[d], T2, W), acc[d]);
            acc[d] = keep ? a : acc[d];
        }
}

// With the centre test (CT) a pixel's detuning is marked kNoLine beyond the
// line's largest span, and a (pixel, depth) lane evaluates only where
// v^2 + a^2 <= zmax of its (line, depth).
// Depth-group slots of a lane: G >= D / NDG full groups (the launch takes
// the smallest instantiation that holds them; fewer slots, fewer registers).
template <int WPX>
constexpr int opacity_max_groups() { return MAXD / (64 / WPX); }

template <int WPX, bool CT, bool WIDE, int G, bool PAIRED, bool FG, class Lds>
__device__ __forceinline__ void opacity_tile_body(const StarDev& s, int tile, int chunk, const Lds& sm) {
    constexpr int NDG = 64 / WPX;
    constexpr int DPT = G;                             // depth-group slots (>= full groups)
    static_assert(G >= 1 && G <= MAXD / NDG, "depth-group slots");
    constexpr int TPX = 8 * WPX;
    const int tid = threadIdx.x;
    const int lane = tid % 64;
    const int wave = tid / 64;
    const int px = wave * WPX + lane % WPX;           // main pixel within the tile
    const int dg = lane / WPX;
    const int D = s.D;
    // FG: every slot holds a full group (D / NDG == G, checked at launch), so
    // the per-group guards below fold away and the groups' sums interleave
    const int nfull = FG ? G : D / NDG, r = D - nfull * NDG;
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

    const int nl = l1 - l0;
    const int nch = (nl + chunk - 1) / chunk;
    // chunk c holds lines c, c + nch, ...: nl / nch of them, one more for c < nl % nch
    const int per_chunk = nch ? nl / nch : 0, extra = nch ? nl - per_chunk * nch : 0;
    auto lines_in = [&](int c) { return per_chunk + (c < extra ? 1 : 0); };
    constexpr bool DB = Lds::NB == 2;                  // double-buffered chunks
    static_assert(!CT || !DB, "the centre test stages one buffer");
    XFields<WPX> f;
    // Sums chunk c from (rows, xs).  DB: first starts the copies of chunk
    // c + 1's rows into nrows; PAIRED, also of chunk c + 2's window fields
    // into fcur, and after the sum chunk c + 1's detunings go to nxs from
    // fnext (its fields, copied during chunk c - 1); else chunk c + 1's
    // fields are loaded into registers first and its detunings written after.
    auto chunk_pass = [&](int c, const float4* __restrict__ rows, const float* __restrict__ xs, float4* __restrict__ nrows, float* __restrict__ nxs, int* fcur,
                          const int* fnext) __attribute__((always_inline)) {
        const int nc = lines_in(c);
        const bool more = DB && c + 1 < nch;
        if (!DB) {                                     // one buffer: stage, then sum
            stage_rows<WPX, CT>(s, l0, c, nch, nc, sm.lp0, sm);
            load_xfields<WPX>(s, l0, c, nch, nc, any_wide, f);
            write_x<WPX, CT, WIDE>(s, l0, c, nch, nc, p0, sm.x0, f);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        } else if (PAIRED) {
            if (more) stage_rows<WPX, CT>(s, l0, c + 1, nch, lines_in(c + 1), nrows, sm);
            if (c + 2 < nch) stage_fields(s, l0, c + 2, nch, lines_in(c + 2), fcur);
        } else if (more) {
            stage_rows<WPX, CT>(s, l0, c + 1, nch, lines_in(c + 1), nrows, sm);
            load_xfields<WPX>(s, l0, c + 1, nch, lines_in(c + 1), any_wide, f);
        }
        for (int q = 0; q < nc; ++q) {
            const float4* row = rows + q * D;
            const float* zrow = CT ? &sm.zmax[q * D] : nullptr;
            const float x = xs[q * TPX + px];
            if (x < 1.0f) {
                float4 pd[DPT];
                float z2[DPT];
                float zmin = 3.0e38f;
#pragma unroll
                for (int d = 0; d < DPT; ++d) {
                    pd[d] = row[d * NDG + dg];         // rows of D: the read past D of the last
                    const float v = x * pd[d].x;       // groups stays inside the buffer, unused
                    z2[d] = fmaf(v, v, pd[d].y);
                    if (d < nfull) zmin = fminf(zmin, z2[d]);
                }
                if (!WIDE && __all(zmin >= PZ_VOIGT_WING_R2)) {
                    // Every lane of every depth group is in the wing: one
                    // wavefront-uniform tier (the most accurate any of them
                    // needs) and straight-line sums.  A line not flagged
                    // wide_a keeps each tier's pair products in range.
                    if (__all(zmin >= PZ_VOIGT_TIER3_R2))
                        wing_sums<1, CT, DPT, NDG>(acc, pd, z2, zrow, dg, nfull, PZ_GH2_T2, PZ_GH2_W);
                    else if (__all(zmin >= PZ_VOIGT_TIER2_R2))
                        wing_sums<2, CT, DPT, NDG>(acc, pd, z2, zrow, dg, nfull, PZ_GH4_T2, PZ_GH4_W);
                    else
                        wing_sums<3, CT, DPT, NDG>(acc, pd, z2, zrow, dg, nfull, PZ_GH6_T2, PZ_GH6_W);
                } else {
#pragma unroll
                    for (int d = 0; d < DPT; ++d) {
                        if (d < nfull) {
                            const float4 p = pd[d];
                            acc[d] = voigt_acc<CT, WIDE>(acc[d], p.y, p.z, p.w, x * p.x, sm.pw,
                                                         CT ? zrow[d * NDG + dg] : 0.0f);
                        }
                    }
                }
            }
            if (tail) {
                const float xt = xs[q * TPX + tpx];
                if (xt < 1.0f) {
                    const float4 p = row[tj];
                    acc_t = voigt_acc<CT, WIDE>(acc_t, p.y, p.z, p.w, xt * p.x, sm.pw, CT ? zrow[tj] : 0.0f);
                }
            }
        }
        if (more) {
            if (PAIRED)
                write_x_lds<WPX, WIDE>(s, lines_in(c + 1), p0, any_wide, fnext, nxs);
            else
                write_x<WPX, CT, WIDE>(s, l0, c + 1, nch, lines_in(c + 1), p0, nxs, f);
        }
        if (DB) __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };
    if (DB) {
        if (nch > 0) {
            stage_rows<WPX, CT>(s, l0, 0, nch, lines_in(0), sm.lp0, sm);
            if (PAIRED && nch > 1) stage_fields(s, l0, 1, nch, lines_in(1), sm.f1);
            load_xfields<WPX>(s, l0, 0, nch, lines_in(0), any_wide, f);
            write_x<WPX, CT, WIDE>(s, l0, 0, nch, lines_in(0), p0, sm.x0, f);
        }
        __builtin_amdgcn_s_waitcnt(0);                // the LDS copies count as loads
        __syncthreads();
        if (PAIRED) {
            // The buffers alternate with a static role in each half of the
            // unrolled pair, so every LDS access names its own array.
            for (int c = 0; c < nch; c += 2) {
                chunk_pass(c, sm.lp0, sm.x0, sm.lp1, sm.x1, sm.f0, sm.f1);
                if (c + 1 < nch) chunk_pass(c + 1, sm.lp1, sm.x1, sm.lp0, sm.x0, sm.f1, sm.f0);
            }
        } else {
            // One loop body, the buffer chosen at run time (fewer registers).
            // The restrict-qualified buffers of chunk_pass tell the compiler
            // that the copies in flight never land in the rows being read.
            for (int c = 0; c < nch; ++c) {
                const bool odd = c & 1;
                chunk_pass(c, odd ? sm.lp1 : sm.lp0, odd ? sm.x1 : sm.x0, odd ? sm.lp0 : sm.lp1,
                           odd ? sm.x0 : sm.x1, nullptr, nullptr);
            }
        }
    } else {
        for (int c = 0; c < nch; ++c) chunk_pass(c, sm.lp0, sm.x0, nullptr, nullptr, nullptr, nullptr);
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
// its own tier.  ANYCT: the workgroup's LDS has the centre test's rows, so
// stars with the centre test are taken too.
// G: depth-group slots, at least the star's D / NDG; FG: exactly D / NDG.
// PAIRED: the plain sum runs its chunks in statically paired buffers (faster
// where the registers allow, as in the single-star kernels; the batch
// kernels, which also hold their work queue's state, take the one-body loop).
template <int WPX, bool WIDE, bool ANYCT, int G, bool PAIRED, bool FG = false>
__device__ __forceinline__ void dev_opacity_tile(const StarDev& s, int tile, int chunk, const OpacityLds<WPX, ANYCT>& sm) {
    if (ANYCT && s.center)
        opacity_tile_body<WPX, ANYCT, WIDE, G, PAIRED, FG>(s, tile, chunk, sm);
    else
        opacity_tile_body<WPX, false, WIDE, G, PAIRED, FG>(s, tile, chunk, sm);
}

}  // namespace pz
