// synth_forward_noalloc: the forward synthesis of synth_forward for callers
// that cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid hipMalloc).  Its per-call workspace (populations,
// Doppler widths, per-line factors, the per-(line, depth) parameters, the line
// opacity, the opacity work-queue counter and, with the centre test, its masks)
// lives in one file-scope device array instead of the plan's workspace.  The
// kernels are the ones synth_forward launches; they receive the array's device
// address through the StarDev workspace pointers.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "pz_internal.h"

namespace pz {
int set_error(int code, const char* msg);
int clear_error();
int check_atmos(const pz_plan* plan, const pz_atmos* atm);
int check_params(const pz_params* par);
StarDev make_star(const pz_plan* p, const pz_atmos* atm, const pz_params* par);
}  // namespace pz

using namespace pz;

namespace {

// Every GPU the library runs on holds this array until the process ends.
static __device__ __align__(256) unsigned char scratch[PZ_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES];   // device address of `scratch` on each device (null: not looked up yet)

// The device address of this device's copy of the array, looked up once per
// device with that device current.  In host code the array's name is only a
// stand-in for the symbol; kernels get this address.
int scratch_on(int dev, unsigned char** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(PZ_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(PZ_E_HIP, "hipGetSymbolAddress of the static scratch failed");
        }
        g_scratch[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return PZ_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" int synth_forward_noalloc(const pz_plan* plan, const pz_atmos* atm, const pz_params* par, float* F,
                                     float* Fc, pz_stream stream) {
    clear_error();
    if (!plan) return set_error(PZ_E_INVALID_ARG, "plan is NULL");
    int rc = check_atmos(plan, atm);
    if (rc) return rc;
    if ((rc = check_params(par))) return rc;
    if (!F || !Fc) return set_error(PZ_E_INVALID_ARG, "F and Fc are required");
    if (atm->sigma_c)
        return set_error(PZ_E_UNSUPPORTED, "synth_forward_noalloc has no scattering transfer (use synth_forward)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(PZ_E_HIP, "hipGetDevice failed");
    if (dev != plan->device) return set_error(PZ_E_INVALID_ARG, "the current device is not the plan's device");

    // workspace layout inside the static array (every piece 256-byte aligned)
    const size_t L = (size_t)plan->L, D = (size_t)plan->D, S = (size_t)plan->S;
    const bool center = plan->center_eta > 0.0;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t o_pop = take(S * 2 * D * 8), o_idv = take(S * D * 8), o_lc = take(L * 32), o_wide = take(L * 4),
                 o_wany = take(4), o_qctr = take(4), o_lp = take(L * D * 16),
                 o_kap = take(D * (size_t)plan->Npad * 4);
    const size_t o_zmax = center ? take(L * D * 4) : 0, o_xlim = center ? take(L * 4) : 0,
                 o_ikc = center ? take(L * 8) : 0;
    if (off > PZ_NOALLOC_SCRATCH_BYTES) {
        char msg[200];
        snprintf(msg, sizeof msg, "plan needs %zu bytes of scratch; synth_forward_noalloc holds at most %zu",
                 off, (size_t)PZ_NOALLOC_SCRATCH_BYTES);
        return set_error(PZ_E_SHAPE, msg);
    }
    unsigned char* base = nullptr;
    if ((rc = scratch_on(dev, &base))) return rc;

    StarDev s = make_star(plan, atm, par);
    s.F = F;
    s.Fc = Fc;
    s.pop = reinterpret_cast<double*>(base + o_pop);
    s.inv_dv = reinterpret_cast<double*>(base + o_idv);
    s.lc = reinterpret_cast<double4*>(base + o_lc);
    s.wide_a = reinterpret_cast<int*>(base + o_wide);
    s.wide_any = reinterpret_cast<int*>(base + o_wany);
    s.qctr = reinterpret_cast<int*>(base + o_qctr);
    s.lp = reinterpret_cast<float4*>(base + o_lp);
    s.kappa = reinterpret_cast<float*>(base + o_kap);
    s.zmax = center ? reinterpret_cast<float*>(base + o_zmax) : nullptr;
    s.xlim = center ? reinterpret_cast<float*>(base + o_xlim) : nullptr;
    s.inv_kcl = center ? reinterpret_cast<double*>(base + o_ikc) : nullptr;
    // the backward-only workspaces stay out of reach
    s.gk = nullptr;
    s.gline = nullptr;
    s.partial = nullptr;
    s.sc = nullptr;
    s.sc_iters = nullptr;

    // Every stage writes its part of the workspace before any stage reads it
    // (the queue counter and the wide-line flag are reset by kernels), so the
    // contents a previous call left behind are never read.
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_populations(s, st);
    if (e == hipSuccess) e = launch_line_params(s, st);
    if (e == hipSuccess) e = launch_opacity(s, plan->chunk, st);
    if (e == hipSuccess) e = launch_flux(s, st);
    if (e != hipSuccess) return set_error(PZ_E_HIP, hipGetErrorString(e));
    return PZ_OK;
}
