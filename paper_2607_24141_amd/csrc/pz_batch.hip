// Batched synthesis over many stars (placeholder: per-star enqueue).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "pz_internal.h"

namespace pz {
int check_atmos(const pz_plan* plan, const pz_atmos* atm);
int check_params(const pz_params* par);
StarDev make_star(const pz_plan* p, const pz_atmos* atm, const pz_params* par);
}  // namespace pz

struct pz_batch {
    std::vector<pz_star> stars;
};

extern "C" {

int pz_batch_create(int32_t n_star, const pz_star* stars, pz_batch** out) {
    if (!out || (n_star > 0 && !stars) || n_star < 0) return PZ_E_INVALID_ARG;
    *out = nullptr;
    for (int b = 0; b < n_star; ++b) {
        if (!stars[b].plan) return PZ_E_INVALID_ARG;
        int rc = pz::check_atmos(stars[b].plan, &stars[b].atm);
        if (rc) return rc;
        if ((rc = pz::check_params(&stars[b].par))) return rc;
    }
    pz_batch* b = new (std::nothrow) pz_batch();
    if (!b) return PZ_E_NOMEM;
    b->stars.assign(stars, stars + n_star);
    *out = b;
    return PZ_OK;
}

void pz_batch_destroy(pz_batch* batch) { delete batch; }

int synth_forward(const pz_plan*, const pz_atmos*, const pz_params*, float*, float*, pz_stream);
int synth_backward(const pz_plan*, const pz_atmos*, const pz_params*, const float*, const float*, float*, float*,
                   float*, float*, pz_stream);

int synth_batch(const pz_batch* batch, int32_t mode, pz_stream stream) {
    if (!batch) return PZ_E_INVALID_ARG;
    if (mode != PZ_MODE_FWD && mode != PZ_MODE_FWD_BWD) return PZ_E_INVALID_ARG;
    for (const pz_star& s : batch->stars) {
        int rc = synth_forward(s.plan, &s.atm, &s.par, s.F, s.Fc, stream);
        if (rc) return rc;
        if (mode == PZ_MODE_FWD_BWD) {
            rc = synth_backward(s.plan, &s.atm, &s.par, s.dL_dF, nullptr, s.g_loggf, s.g_damp, s.g_abund, s.g_xi,
                                stream);
            if (rc) return rc;
        }
    }
    return PZ_OK;
}

}  // extern "C"
