// Host interface of the 3D path (periodic boxes): a context of its own behind
// the same C ABI (lelbm_api.hip dispatches to it when lelbm_params.nz > 1).
#pragma once
#include "lelbm_internal.h"

namespace lelbm {

struct Ctx3;
struct Step3Timer {           // event hooks around each kernel of a 3D step (kinds as lelbm_kernel_times)
    void *ctx;
    void (*begin)(void *ctx, int kind, hipStream_t s);
    void (*end)(void *ctx, int kind, hipStream_t s);
};
struct Step3Failure {
    int err, step, detail, species;
    long long node;
    double residual;
};
int ctx3_create(const lelbm_params *p, const Phys &ph, int mixed, const void *moments, int src_fp32, int on_device,
                hipStream_t stream, Ctx3 **out);
int ctx3_step(Ctx3 *c, int nsteps, lelbm_stats *st, const Step3Timer &tm, Step3Failure *fail);
int ctx3_read(const Ctx3 *c, void *out, int to_device);
int ctx3_memory(const Ctx3 *c, long long *persistent, long long *scratch);
void ctx3_set_budget(Ctx3 *c, long long bytes);   // record scratch budget (bytes): bands of tile layers beyond it
void ctx3_destroy(Ctx3 *c);

}  // namespace lelbm
