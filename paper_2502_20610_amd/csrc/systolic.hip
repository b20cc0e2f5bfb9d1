// Systolic scheme (placeholder until the persistent kernel lands).
#include "fdtd_internal.h"

namespace fdtd {

struct SystolicState {};

int systolic_supported(const fdtd_ctx* ctx, std::string* why)
{
    (void)ctx;
    *why = "not implemented yet";
    return 0;
}

int systolic_step(fdtd_ctx* ctx, int64_t nsteps)
{
    (void)nsteps;
    return fail(ctx, FDTD_EUNSUPPORTED, "systolic: not implemented yet");
}

void systolic_release(fdtd_ctx* ctx) { (void)ctx; }

}  // namespace fdtd
