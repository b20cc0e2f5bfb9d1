// Measured choice of the systolic scheme's tile width and band length.
//
// Section 4 sizes the paper's subdomain block for one GPU's on-chip memory
// and steps per exchange by hand.  Here the candidates are timed on the
// context's own grid: the 15- and 11-cell tile widths along x (lossless
// FP32; conductive grids have only the 11-wide tile, FP16 storage only the
// 15-wide one) and bands of 8 to 64 steps, each run for one call of the
// length the caller will use, from the context's current state, which is
// restored after every run.  The fastest pair becomes the context's options
// and is kept for the process, keyed by everything the choice depends on.
// With FP32 storage, where every scheme computes the same bits, the plain
// two-launch scheme (replayed as a graph) can be timed too: small grids,
// whose state sits in the last-level cache and whose few tiles cannot fill a
// systolic pipeline, run faster on it, and the context then switches to it.
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "fdtd_internal.h"

namespace fdtd {

namespace {

std::mutex g_tune_mu;
// key -> (tile width, band); (0, 0) when the plain scheme won
std::map<std::vector<int64_t>, std::pair<int, int>> g_tuned;

// the plain two-launch scheme takes part: asked for, and FP32 storage (the
// FP16 schemes round at different places, so switching would change results)
bool plain_candidate(const fdtd_ctx* ctx) { return ctx->tune_plain && ctx->storage == FDTD_FP32; }

std::vector<int64_t> tune_key(const fdtd_ctx* ctx, int64_t probe)
{
    return {ctx->nx, ctx->ny, ctx->nz, ctx->cfg.bc[0], ctx->cfg.bc[1], ctx->cfg.bc[2], ctx->storage,
            ctx->ca[0] != nullptr, ctx->use_mat && ctx->nmat > 0, probe, plain_candidate(ctx)};
}

}  // namespace

int autotune_run(fdtd_ctx* ctx, int64_t nsteps, int64_t* out_tile, int64_t* out_band)
{
    if (ctx->scheme != FDTD_SCHEME_SYSTOLIC) return fail(ctx, FDTD_EUNSUPPORTED, "autotune: systolic scheme only");
    if (nsteps < 1) return fail(ctx, FDTD_EINVAL, "autotune: nsteps must be >= 1");
    const int64_t probe = std::min<int64_t>(nsteps, 64);
    const std::vector<int64_t> key = tune_key(ctx, probe);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            if (it->second.first == 0) {
                ctx->scheme = FDTD_SCHEME_PLAIN;
            } else {
                ctx->tile_wx = (int)it->second.first;
                ctx->band_steps = it->second.second;
            }
            if (out_tile) *out_tile = it->second.first;
            if (out_band) *out_band = it->second.second;
            return FDTD_OK;
        }
    }
    const bool h16 = ctx->storage == FDTD_FP16_STORAGE;
    const bool lossy = ctx->ca[0] != nullptr;
    const bool ids = ctx->use_mat && ctx->nmat > 0 && ctx->mat_id;  // (the 19-wide tile needs them)
    std::vector<int> widths;
    if (lossy)
        widths = {11};
    else if (h16)
        widths = ids ? std::vector<int>{15, 19} : std::vector<int>{15};
    else
        widths = ids ? std::vector<int>{15, 11, 19} : std::vector<int>{15, 11};
    std::vector<int> bands;
    for (int K : {8, 12, 16, 24, 32, 48, 64})
        if (K < probe) bands.push_back(K);
    bands.push_back((int)probe);

    // the state every run starts from
    (void)hipSetDevice(ctx->device);
    const size_t es = h16 ? 2 : 4;
    const size_t bytes = (size_t)ctx->ncell * es;
    void* saved = nullptr;
    hipError_t e = hipMalloc(&saved, 6 * bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, "autotune: no room for a copy of the fields");
    }
    auto arr = [&](int c) -> void* { return h16 ? (void*)ctx->field16[c] : (void*)ctx->field[c]; };
    for (int c = 0; c < 6 && e == hipSuccess; ++c)
        e = hipMemcpyAsync((char*)saved + c * bytes, arr(c), bytes, hipMemcpyDeviceToDevice, ctx->stream);
    const int64_t step0 = ctx->step_count;
    const int band0 = ctx->band_steps;
    const int wx0 = ctx->tile_wx;
    auto restore = [&]() {
        hipError_t r = hipSuccess;
        for (int c = 0; c < 6 && r == hipSuccess; ++c)
            r = hipMemcpyAsync(arr(c), (char*)saved + c * bytes, bytes, hipMemcpyDeviceToDevice, ctx->stream);
        ctx->step_count = step0;
        return r;
    };
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    int best_w = widths[0], best_k = bands.back();
    float best_ms = 0.0f;
    bool have = false;
    int rc = FDTD_OK;
    for (size_t wi = 0; wi < widths.size() && e == hipSuccess && !rc; ++wi)
        for (size_t ki = 0; ki < bands.size() && e == hipSuccess && !rc; ++ki) {
            ctx->tile_wx = widths[wi];
            ctx->band_steps = bands[ki];
            float ms = 0.0f;
            // twice: the first run also pays for plan, rings and code loading
            for (int rep = 0; rep < 2 && !rc && e == hipSuccess; ++rep) {
                int r = systolic_prepare(ctx, probe);
                if (r == FDTD_EUNSUPPORTED) break;  // (rings too large, group not resident): not a candidate
                if (r) {
                    rc = r;
                    break;
                }
                if ((e = restore()) != hipSuccess) break;
                if ((e = hipEventRecord(ev[0], ctx->stream)) != hipSuccess) break;
                if ((r = systolic_step(ctx, probe)) != FDTD_OK) {
                    if (r == FDTD_EUNSUPPORTED) break;
                    rc = r;
                    break;
                }
                if ((e = hipEventRecord(ev[1], ctx->stream)) != hipSuccess ||
                    (e = hipEventSynchronize(ev[1])) != hipSuccess ||
                    (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess)
                    break;
                if (rep == 1 && (!have || ms < best_ms)) {
                    have = true;
                    best_ms = ms;
                    best_w = widths[wi];
                    best_k = bands[ki];
                }
            }
            // a device error of the run (e.g. a wait that timed out) ends the search
            if (!rc && e == hipSuccess) {
                int d = device_error(ctx);
                if (d) rc = d;
            }
        }
    // the plain two-launch scheme, timed the same way (twice: the first run
    // also captures its step graph)
    bool plain_wins = false;
    if (plain_candidate(ctx) && have && !rc && e == hipSuccess) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && !rc && e == hipSuccess; ++rep) {
            if ((e = restore()) != hipSuccess) break;
            if ((e = hipEventRecord(ev[0], ctx->stream)) != hipSuccess) break;
            int r = plain_step(ctx, probe);
            if (r) {
                rc = r;
                break;
            }
            if ((e = hipEventRecord(ev[1], ctx->stream)) != hipSuccess || (e = hipEventSynchronize(ev[1])) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess)
                break;
            if (rep == 1 && ms < best_ms) plain_wins = true;
        }
    }
    // back to the state and options the context had
    hipError_t e2 = restore();
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(saved);
    ctx->band_steps = band0;
    ctx->tile_wx = wx0;
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
    if (!have) return fail(ctx, FDTD_EUNSUPPORTED, "autotune: no candidate runs on this grid");
    if (plain_wins) {
        ctx->scheme = FDTD_SCHEME_PLAIN;
        best_w = best_k = 0;
    } else {
        ctx->tile_wx = best_w;
        ctx->band_steps = best_k;
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key] = {best_w, best_k};
    }
    if (out_tile) *out_tile = best_w;
    if (out_band) *out_band = best_k;
    return FDTD_OK;
}

}  // namespace fdtd
