// Plain ("naive") scheme: one launch per half-step over the whole grid, the
// implementation whose per-thread throughput the paper measures in Fig. 1.
//
// Each thread owns one (j, k) column and streams along x, so the x-neighbour
// the stencil needs (H at i-1 for E, E at i+1 for H) is carried in registers
// from the previous iteration; y- and z-neighbours come from the columns of
// adjacent threads through the caches.  Lanes run along z, so every load and
// store of a wavefront is a contiguous 256-byte run.  Algorithmic traffic:
// E half-step 48 B/cell (E in/out, cE, H), H half-step 36 B/cell (H in/out,
// E) -- 84 B per cell update.
#include "fdtd_internal.h"

namespace {

constexpr int kBX = 64;  // threads along z (one wavefront)
constexpr int kBY = 4;   // threads along y

// E half-step (in place): reads H at the backward neighbours (i-1, j-1, k-1).
// LOSSY: E = (ca E + cb d1) - cb d2 with the conductive coefficients (cE is
// then cb); with ca = 1 that is the lossless update bit for bit.
template <bool LOSSY>
__global__ __launch_bounds__(kBX* kBY) void plain_E_kernel(
    float* __restrict__ Ex, float* __restrict__ Ey, float* __restrict__ Ez,
    const float* __restrict__ Hx, const float* __restrict__ Hy, const float* __restrict__ Hz,
    const float* __restrict__ cEx, const float* __restrict__ cEy, const float* __restrict__ cEz,
    const float* __restrict__ cax, const float* __restrict__ cay, const float* __restrict__ caz,
    int nx, int ny, int nz, int xchunk)
{
    const int k = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int i0 = blockIdx.z * xchunk;
    const int i1 = min(nx, i0 + xchunk);
    if (k >= nz || j >= ny || i0 >= nx) return;
    const int km = k == 0 ? nz - 1 : k - 1;
    const int jm = j == 0 ? ny - 1 : j - 1;
    const long long plane = (long long)ny * nz;
    const long long row = (long long)j * nz + k;
    const long long row_jm = (long long)jm * nz + k;
    const long long row_km = (long long)j * nz + km;
    const int im0 = i0 == 0 ? nx - 1 : i0 - 1;
    float hy_im = Hy[im0 * plane + row];
    float hz_im = Hz[im0 * plane + row];
    for (int i = i0; i < i1; ++i) {
        const long long b = (long long)i * plane;
        const long long p = b + row;
        const float hx = Hx[p], hy = Hy[p], hz = Hz[p];
        const float hz_jm = Hz[b + row_jm], hx_jm = Hx[b + row_jm];
        const float hy_km = Hy[b + row_km], hx_km = Hx[b + row_km];
        const float cx = cEx[p], cy = cEy[p], cz = cEz[p];
        float ex = Ex[p], ey = Ey[p], ez = Ez[p];
        if (LOSSY) {
            ex = cax[p] * ex;
            ey = cay[p] * ey;
            ez = caz[p] * ez;
        }
        ex = (ex + cx * (hz - hz_jm)) - cx * (hy - hy_km);
        ey = (ey + cy * (hx - hx_km)) - cy * (hz - hz_im);
        ez = (ez + cz * (hy - hy_im)) - cz * (hx - hx_jm);
        Ex[p] = ex;
        Ey[p] = ey;
        Ez[p] = ez;
        hy_im = hy;
        hz_im = hz;
    }
}

// H half-step (in place): reads the new E at the forward neighbours.
__global__ __launch_bounds__(kBX* kBY) void plain_H_kernel(
    const float* __restrict__ Ex, const float* __restrict__ Ey, const float* __restrict__ Ez,
    float* __restrict__ Hx, float* __restrict__ Hy, float* __restrict__ Hz, float cH, int nx,
    int ny, int nz, int xchunk)
{
    const int k = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int i0 = blockIdx.z * xchunk;
    const int i1 = min(nx, i0 + xchunk);
    if (k >= nz || j >= ny || i0 >= nx) return;
    const int kp = k == nz - 1 ? 0 : k + 1;
    const int jp = j == ny - 1 ? 0 : j + 1;
    const long long plane = (long long)ny * nz;
    const long long row = (long long)j * nz + k;
    const long long row_jp = (long long)jp * nz + k;
    const long long row_kp = (long long)j * nz + kp;
    float ey_c = Ey[i0 * plane + row];
    float ez_c = Ez[i0 * plane + row];
    for (int i = i0; i < i1; ++i) {
        const long long b = (long long)i * plane;
        const long long p = b + row;
        const long long bp = (long long)(i == nx - 1 ? 0 : i + 1) * plane;
        const float ey_ip = Ey[bp + row], ez_ip = Ez[bp + row];
        const float ex = Ex[p];
        const float ez_jp = Ez[b + row_jp], ex_jp = Ex[b + row_jp];
        const float ey_kp = Ey[b + row_kp], ex_kp = Ex[b + row_kp];
        float hx = Hx[p], hy = Hy[p], hz = Hz[p];
        hx = (hx - cH * (ez_jp - ez_c)) + cH * (ey_kp - ey_c);
        hy = (hy - cH * (ex_kp - ex)) + cH * (ez_ip - ez_c);
        hz = (hz - cH * (ey_ip - ey_c)) + cH * (ex_jp - ex);
        Hx[p] = hx;
        Hy[p] = hy;
        Hz[p] = hz;
        ey_c = ey_ip;
        ez_c = ez_ip;
    }
}

void plain_grid(const fdtd_ctx* ctx, dim3* grid, int* xchunk)
{
    const int gx = (ctx->nz + kBX - 1) / kBX;
    const int gy = (ctx->ny + kBY - 1) / kBY;
    // enough blocks to fill 256 CUs several times over, while keeping x runs long
    long long base = (long long)gx * gy;
    long long nchunks = (8192 + base - 1) / base;
    if (nchunks > ctx->nx) nchunks = ctx->nx;
    if (nchunks < 1) nchunks = 1;
    *xchunk = (int)((ctx->nx + nchunks - 1) / nchunks);
    const int gz = (ctx->nx + *xchunk - 1) / *xchunk;
    *grid = dim3(gx, gy, gz);
}

}  // namespace

namespace fdtd {

int plain_step(fdtd_ctx* ctx, int64_t nsteps)
{
    dim3 grid;
    int xchunk;
    plain_grid(ctx, &grid, &xchunk);
    const dim3 block(kBX, kBY);
    for (int64_t n = 0; n < nsteps; ++n) {
        const int64_t s = ctx->step_count;
        PendingTiming t;
        timing_begin(ctx, FDTD_KERNEL_PLAIN_E, &t);
        if (ctx->ca[0])
            hipLaunchKernelGGL(plain_E_kernel<true>, grid, block, 0, ctx->stream, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->coef[0], ctx->coef[1], ctx->coef[2], ctx->ca[0], ctx->ca[1],
                               ctx->ca[2], ctx->nx, ctx->ny, ctx->nz, xchunk);
        else
            hipLaunchKernelGGL(plain_E_kernel<false>, grid, block, 0, ctx->stream, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->coef[0], ctx->coef[1], ctx->coef[2], nullptr, nullptr, nullptr,
                               ctx->nx, ctx->ny, ctx->nz, xchunk);
        timing_end(ctx, &t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(plain E)");
        if (sources_active(ctx, s)) {
            int rc = launch_sources(ctx, s);
            if (rc) return rc;
        }
        timing_begin(ctx, FDTD_KERNEL_PLAIN_H, &t);
        hipLaunchKernelGGL(plain_H_kernel, grid, block, 0, ctx->stream, ctx->field[0], ctx->field[1],
                           ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5], ctx->cH,
                           ctx->nx, ctx->ny, ctx->nz, xchunk);
        timing_end(ctx, &t);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(plain H)");
        ctx->step_count += 1;
    }
    return FDTD_OK;
}

}  // namespace fdtd
