// Plain ("naive") scheme: one launch per half-step over the whole grid, the
// implementation whose per-thread throughput the paper measures in Fig. 1.
//
// Each thread owns one (j, k) column and streams along x, so the x-neighbour
// the stencil needs (H at i-1 for E, E at i+1 for H) is carried in registers
// from the previous iteration; y- and z-neighbours come from the columns of
// adjacent threads through the caches.  Lanes run along z, so every load and
// store of a wavefront is a contiguous 256-byte run.  Algorithmic traffic:
// E half-step 48 B/cell (E in/out, cE, H), H half-step 36 B/cell (H in/out,
// E) -- 84 B per cell update; half of that with FP16 storage.
//
// FP16 storage: every array is IEEE binary16 (field component c holds
// v * 2^-e_c); a kernel converts what it loads to FP32, computes exactly as
// with FP32 storage, and rounds what it stores (round to nearest even).  The
// plain scheme therefore rounds the fields after every half-step.
#include "fdtd_internal.h"

namespace {

constexpr int kBX = 64;  // threads along z (one wavefront)
constexpr int kBY = 4;   // threads along y

// Storage formats: loads return FP32, stores take FP32.
struct Scales {
    float s[6], inv[6];  // field scale 2^e_c and its inverse (FP16 storage)
};
struct F32Store {
    using T = float;
    static __device__ __forceinline__ float ld(const float* p, long long i, float) { return p[i]; }
    static __device__ __forceinline__ float ldc(const float* p, long long i) { return p[i]; }
    static __device__ __forceinline__ void st(float* p, long long i, float v, float) { p[i] = v; }
};
struct F16Store {
    using T = uint16_t;
    static __device__ __forceinline__ float ld(const uint16_t* p, long long i, float s)
    {
        return (float)__builtin_bit_cast(_Float16, p[i]) * s;
    }
    static __device__ __forceinline__ float ldc(const uint16_t* p, long long i)
    {
        return (float)__builtin_bit_cast(_Float16, p[i]);
    }
    static __device__ __forceinline__ void st(uint16_t* p, long long i, float v, float inv)
    {
        // (the empty asm keeps the multiply and the conversion apart: fused
        // into v_fma_mix with a +0 addend they would turn -0 into +0)
        float x = v * inv;
        asm volatile("" : "+v"(x));
        p[i] = __builtin_bit_cast(uint16_t, (_Float16)x);
    }
};

// E half-step (in place): reads H at the backward neighbours (i-1, j-1, k-1).
// LOSSY: E = (ca E + cb d1) - cb d2 with the conductive coefficients (cE is
// then cb); with ca = 1 that is the lossless update bit for bit.
template <bool LOSSY, typename S>
__global__ __launch_bounds__(kBX* kBY) void plain_E_kernel(
    typename S::T* __restrict__ Ex, typename S::T* __restrict__ Ey, typename S::T* __restrict__ Ez,
    const typename S::T* __restrict__ Hx, const typename S::T* __restrict__ Hy,
    const typename S::T* __restrict__ Hz, const typename S::T* __restrict__ cEx,
    const typename S::T* __restrict__ cEy, const typename S::T* __restrict__ cEz,
    const float* __restrict__ cax, const float* __restrict__ cay, const float* __restrict__ caz,
    int nx, int ny, int nz, int xchunk, Scales sc)
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
    float hy_im = S::ld(Hy, im0 * plane + row, sc.s[4]);
    float hz_im = S::ld(Hz, im0 * plane + row, sc.s[5]);
    for (int i = i0; i < i1; ++i) {
        const long long b = (long long)i * plane;
        const long long p = b + row;
        const float hx = S::ld(Hx, p, sc.s[3]), hy = S::ld(Hy, p, sc.s[4]), hz = S::ld(Hz, p, sc.s[5]);
        const float hz_jm = S::ld(Hz, b + row_jm, sc.s[5]), hx_jm = S::ld(Hx, b + row_jm, sc.s[3]);
        const float hy_km = S::ld(Hy, b + row_km, sc.s[4]), hx_km = S::ld(Hx, b + row_km, sc.s[3]);
        const float cx = S::ldc(cEx, p), cy = S::ldc(cEy, p), cz = S::ldc(cEz, p);
        float ex = S::ld(Ex, p, sc.s[0]), ey = S::ld(Ey, p, sc.s[1]), ez = S::ld(Ez, p, sc.s[2]);
        if (LOSSY) {
            ex = cax[p] * ex;
            ey = cay[p] * ey;
            ez = caz[p] * ez;
        }
        ex = (ex + cx * (hz - hz_jm)) - cx * (hy - hy_km);
        ey = (ey + cy * (hx - hx_km)) - cy * (hz - hz_im);
        ez = (ez + cz * (hy - hy_im)) - cz * (hx - hx_jm);
        S::st(Ex, p, ex, sc.inv[0]);
        S::st(Ey, p, ey, sc.inv[1]);
        S::st(Ez, p, ez, sc.inv[2]);
        hy_im = hy;
        hz_im = hz;
    }
}

// H half-step (in place): reads the new E at the forward neighbours.
template <typename S>
__global__ __launch_bounds__(kBX* kBY) void plain_H_kernel(
    const typename S::T* __restrict__ Ex, const typename S::T* __restrict__ Ey,
    const typename S::T* __restrict__ Ez, typename S::T* __restrict__ Hx, typename S::T* __restrict__ Hy,
    typename S::T* __restrict__ Hz, float cH, int nx, int ny, int nz, int xchunk, Scales sc)
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
    float ey_c = S::ld(Ey, i0 * plane + row, sc.s[1]);
    float ez_c = S::ld(Ez, i0 * plane + row, sc.s[2]);
    for (int i = i0; i < i1; ++i) {
        const long long b = (long long)i * plane;
        const long long p = b + row;
        const long long bp = (long long)(i == nx - 1 ? 0 : i + 1) * plane;
        const float ey_ip = S::ld(Ey, bp + row, sc.s[1]), ez_ip = S::ld(Ez, bp + row, sc.s[2]);
        const float ex = S::ld(Ex, p, sc.s[0]);
        const float ez_jp = S::ld(Ez, b + row_jp, sc.s[2]), ex_jp = S::ld(Ex, b + row_jp, sc.s[0]);
        const float ey_kp = S::ld(Ey, b + row_kp, sc.s[1]), ex_kp = S::ld(Ex, b + row_kp, sc.s[0]);
        float hx = S::ld(Hx, p, sc.s[3]), hy = S::ld(Hy, p, sc.s[4]), hz = S::ld(Hz, p, sc.s[5]);
        hx = (hx - cH * (ez_jp - ez_c)) + cH * (ey_kp - ey_c);
        hy = (hy - cH * (ex_kp - ex)) + cH * (ez_ip - ez_c);
        hz = (hz - cH * (ey_ip - ey_c)) + cH * (ex_jp - ex);
        S::st(Hx, p, hx, sc.inv[3]);
        S::st(Hy, p, hy, sc.inv[4]);
        S::st(Hz, p, hz, sc.inv[5]);
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
    Scales sc;
    for (int c = 0; c < 6; ++c) {
        sc.s[c] = ldexpf(1.0f, ctx->fexp[c]);
        sc.inv[c] = ldexpf(1.0f, -ctx->fexp[c]);
    }
    const bool h16 = ctx->storage == FDTD_FP16_STORAGE;
    uint16_t* const* f16 = ctx->field16;
    uint16_t* const* c16 = ctx->coef16;
    for (int64_t n = 0; n < nsteps; ++n) {
        const int64_t s = ctx->step_count;
        PendingTiming t;
        timing_begin(ctx, FDTD_KERNEL_PLAIN_E, &t);
        if (h16)
            hipLaunchKernelGGL((plain_E_kernel<false, F16Store>), grid, block, 0, ctx->stream, f16[0], f16[1],
                               f16[2], f16[3], f16[4], f16[5], c16[0], c16[1], c16[2], nullptr, nullptr,
                               nullptr, ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        else if (ctx->ca[0])
            hipLaunchKernelGGL((plain_E_kernel<true, F32Store>), grid, block, 0, ctx->stream, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->coef[0], ctx->coef[1], ctx->coef[2], ctx->ca[0], ctx->ca[1],
                               ctx->ca[2], ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        else
            hipLaunchKernelGGL((plain_E_kernel<false, F32Store>), grid, block, 0, ctx->stream, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->coef[0], ctx->coef[1], ctx->coef[2], nullptr, nullptr, nullptr,
                               ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        timing_end(ctx, &t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(plain E)");
        if (sources_active(ctx, s)) {
            int rc = launch_sources(ctx, s);
            if (rc) return rc;
        }
        timing_begin(ctx, FDTD_KERNEL_PLAIN_H, &t);
        if (h16)
            hipLaunchKernelGGL(plain_H_kernel<F16Store>, grid, block, 0, ctx->stream, f16[0], f16[1], f16[2],
                               f16[3], f16[4], f16[5], ctx->cH, ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        else
            hipLaunchKernelGGL(plain_H_kernel<F32Store>, grid, block, 0, ctx->stream, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->cH, ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        timing_end(ctx, &t);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(plain H)");
        ctx->step_count += 1;
    }
    return FDTD_OK;
}

}  // namespace fdtd
