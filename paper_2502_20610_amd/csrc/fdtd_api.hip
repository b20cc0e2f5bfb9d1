// Host runtime of libfdtd.so: context lifetime, validation, allocation, the
// coefficient build, sources, field I/O, timing and dispatch to a scheme.
// The public contract is include/fdtd.h.
#include <math.h>
#include <string.h>

#include <new>
#include <string>

#include "fdtd_internal.h"

using namespace fdtd;

namespace {

thread_local std::string g_create_error = "no error";

constexpr int kThreads = 256;

// binary16 <-> FP32 (round to nearest even; the scales are powers of two,
// so scaling is exact and the conversion rounds once).  The empty asm keeps
// the conversion a plain v_cvt_f16_f32: otherwise a preceding multiply is
// folded into v_fma_mix with a +0 addend, which turns a -0 product into +0.
__device__ __forceinline__ uint16_t to_h(float v)
{
    asm volatile("" : "+v"(v));
    return __builtin_bit_cast(uint16_t, (_Float16)v);
}
__device__ __forceinline__ float from_h(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// cE_c = (float)(dt / ((double)eps * dx)), zero on the index-0 plane of every
// PEC axis tangential to component `comp` (bc[a] == 0 means PEC).  The
// division is IEEE double, so the rounded result is the same on any
// conforming machine.  With out16 the FP32 value is stored rounded to
// binary16 instead.  Bad permittivity (< 1 or not finite) sets bit 0 of *err.
__global__ void build_coef_kernel(const float* __restrict__ eps, float* __restrict__ out,
                                  uint16_t* __restrict__ out16, int comp, int nx, int ny, int nz,
                                  int bcx, int bcy, int bcz, double dt, double dx, int* err)
{
    const long long n = (long long)nx * ny * nz;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        int k = (int)(p % nz);
        long long r = p / nz;
        int j = (int)(r % ny);
        int i = (int)(r / ny);
        float e = eps[p];
        if (!(e >= 1.0f) || !(e <= 3.0e38f)) atomicOr(err, 1);
        double c = dt / ((double)e * dx);
        if ((comp != 0 && bcx == FDTD_BC_PEC && i == 0) || (comp != 1 && bcy == FDTD_BC_PEC && j == 0) ||
            (comp != 2 && bcz == FDTD_BC_PEC && k == 0))
            c = 0.0;
        if (out16)
            out16[p] = to_h((float)c);
        else
            out[p] = (float)c;
    }
}

// FP16 storage: dst = binary16(src * inv), and back, src * scale.
__global__ void to_f16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, long long n,
                              float inv)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x)
        dst[p] = to_h(src[p] * inv);
}

__global__ void from_f16_kernel(const uint16_t* __restrict__ src, float* __restrict__ dst, long long n,
                                float scale)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x)
        dst[p] = from_h(src[p]) * scale;
}

// Re-encode binary16 values under a new scale: h * old * inv_new.
__global__ void rescale_f16_kernel(uint16_t* __restrict__ a, long long n, float old_scale, float inv_new)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x)
        a[p] = to_h((from_h(a[p]) * old_scale) * inv_new);
}

// Conductive coefficients of component `comp`, in IEEE double like cE:
// h = sigma dt / (2 eps), ca = (1 - h) / (1 + h), cb = (dt / (eps dx)) / (1 + h);
// on PEC-tangential index-0 entries ca = 1, cb = 0.  Bad permittivity or
// conductivity (eps < 1, sigma < 0, not finite) sets bit 0 of *err.
__global__ void build_lossy_kernel(const float* __restrict__ eps, const float* __restrict__ sig,
                                   float* __restrict__ ca, float* __restrict__ cb, int comp, int nx,
                                   int ny, int nz, int bcx, int bcy, int bcz, double dt, double dx,
                                   int* err)
{
    const long long n = (long long)nx * ny * nz;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        int k = (int)(p % nz);
        long long r = p / nz;
        int j = (int)(r % ny);
        int i = (int)(r / ny);
        float ef = eps[p], sf = sig[p];
        if (!(ef >= 1.0f) || !(ef <= 3.0e38f) || !(sf >= 0.0f) || !(sf <= 3.0e38f)) atomicOr(err, 1);
        const double e = (double)ef;
        const double h = (double)sf * dt / (2.0 * e);
        double a = (1.0 - h) / (1.0 + h);
        double b = (dt / (e * dx)) / (1.0 + h);
        if ((comp != 0 && bcx == FDTD_BC_PEC && i == 0) || (comp != 1 && bcy == FDTD_BC_PEC && j == 0) ||
            (comp != 2 && bcz == FDTD_BC_PEC && k == 0)) {
            a = 1.0;
            b = 0.0;
        }
        ca[p] = (float)a;
        cb[p] = (float)b;
    }
}

// Force the PEC-tangential entries of E component `comp` to +0 (all-zero
// bits in both storage formats).
template <typename T>
__global__ void zero_pec_kernel(T* __restrict__ f, int comp, int nx, int ny, int nz, int bcx,
                                int bcy, int bcz)
{
    // three planes at most; one thread per element of the largest plane
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    // plane normal to x (i = 0): ny*nz entries
    if (comp != 0 && bcx == FDTD_BC_PEC && t < (long long)ny * nz) f[t] = T(0);
    // plane normal to y (j = 0): nx*nz entries
    if (comp != 1 && bcy == FDTD_BC_PEC && t < (long long)nx * nz) {
        long long i = t / nz, k = t % nz;
        f[(i * ny) * nz + k] = T(0);
    }
    // plane normal to z (k = 0): nx*ny entries
    if (comp != 2 && bcz == FDTD_BC_PEC && t < (long long)nx * ny) f[t * nz] = T(0);
}

// With stepp (a step loop replayed as a graph) the step is read from *stepp,
// which the kernel then advances; otherwise it is s.
__global__ void sources_kernel(float* Ex, float* Ey, float* Ez, const DevSource* __restrict__ src,
                               int nsrc, long long s, int ny, int nz, long long* stepp)
{
    // One thread; sources are applied in table order (several sources on one
    // cell add up in the same order as in any other scheme).
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (stepp) {
        s = *stepp;
        *stepp = s + 1;
    }
    for (int q = 0; q < nsrc; ++q) {
        long long m = s - src[q].first;
        if (m < 0 || m >= src[q].len) continue;
        float* f = src[q].comp == 0 ? Ex : (src[q].comp == 1 ? Ey : Ez);
        long long p = ((long long)src[q].i * ny + src[q].j) * nz + src[q].k;
        f[p] = f[p] + src[q].wave[m];
    }
}

// FP16 storage: the source cell is read, the sample added in FP32 and the
// sum stored rounded again.
__global__ void sources_f16_kernel(uint16_t* Ex, uint16_t* Ey, uint16_t* Ez, const DevSource* __restrict__ src,
                                   int nsrc, long long s, int ny, int nz, float sx, float sy, float sz,
                                   float ix, float iy, float iz, long long* stepp)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (stepp) {
        s = *stepp;
        *stepp = s + 1;
    }
    for (int q = 0; q < nsrc; ++q) {
        long long m = s - src[q].first;
        if (m < 0 || m >= src[q].len) continue;
        const int c = src[q].comp;
        uint16_t* f = c == 0 ? Ex : (c == 1 ? Ey : Ez);
        const float sc = c == 0 ? sx : (c == 1 ? sy : sz), inv = c == 0 ? ix : (c == 1 ? iy : iz);
        long long p = ((long long)src[q].i * ny + src[q].j) * nz + src[q].k;
        f[p] = to_h((from_h(f[p]) * sc + src[q].wave[m]) * inv);
    }
}

bool ok_ptr(const void* p) { return p != nullptr; }

int check_live(fdtd_ctx* ctx)
{
    if (!ctx) return FDTD_EINVAL;
    if (ctx->poisoned) {
        return FDTD_ESTATE;
    }
    return FDTD_OK;
}

hipMemcpyKind kind_from(int where, bool to_device)
{
    if (where == FDTD_DEVICE) return hipMemcpyDeviceToDevice;
    return to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
}

int collect_timings(fdtd_ctx* ctx)
{
    for (auto& t : ctx->pending) {
        hipError_t e = hipEventSynchronize(t.stop);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
        ctx->launches[t.kernel] += 1;
        ctx->total_ms[t.kernel] += ms;
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    ctx->pending.clear();
    return FDTD_OK;
}

int check_device_error(fdtd_ctx* ctx)
{
    int h = 0;
    hipError_t e = hipMemcpy(&h, ctx->dev_error, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(error word)");
    if (h & 2) {
        ctx->poisoned = true;
        return fail(ctx, FDTD_ETIMEOUT,
                    "systolic kernel: a neighbour-flag wait exceeded the spin limit");
    }
    if (h & 1) {
        int z = 0;
        (void)hipMemcpy(ctx->dev_error, &z, sizeof(int), hipMemcpyHostToDevice);
        return fail(ctx, FDTD_EINVAL,
                    "set_materials: permittivity < 1, conductivity < 0, or not finite (device input)");
    }
    return FDTD_OK;
}

int rebuild_dev_sources(fdtd_ctx* ctx)
{
    if (ctx->dev_sources) {
        (void)hipFree(ctx->dev_sources);
        ctx->dev_sources = nullptr;
    }
    ctx->dev_sources_n = (int)ctx->sources.size();
    if (ctx->sources.empty()) return FDTD_OK;
    std::vector<DevSource> h(ctx->sources.size());
    for (size_t q = 0; q < ctx->sources.size(); ++q) {
        const SourceRec& s = ctx->sources[q];
        h[q] = DevSource{s.comp, s.i, s.j, s.k, (long long)s.len, (long long)s.first, s.wave};
    }
    hipError_t e = hipMalloc(&ctx->dev_sources, h.size() * sizeof(DevSource));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(sources)");
    e = hipMemcpyAsync(ctx->dev_sources, h.data(), h.size() * sizeof(DevSource),
                       hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(sources)");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    return FDTD_OK;
}

int grid_for(long long n)
{
    long long g = (n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

namespace fdtd {

int device_error(fdtd_ctx* ctx) { return check_device_error(ctx); }

int fail(fdtd_ctx* ctx, int code, const std::string& msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_create_error = msg;
    return code;
}

int hip_fail(fdtd_ctx* ctx, hipError_t e, const char* what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (ctx) ctx->poisoned = true;
    return fail(ctx, FDTD_EHIP, msg);
}

void timing_begin(fdtd_ctx* ctx, int kernel, PendingTiming* t)
{
    t->kernel = -1;
    if (!ctx->profile) return;
    if (hipEventCreate(&t->start) != hipSuccess) return;
    if (hipEventCreate(&t->stop) != hipSuccess) {
        (void)hipEventDestroy(t->start);
        return;
    }
    t->kernel = kernel;
    (void)hipEventRecord(t->start, ctx->stream);
}

void timing_end(fdtd_ctx* ctx, PendingTiming* t)
{
    if (t->kernel < 0) return;
    (void)hipEventRecord(t->stop, ctx->stream);
    ctx->pending.push_back(*t);
}

bool sources_active(const fdtd_ctx* ctx, int64_t s)
{
    for (const auto& q : ctx->sources)
        if (s - q.first >= 0 && s - q.first < q.len) return true;
    return false;
}

int launch_sources(fdtd_ctx* ctx, int64_t s, hipStream_t st, long long* stepp)
{
    PendingTiming t;
    if (!stepp) timing_begin(ctx, FDTD_KERNEL_SOURCES, &t);
    if (ctx->storage == FDTD_FP16_STORAGE)
        hipLaunchKernelGGL(sources_f16_kernel, dim3(1), dim3(64), 0, st, ctx->field16[0],
                           ctx->field16[1], ctx->field16[2], ctx->dev_sources, ctx->dev_sources_n,
                           (long long)s, ctx->ny, ctx->nz, ldexpf(1.0f, ctx->fexp[0]), ldexpf(1.0f, ctx->fexp[1]),
                           ldexpf(1.0f, ctx->fexp[2]), ldexpf(1.0f, -ctx->fexp[0]), ldexpf(1.0f, -ctx->fexp[1]),
                           ldexpf(1.0f, -ctx->fexp[2]), stepp);
    else
        hipLaunchKernelGGL(sources_kernel, dim3(1), dim3(64), 0, st, ctx->field[0],
                           ctx->field[1], ctx->field[2], ctx->dev_sources, ctx->dev_sources_n,
                           (long long)s, ctx->ny, ctx->nz, stepp);
    if (!stepp) timing_end(ctx, &t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "launch(sources)");
    return FDTD_OK;
}

}  // namespace fdtd

extern "C" {

int fdtd_create(const fdtd_config* cfg, fdtd_ctx** out)
{
    if (!out) return fail(nullptr, FDTD_EINVAL, "fdtd_create: out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, FDTD_EINVAL, "fdtd_create: cfg is NULL");
    if (cfg->struct_size != sizeof(fdtd_config))
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: struct_size != sizeof(fdtd_config)");
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: every dimension must be >= 1");
    const int64_t ncell = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    if (ncell > (int64_t(1) << 30))
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: nx*ny*nz must be <= 2^30");
    if (!(cfg->dt > 0.0) || !(cfg->dx > 0.0) || !isfinite(cfg->dt) || !isfinite(cfg->dx))
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: dt and dx must be finite and > 0");
    if (!(cfg->dt * sqrt(3.0) < cfg->dx))
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: Courant condition dt*sqrt(3) < dx violated");
    for (int a = 0; a < 3; ++a)
        if (cfg->bc[a] != FDTD_BC_PEC && cfg->bc[a] != FDTD_BC_PERIODIC)
            return fail(nullptr, FDTD_EINVAL, "fdtd_create: bc must be FDTD_BC_PEC or FDTD_BC_PERIODIC");
    if (cfg->scheme != FDTD_SCHEME_PLAIN && cfg->scheme != FDTD_SCHEME_SYSTOLIC &&
        cfg->scheme != FDTD_SCHEME_PLAIN_FUSED)
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: unknown scheme");
    if (cfg->storage != FDTD_FP32 && cfg->storage != FDTD_FP16_STORAGE)
        return fail(nullptr, FDTD_EINVAL, "fdtd_create: unknown storage");
    if (cfg->device < 0) return fail(nullptr, FDTD_EINVAL, "fdtd_create: device must be >= 0");

    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return fail(nullptr, FDTD_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    // the device address of the allocation-free entry point's scratch, once
    // per device (this device is current)
    if (invariants_scratch_init(cfg->device) != FDTD_OK)
        return fail(nullptr, FDTD_EHIP, "fdtd_create: hipGetSymbolAddress of the invariants scratch failed");

    fdtd_ctx* ctx = new (std::nothrow) fdtd_ctx();
    if (!ctx) return fail(nullptr, FDTD_ENOMEM, "fdtd_create: host allocation failed");
    ctx->cfg = *cfg;
    ctx->nx = cfg->nx;
    ctx->ny = cfg->ny;
    ctx->nz = cfg->nz;
    ctx->ncell = ncell;
    ctx->device = cfg->device;
    ctx->scheme = cfg->scheme;
    ctx->storage = cfg->storage;
    ctx->band_steps = 0;  // 0 = choose per call
    ctx->workgroups = 0;
    ctx->spin_limit = int64_t(1) << 22;
    ctx->profile = false;
    ctx->use_mat = true;
    ctx->use_graphs = true;
    ctx->cH = (float)(cfg->dt / cfg->dx);
    ctx->err = "no error";

    auto bail = [&](int code) {
        fdtd_destroy(ctx);
        return code;
    };
    if (cfg->stream) {
        ctx->stream = (hipStream_t)cfg->stream;
        ctx->own_stream = false;
    } else {
        e = hipStreamCreate(&ctx->stream);
        if (e != hipSuccess) {
            fail(nullptr, FDTD_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
            delete ctx;
            return FDTD_EHIP;
        }
        ctx->own_stream = true;
    }
    const bool h16 = cfg->storage == FDTD_FP16_STORAGE;
    const size_t bytes = (size_t)ncell * sizeof(float);
    const size_t sbytes = (size_t)ncell * (h16 ? sizeof(uint16_t) : sizeof(float));  // stored arrays
    for (int c = 0; c < 6; ++c) {
        void* p = nullptr;
        e = hipMalloc(&p, sbytes);
        if (e != hipSuccess) {
            fail(nullptr, FDTD_ENOMEM, std::string("hipMalloc(field): ") + hipGetErrorString(e));
            return bail(FDTD_ENOMEM);
        }
        if (h16)
            ctx->field16[c] = (uint16_t*)p;
        else
            ctx->field[c] = (float*)p;
        e = hipMemsetAsync(p, 0, sbytes, ctx->stream);
        if (e != hipSuccess) {
            fail(nullptr, FDTD_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
            return bail(FDTD_EHIP);
        }
    }
    for (int c = 0; c < 3; ++c) {
        void* p = nullptr;
        e = hipMalloc(&p, sbytes);
        if (e != hipSuccess) {
            fail(nullptr, FDTD_ENOMEM, std::string("hipMalloc(coef): ") + hipGetErrorString(e));
            return bail(FDTD_ENOMEM);
        }
        if (h16)
            ctx->coef16[c] = (uint16_t*)p;
        else
            ctx->coef[c] = (float*)p;
    }
    e = hipMalloc(&ctx->dev_error, sizeof(int));
    if (e != hipSuccess) {
        fail(nullptr, FDTD_ENOMEM, std::string("hipMalloc(error): ") + hipGetErrorString(e));
        return bail(FDTD_ENOMEM);
    }
    e = hipMemsetAsync(ctx->dev_error, 0, sizeof(int), ctx->stream);
    if (e != hipSuccess) {
        fail(nullptr, FDTD_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
        return bail(FDTD_EHIP);
    }
    // eps = 1 everywhere: build the coefficients from a device array of ones
    float* ones = nullptr;
    e = hipMalloc(&ones, bytes);
    if (e != hipSuccess) {
        fail(nullptr, FDTD_ENOMEM, std::string("hipMalloc(eps): ") + hipGetErrorString(e));
        return bail(FDTD_ENOMEM);
    }
    // fill with 1.0f: 0x3f800000
    e = hipMemsetD32Async((hipDeviceptr_t)ones, 0x3f800000, (size_t)ncell, ctx->stream);
    if (e == hipSuccess) {
        for (int c = 0; c < 3 && e == hipSuccess; ++c) {
            hipLaunchKernelGGL(build_coef_kernel, dim3(grid_for(ncell)), dim3(kThreads), 0, ctx->stream,
                               ones, ctx->coef[c], ctx->coef16[c], c, ctx->nx, ctx->ny, ctx->nz,
                               cfg->bc[0], cfg->bc[1], cfg->bc[2], cfg->dt, cfg->dx, ctx->dev_error);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(ones);
    if (e != hipSuccess) {
        fail(nullptr, FDTD_EHIP, std::string("fdtd_create init: ") + hipGetErrorString(e));
        return bail(FDTD_EHIP);
    }
    if (build_material_ids(ctx) != FDTD_OK) {
        fail(nullptr, FDTD_EHIP, "fdtd_create init: " + ctx->err);
        return bail(FDTD_EHIP);
    }
    *out = ctx;
    return FDTD_OK;
}

int fdtd_destroy(fdtd_ctx* ctx)
{
    if (!ctx) return FDTD_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto& t : ctx->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    ctx->pending.clear();
    systolic_release(ctx);
    release_material_ids(ctx);
    release_step_graph(ctx);
    for (int c = 0; c < 6; ++c) {
        if (ctx->field[c]) (void)hipFree(ctx->field[c]);
        if (ctx->field16[c]) (void)hipFree(ctx->field16[c]);
        if (ctx->alt[c]) (void)hipFree(ctx->alt[c]);
    }
    for (int c = 0; c < 3; ++c) {
        if (ctx->coef[c]) (void)hipFree(ctx->coef[c]);
        if (ctx->coef16[c]) (void)hipFree(ctx->coef16[c]);
        if (ctx->ca[c]) (void)hipFree(ctx->ca[c]);
    }
    for (auto& s : ctx->sources)
        if (s.wave) (void)hipFree(s.wave);
    if (ctx->dev_sources) (void)hipFree(ctx->dev_sources);
    if (ctx->dev_error) (void)hipFree(ctx->dev_error);
    if (ctx->inv_scratch) (void)hipFree(ctx->inv_scratch);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return FDTD_OK;
}

int fdtd_set_materials(fdtd_ctx* ctx, const float* eps_x, const float* eps_y, const float* eps_z,
                       int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (where != FDTD_HOST && where != FDTD_DEVICE) return fail(ctx, FDTD_EINVAL, "bad `where`");
    const float* eps[3] = {eps_x, eps_y, eps_z};
    for (int c = 0; c < 3; ++c)
        if (!ok_ptr(eps[c])) return fail(ctx, FDTD_EINVAL, "set_materials: NULL array");
    if (where == FDTD_HOST) {
        for (int c = 0; c < 3; ++c)
            for (int64_t p = 0; p < ctx->ncell; ++p) {
                float v = eps[c][p];
                if (!(v >= 1.0f) || !(v <= 3.0e38f))
                    return fail(ctx, FDTD_EINVAL, "set_materials: permittivity < 1 or not finite");
            }
    }
    (void)hipSetDevice(ctx->device);
    const size_t bytes = (size_t)ctx->ncell * sizeof(float);
    float* stage = nullptr;
    if (where == FDTD_HOST) {
        hipError_t e = hipMalloc(&stage, bytes);
        if (e != hipSuccess) return fail(ctx, FDTD_ENOMEM, "set_materials: staging allocation failed");
    }
    hipError_t e = hipSuccess;
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        const float* src = eps[c];
        if (where == FDTD_HOST) {
            e = hipMemcpyAsync(stage, eps[c], bytes, hipMemcpyHostToDevice, ctx->stream);
            src = stage;
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(build_coef_kernel, dim3(grid_for(ctx->ncell)), dim3(kThreads), 0,
                               ctx->stream, src, ctx->coef[c], ctx->coef16[c], c, ctx->nx, ctx->ny,
                               ctx->nz, ctx->cfg.bc[0], ctx->cfg.bc[1], ctx->cfg.bc[2], ctx->cfg.dt,
                               ctx->cfg.dx, ctx->dev_error);
            e = hipGetLastError();
        }
        if (e == hipSuccess && where == FDTD_HOST) e = hipStreamSynchronize(ctx->stream);
    }
    if (stage) {
        hipError_t e2 = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) e = e2;
        (void)hipFree(stage);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "set_materials");
    // lossless from now on
    for (int c = 0; c < 3; ++c) {
        if (ctx->ca[c]) (void)hipFree(ctx->ca[c]);
        ctx->ca[c] = nullptr;
    }
    return build_material_ids(ctx);
}

int fdtd_set_lossy_materials(fdtd_ctx* ctx, const float* eps_x, const float* eps_y,
                             const float* eps_z, const float* sigma_x, const float* sigma_y,
                             const float* sigma_z, int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (where != FDTD_HOST && where != FDTD_DEVICE) return fail(ctx, FDTD_EINVAL, "bad `where`");
    const float* eps[3] = {eps_x, eps_y, eps_z};
    const float* sig[3] = {sigma_x, sigma_y, sigma_z};
    for (int c = 0; c < 3; ++c)
        if (!ok_ptr(eps[c]) || !ok_ptr(sig[c])) return fail(ctx, FDTD_EINVAL, "set_lossy_materials: NULL array");
    if (ctx->storage == FDTD_FP16_STORAGE)
        return fail(ctx, FDTD_EUNSUPPORTED, "set_lossy_materials: conductivity needs FP32 storage");
    if (where == FDTD_HOST) {
        for (int c = 0; c < 3; ++c)
            for (int64_t p = 0; p < ctx->ncell; ++p) {
                float v = eps[c][p], g = sig[c][p];
                if (!(v >= 1.0f) || !(v <= 3.0e38f) || !(g >= 0.0f) || !(g <= 3.0e38f))
                    return fail(ctx, FDTD_EINVAL,
                                "set_lossy_materials: permittivity < 1, conductivity < 0, or not finite");
            }
    }
    (void)hipSetDevice(ctx->device);
    const size_t bytes = (size_t)ctx->ncell * sizeof(float);
    hipError_t e = hipSuccess;
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
        if (!ctx->ca[c]) e = hipMalloc(&ctx->ca[c], bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, "set_lossy_materials: allocation failed");
    }
    float* stage = nullptr;
    if (where == FDTD_HOST && (e = hipMalloc(&stage, 2 * bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, "set_lossy_materials: staging allocation failed");
    }
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        const float* se = eps[c];
        const float* ss = sig[c];
        if (where == FDTD_HOST) {
            e = hipMemcpyAsync(stage, eps[c], bytes, hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(stage + ctx->ncell, sig[c], bytes, hipMemcpyHostToDevice, ctx->stream);
            se = stage;
            ss = stage + ctx->ncell;
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(build_lossy_kernel, dim3(grid_for(ctx->ncell)), dim3(kThreads), 0,
                               ctx->stream, se, ss, ctx->ca[c], ctx->coef[c], c, ctx->nx, ctx->ny,
                               ctx->nz, ctx->cfg.bc[0], ctx->cfg.bc[1], ctx->cfg.bc[2], ctx->cfg.dt,
                               ctx->cfg.dx, ctx->dev_error);
            e = hipGetLastError();
        }
        if (e == hipSuccess && where == FDTD_HOST) e = hipStreamSynchronize(ctx->stream);
    }
    if (stage) {
        hipError_t e2 = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) e = e2;
        (void)hipFree(stage);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "set_lossy_materials");
    release_material_ids(ctx);  // the conductive update reads its per-cell arrays
    return FDTD_OK;
}

int fdtd_set_fields(fdtd_ctx* ctx, uint32_t comp_mask, const float* const src[6], int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (where != FDTD_HOST && where != FDTD_DEVICE) return fail(ctx, FDTD_EINVAL, "bad `where`");
    if (comp_mask & ~0x3Fu) return fail(ctx, FDTD_EINVAL, "set_fields: comp_mask has bits above 5");
    if (comp_mask && !src) return fail(ctx, FDTD_EINVAL, "set_fields: src is NULL");
    for (int c = 0; c < 6; ++c)
        if ((comp_mask >> c & 1u) && !src[c]) return fail(ctx, FDTD_EINVAL, "set_fields: NULL array");
    (void)hipSetDevice(ctx->device);
    const size_t bytes = (size_t)ctx->ncell * sizeof(float);
    const bool h16 = ctx->storage == FDTD_FP16_STORAGE;
    float* stage = nullptr;
    hipError_t e = hipSuccess;
    if (h16 && where == FDTD_HOST && comp_mask && (e = hipMalloc(&stage, bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, "set_fields: staging allocation failed");
    }
    for (int c = 0; c < 6 && e == hipSuccess; ++c) {
        if (!(comp_mask >> c & 1u)) continue;
        if (h16) {
            // FP16 storage: the input rounded once under the component's scale
            const float* in = src[c];
            if (where == FDTD_HOST) {
                e = hipMemcpyAsync(stage, src[c], bytes, hipMemcpyHostToDevice, ctx->stream);
                in = stage;
            }
            if (e == hipSuccess) {
                hipLaunchKernelGGL(to_f16_kernel, dim3(grid_for(ctx->ncell)), dim3(kThreads), 0, ctx->stream,
                                   in, ctx->field16[c], (long long)ctx->ncell, ldexpf(1.0f, -ctx->fexp[c]));
                e = hipGetLastError();
            }
        } else {
            e = hipMemcpyAsync(ctx->field[c], src[c], bytes, kind_from(where, true), ctx->stream);
        }
        if (e == hipSuccess && c < 3) {
            long long m = (long long)ctx->ny * ctx->nz;
            m = m > (long long)ctx->nx * ctx->nz ? m : (long long)ctx->nx * ctx->nz;
            m = m > (long long)ctx->nx * ctx->ny ? m : (long long)ctx->nx * ctx->ny;
            const dim3 g((unsigned)((m + kThreads - 1) / kThreads));
            if (h16)
                hipLaunchKernelGGL(zero_pec_kernel<uint16_t>, g, dim3(kThreads), 0, ctx->stream, ctx->field16[c],
                                   c, ctx->nx, ctx->ny, ctx->nz, ctx->cfg.bc[0], ctx->cfg.bc[1], ctx->cfg.bc[2]);
            else
                hipLaunchKernelGGL(zero_pec_kernel<float>, g, dim3(kThreads), 0, ctx->stream, ctx->field[c], c,
                                   ctx->nx, ctx->ny, ctx->nz, ctx->cfg.bc[0], ctx->cfg.bc[1], ctx->cfg.bc[2]);
            e = hipGetLastError();
        }
        // the staging buffer is reused by the next component
        if (e == hipSuccess && stage) e = hipStreamSynchronize(ctx->stream);
    }
    if (e == hipSuccess && where == FDTD_HOST) e = hipStreamSynchronize(ctx->stream);
    if (stage) (void)hipFree(stage);
    if (e != hipSuccess) return hip_fail(ctx, e, "set_fields");
    return FDTD_OK;
}

int fdtd_set_field_scale(fdtd_ctx* ctx, const int32_t exp2[6])
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (!exp2) return fail(ctx, FDTD_EINVAL, "set_field_scale: exp2 is NULL");
    if (ctx->storage != FDTD_FP16_STORAGE)
        return fail(ctx, FDTD_EINVAL, "set_field_scale: scales apply to FP16 storage only");
    for (int c = 0; c < 6; ++c)
        if (exp2[c] < -30 || exp2[c] > 30) return fail(ctx, FDTD_EINVAL, "set_field_scale: exponent out of [-30, 30]");
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipSuccess;
    for (int c = 0; c < 6 && e == hipSuccess; ++c) {
        if (exp2[c] == ctx->fexp[c]) continue;
        hipLaunchKernelGGL(rescale_f16_kernel, dim3(grid_for(ctx->ncell)), dim3(kThreads), 0, ctx->stream,
                           ctx->field16[c], (long long)ctx->ncell, ldexpf(1.0f, ctx->fexp[c]),
                           ldexpf(1.0f, -exp2[c]));
        e = hipGetLastError();
        ctx->fexp[c] = exp2[c];
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "set_field_scale");
    return FDTD_OK;
}

int fdtd_add_source(fdtd_ctx* ctx, int comp, int32_t i, int32_t j, int32_t k, const float* waveform,
                    int64_t len, int64_t first_step, int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (where != FDTD_HOST && where != FDTD_DEVICE) return fail(ctx, FDTD_EINVAL, "bad `where`");
    if (comp < FDTD_EX || comp > FDTD_EZ) return fail(ctx, FDTD_EINVAL, "add_source: comp must be Ex, Ey or Ez");
    if (i < 0 || i >= ctx->nx || j < 0 || j >= ctx->ny || k < 0 || k >= ctx->nz)
        return fail(ctx, FDTD_EINVAL, "add_source: cell out of range");
    if (len < 1 || !waveform) return fail(ctx, FDTD_EINVAL, "add_source: empty waveform");
    if (first_step < 0) return fail(ctx, FDTD_EINVAL, "add_source: first_step must be >= 0");
    const int coord[3] = {i, j, k};
    for (int a = 0; a < 3; ++a)
        if (a != comp && ctx->cfg.bc[a] == FDTD_BC_PEC && coord[a] == 0)
            return fail(ctx, FDTD_EINVAL, "add_source: cell lies on a PEC-frozen entry");
    (void)hipSetDevice(ctx->device);
    SourceRec s{comp, i, j, k, len, first_step, nullptr};
    hipError_t e = hipMalloc(&s.wave, (size_t)len * sizeof(float));
    if (e != hipSuccess) return fail(ctx, FDTD_ENOMEM, "add_source: allocation failed");
    e = hipMemcpyAsync(s.wave, waveform, (size_t)len * sizeof(float), kind_from(where, true), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(s.wave);
        return hip_fail(ctx, e, "add_source copy");
    }
    ctx->sources.push_back(s);
    rc = rebuild_dev_sources(ctx);
    if (rc) return rc;
    return (int)ctx->sources.size() - 1;
}

int fdtd_step(fdtd_ctx* ctx, int64_t nsteps)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (nsteps < 0) return fail(ctx, FDTD_EINVAL, "step: nsteps must be >= 0");
    if (nsteps == 0) return FDTD_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->scheme == FDTD_SCHEME_PLAIN) return plain_step(ctx, nsteps);
    if (ctx->scheme == FDTD_SCHEME_PLAIN_FUSED) return plain_fused_step(ctx, nsteps);
    std::string why;
    if (!systolic_supported(ctx, &why)) return fail(ctx, FDTD_EUNSUPPORTED, "systolic: " + why);
    return systolic_step(ctx, nsteps);
}

int fdtd_prepare(fdtd_ctx* ctx, int64_t nsteps)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (nsteps < 0) return fail(ctx, FDTD_EINVAL, "prepare: nsteps must be >= 0");
    if (nsteps == 0) return FDTD_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->scheme == FDTD_SCHEME_PLAIN) return FDTD_OK;
    if (ctx->scheme == FDTD_SCHEME_PLAIN_FUSED) return plain_fused_prepare(ctx);
    std::string why;
    if (!systolic_supported(ctx, &why)) return fail(ctx, FDTD_EUNSUPPORTED, "systolic: " + why);
    return systolic_prepare(ctx, nsteps);
}

int fdtd_step_batch(fdtd_ctx* const* ctxs, int n, int64_t nsteps)
{
    if (!ctxs || n < 1 || n > 65536) return FDTD_EINVAL;
    for (int i = 0; i < n; ++i) {
        int rc = check_live(ctxs[i]);
        if (rc) return rc == FDTD_ESTATE ? fail(ctxs[i], rc, "context is poisoned") : rc;
    }
    fdtd_ctx* lead = ctxs[0];
    if (nsteps < 0) return fail(lead, FDTD_EINVAL, "step_batch: nsteps must be >= 0");
    for (int i = 0; i < n; ++i) {
        if (ctxs[i]->device != lead->device)
            return fail(lead, FDTD_EINVAL, "step_batch: all contexts must be on one device");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(lead, FDTD_EINVAL, "step_batch: a context appears twice");
        std::string why;
        if (!systolic_supported(ctxs[i], &why))
            return fail(lead, FDTD_EUNSUPPORTED, "step_batch: context " + std::to_string(i) + ": " + why);
    }
    if (nsteps == 0) return FDTD_OK;
    (void)hipSetDevice(lead->device);
    return systolic_step_batch(ctxs, n, nsteps);
}

int fdtd_read_fields(fdtd_ctx* ctx, uint32_t comp_mask, float* const dst[6], int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (where != FDTD_HOST && where != FDTD_DEVICE) return fail(ctx, FDTD_EINVAL, "bad `where`");
    if (comp_mask & ~0x3Fu) return fail(ctx, FDTD_EINVAL, "read_fields: comp_mask has bits above 5");
    if (comp_mask && !dst) return fail(ctx, FDTD_EINVAL, "read_fields: dst is NULL");
    for (int c = 0; c < 6; ++c)
        if ((comp_mask >> c & 1u) && !dst[c]) return fail(ctx, FDTD_EINVAL, "read_fields: NULL array");
    (void)hipSetDevice(ctx->device);
    const size_t bytes = (size_t)ctx->ncell * sizeof(float);
    const bool h16 = ctx->storage == FDTD_FP16_STORAGE;
    float* stage = nullptr;
    hipError_t e = hipSuccess;
    if (h16 && where == FDTD_HOST && comp_mask && (e = hipMalloc(&stage, bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, "read_fields: staging allocation failed");
    }
    for (int c = 0; c < 6 && e == hipSuccess; ++c) {
        if (!(comp_mask >> c & 1u)) continue;
        if (h16) {
            // FP16 storage: the stored value times the component's scale, exactly
            float* out = where == FDTD_HOST ? stage : dst[c];
            hipLaunchKernelGGL(from_f16_kernel, dim3(grid_for(ctx->ncell)), dim3(kThreads), 0, ctx->stream,
                               ctx->field16[c], out, (long long)ctx->ncell, ldexpf(1.0f, ctx->fexp[c]));
            e = hipGetLastError();
            if (e == hipSuccess && where == FDTD_HOST)
                e = hipMemcpyAsync(dst[c], stage, bytes, hipMemcpyDeviceToHost, ctx->stream);
            if (e == hipSuccess && where == FDTD_HOST) e = hipStreamSynchronize(ctx->stream);
        } else {
            e = hipMemcpyAsync(dst[c], ctx->field[c], bytes, kind_from(where, false), ctx->stream);
        }
    }
    if (e == hipSuccess && where == FDTD_HOST) e = hipStreamSynchronize(ctx->stream);
    if (stage) (void)hipFree(stage);
    if (e != hipSuccess) return hip_fail(ctx, e, "read_fields");
    if (where == FDTD_HOST) return check_device_error(ctx);
    return FDTD_OK;
}

int fdtd_synchronize(fdtd_ctx* ctx)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    return check_device_error(ctx);
}

int64_t fdtd_current_step(const fdtd_ctx* ctx) { return ctx ? ctx->step_count : -1; }

const char* fdtd_last_error(const fdtd_ctx* ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int fdtd_invariants(fdtd_ctx* ctx, double* sums, double* div_e, double* div_h, int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (where != FDTD_HOST && where != FDTD_DEVICE) return fail(ctx, FDTD_EINVAL, "bad `where`");
    if (!sums) return fail(ctx, FDTD_EINVAL, "invariants: sums is NULL");
    (void)hipSetDevice(ctx->device);
    hipError_t e;
    if (!ctx->inv_scratch) {
        if ((e = hipMalloc(&ctx->inv_scratch, invariants_scratch_doubles() * sizeof(double))) != hipSuccess) {
            (void)hipGetLastError();
            ctx->inv_scratch = nullptr;
            return fail(ctx, FDTD_ENOMEM, std::string("invariants: scratch allocation: ") + hipGetErrorString(e));
        }
    }
    const size_t bytes = (size_t)ctx->ncell * sizeof(double);
    double* stage[2] = {nullptr, nullptr};
    double* want[2] = {div_e, div_h};
    for (int q = 0; q < 2; ++q) {
        if (!want[q] || where == FDTD_DEVICE) continue;
        if ((e = hipMalloc(&stage[q], bytes)) != hipSuccess) {
            (void)hipGetLastError();
            if (stage[0]) (void)hipFree(stage[0]);
            return fail(ctx, FDTD_ENOMEM, "invariants: staging allocation failed");
        }
    }
    double* de = where == FDTD_DEVICE ? div_e : stage[0];
    double* dh = where == FDTD_DEVICE ? div_h : stage[1];
    double* dsum = ctx->inv_scratch + invariants_sums_offset();
    rc = invariants_launch(ctx, ctx->inv_scratch, dsum, de, dh);
    e = hipSuccess;
    if (!rc) {
        e = hipMemcpyAsync(sums, dsum, FDTD_INV_COUNT * sizeof(double), kind_from(where, false), ctx->stream);
        for (int q = 0; q < 2 && e == hipSuccess; ++q)
            if (stage[q]) e = hipMemcpyAsync(want[q], stage[q], bytes, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess && where == FDTD_HOST) e = hipStreamSynchronize(ctx->stream);
    }
    for (int q = 0; q < 2; ++q)
        if (stage[q]) (void)hipFree(stage[q]);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(ctx, e, "invariants");
    if (where == FDTD_HOST) return check_device_error(ctx);
    return FDTD_OK;
}

int fdtd_autotune(fdtd_ctx* ctx, int64_t nsteps, int64_t* tile_x, int64_t* band_steps)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    return autotune_run(ctx, nsteps, tile_x, band_steps);
}

int fdtd_invariants_noalloc(fdtd_ctx* ctx, double* sums, double* div_e, double* div_h)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (!sums) return fail(ctx, FDTD_EINVAL, "invariants_noalloc: sums is NULL");
    if (invariants_scratch_doubles() > kInvScratchDoubles)
        return fail(ctx, FDTD_EUNSUPPORTED, "invariants_noalloc: the reduction needs more scratch than the "
                                            "static array holds");
    double* part = invariants_scratch_ptr(ctx->device);
    if (!part)
        return fail(ctx, FDTD_EUNSUPPORTED, "invariants_noalloc: no static scratch on this device "
                                            "(device ordinal >= 64)");
    (void)hipSetDevice(ctx->device);
    return invariants_launch(ctx, part, sums, div_e, div_h);
}

int fdtd_adjoint(fdtd_ctx* ctx, fdtd_adjoint_spec* spec, float* grad_eps, int where)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    return adjoint_run(ctx, spec, grad_eps, where);
}

int fdtd_set_option(fdtd_ctx* ctx, int option, int64_t value)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    switch (option) {
    case FDTD_OPT_SCHEME:
        if (value != FDTD_SCHEME_PLAIN && value != FDTD_SCHEME_SYSTOLIC && value != FDTD_SCHEME_PLAIN_FUSED)
            return fail(ctx, FDTD_EINVAL, "set_option: unknown scheme");
        ctx->scheme = (int)value;
        return FDTD_OK;
    case FDTD_OPT_BAND_STEPS:
        if (value < 0 || value > 4096) return fail(ctx, FDTD_EINVAL, "set_option: band steps out of range");
        ctx->band_steps = (int)value;
        return FDTD_OK;
    case FDTD_OPT_WORKGROUPS:
        if (value < 0 || value > (1 << 20)) return fail(ctx, FDTD_EINVAL, "set_option: workgroups out of range");
        ctx->workgroups = (int)value;
        return FDTD_OK;
    case FDTD_OPT_SPIN_LIMIT:
        if (value < 1) return fail(ctx, FDTD_EINVAL, "set_option: spin limit must be >= 1");
        ctx->spin_limit = value;
        return FDTD_OK;
    case FDTD_OPT_TILE_X:
        if (value != 0 && value != 11 && value != 15 && value != 19)
            return fail(ctx, FDTD_EINVAL, "set_option: tile width is 0 (default), 11, 15 or 19");
        if (value == 11 && ctx->storage != FDTD_FP32)
            return fail(ctx, FDTD_EUNSUPPORTED, "set_option: the 11-wide tile needs FP32 storage");
        ctx->tile_wx = (int)value;
        return FDTD_OK;
    case FDTD_OPT_AUTOTUNE_PLAIN:
        if (value != 0 && value != 1) return fail(ctx, FDTD_EINVAL, "set_option: autotune-plain is 0 or 1");
        ctx->tune_plain = value == 1;
        return FDTD_OK;
    case FDTD_OPT_GRAPHS:
        if (value != 0 && value != 1) return fail(ctx, FDTD_EINVAL, "set_option: graphs is 0 or 1");
        ctx->use_graphs = value == 1;
        return FDTD_OK;
    case FDTD_OPT_MATERIAL_IDS:
        if (value != 0 && value != 1) return fail(ctx, FDTD_EINVAL, "set_option: material ids is 0 or 1");
        ctx->use_mat = value == 1;
        return FDTD_OK;
    case FDTD_OPT_PROFILE:
        if (value != 0 && value != 1) return fail(ctx, FDTD_EINVAL, "set_option: profile is 0 or 1");
        if (value == 1) {
            rc = collect_timings(ctx);
            if (rc) return rc;
            for (int k = 0; k < FDTD_KERNEL_COUNT; ++k) {
                ctx->launches[k] = 0;
                ctx->total_ms[k] = 0.0;
            }
        }
        ctx->profile = value == 1;
        return FDTD_OK;
    default:
        return fail(ctx, FDTD_EINVAL, "set_option: unknown option");
    }
}

int fdtd_kernel_stats(fdtd_ctx* ctx, int kernel, int64_t* launches, double* total_ms)
{
    int rc = check_live(ctx);
    if (rc) return rc == FDTD_ESTATE ? fail(ctx, rc, "context is poisoned") : rc;
    if (kernel < 0 || kernel >= FDTD_KERNEL_COUNT) return fail(ctx, FDTD_EINVAL, "kernel_stats: bad kernel id");
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    rc = collect_timings(ctx);
    if (rc) return rc;
    if (launches) *launches = ctx->launches[kernel];
    if (total_ms) *total_ms = ctx->total_ms[kernel];
    return FDTD_OK;
}

int fdtd_get_info(const fdtd_ctx* ctx, int key, int64_t* value)
{
    if (!ctx || !value) return FDTD_EINVAL;
    int wx, wy, wz;
    systolic_tile(ctx, &wx, &wy, &wz);
    switch (key) {
    case FDTD_INFO_SYSTOLIC_GRID: *value = ctx->sys_grid; return FDTD_OK;
    case FDTD_INFO_SYSTOLIC_BAND: *value = ctx->sys_band; return FDTD_OK;
    case FDTD_INFO_SYSTOLIC_TICKETS: *value = ctx->sys_tickets; return FDTD_OK;
    case FDTD_INFO_RING_SLOTS: *value = ctx->sys_ring_slots; return FDTD_OK;
    case FDTD_INFO_TILE_X: *value = wx; return FDTD_OK;
    case FDTD_INFO_TILE_Y: *value = wy; return FDTD_OK;
    case FDTD_INFO_TILE_Z: *value = wz; return FDTD_OK;
    case FDTD_INFO_MATERIALS: *value = ctx->nmat; return FDTD_OK;
    case FDTD_INFO_SCHEME: *value = ctx->scheme; return FDTD_OK;
    default: return FDTD_EINVAL;
    }
}

}  // extern "C"
