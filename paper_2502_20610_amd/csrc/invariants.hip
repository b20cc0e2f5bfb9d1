// Discrete invariants of the Yee update, reduced in FP64 on the device.
//
// The update of Section 2 (Eq. (1) and its cyclic permutations, E before H)
// is, with the coefficients the context actually applies,
//     E^{n+1} = E^n + cE (.) C_h H^{n+1/2},   H^{n+3/2} = H^{n+1/2} - cH C_e E^{n+1},
// where C_h is the backward-difference curl, C_e the forward-difference one
// and C_e = C_h^T on the periodic-index grid.  Two consequences hold exactly
// for every state the update produces (in exact arithmetic):
//   * the leapfrog energy Q = sum eps|E|^2 + sum |H|^2 + cH sum E . (C_h H),
//     with eps_c = cH / cE_c per entry (the permittivity the coefficients
//     encode), is constant in a lossless box;
//   * the backward divergence of eps E at every node off the PEC walls and
//     the forward divergence of H at every cell do not change without
//     sources (Gauss's laws of the discrete update).
// With conductivity E^{n+1} = ca E^n + cb C_h H^{n+1/2}; the permittivity is
// then cH (1 + ca) / (2 cb) and Q decays.  Entries frozen by a PEC wall (the
// tangential E components on its index-0 plane) are excluded from the sums
// and read as eps E = 0 in the divergence.
//
// Every sum is accumulated in double from the stored FP32 (or binary16)
// values.  The reduction is deterministic: a fixed number of blocks, each
// with a fixed cell range, writes its partial sums, and one block adds them
// in a fixed order.
#include <string.h>

#include <mutex>

#include "fdtd_internal.h"

namespace fdtd {

namespace {

constexpr int kRedThreads = 256;
constexpr int kPart = 8;  // doubles per partial record (FDTD_INV_COUNT used)
static_assert(kInvScratchDoubles == (size_t)kInvBlocks * kPart + kPart, "scratch: partials + sums");

struct InvArgs {
    const float* f[6];
    const uint16_t* f16[6];
    float sc[6];  // binary16 storage: value = stored * sc
    const float* cE[3];
    const uint16_t* c16[3];
    const float* ca[3];  // conductive decay (lossy variant only)
    int nx, ny, nz;
    int pec[3];    // 1 = PEC axis
    double cH;
    double* part;  // [blocks][kPart] partial sums
    double* div_e; // per node, or null
    double* div_h; // per cell, or null
};

template <bool F16>
__device__ __forceinline__ double fld(const InvArgs& A, int q, long long p)
{
    if (F16) return (double)((float)__builtin_bit_cast(_Float16, A.f16[q][p]) * A.sc[q]);
    return (double)A.f[q][p];
}

// eps of E component c at p, from the coefficients (0 on a frozen entry)
template <bool F16, bool LOSSY>
__device__ __forceinline__ double eps_of(const InvArgs& A, int c, long long p, bool frozen)
{
    if (frozen) return 0.0;
    double ce = F16 ? (double)(float)__builtin_bit_cast(_Float16, A.c16[c][p]) : (double)A.cE[c][p];
    if (LOSSY) return A.cH * (1.0 + (double)A.ca[c][p]) / (2.0 * ce);
    return A.cH / ce;
}

// E component c at (i, j, k) is frozen by a PEC wall: it lies on the
// index-0 plane of a PEC axis to which it is tangential
__device__ __forceinline__ bool frozen_at(const InvArgs& A, int c, int i, int j, int k)
{
    return (c != 0 && A.pec[0] && i == 0) || (c != 1 && A.pec[1] && j == 0) || (c != 2 && A.pec[2] && k == 0);
}

template <bool F16, bool LOSSY>
__global__ __launch_bounds__(kRedThreads) void invariants_kernel(InvArgs A)
{
    __shared__ double red[kRedThreads];
    const long long plane = (long long)A.ny * A.nz;
    const long long n = (long long)A.nx * plane;
    double s[FDTD_INV_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    // sums: 0 Q (filled at the end), 1 eps|E|^2, 2 |H|^2, 3 |div eps E|, 4 (div eps E)^2,
    //       5 |div H|, 6 (div H)^2; the coupling E.(C_h H) is kept apart
    double cpl = 0.0;
    for (long long p = (long long)blockIdx.x * kRedThreads + threadIdx.x; p < n;
         p += (long long)gridDim.x * kRedThreads) {
        const int k = (int)(p % A.nz);
        const int j = (int)((p / A.nz) % A.ny);
        const int i = (int)(p / plane);
        const long long pim = i == 0 ? p + (long long)(A.nx - 1) * plane : p - plane;
        const long long pjm = j == 0 ? p + (long long)(A.ny - 1) * A.nz : p - A.nz;
        const long long pkm = k == 0 ? p + (A.nz - 1) : p - 1;
        const long long pip = i == A.nx - 1 ? p - (long long)(A.nx - 1) * plane : p + plane;
        const long long pjp = j == A.ny - 1 ? p - (long long)(A.ny - 1) * A.nz : p + A.nz;
        const long long pkp = k == A.nz - 1 ? p - (A.nz - 1) : p + 1;
        const double ex = fld<F16>(A, 0, p), ey = fld<F16>(A, 1, p), ez = fld<F16>(A, 2, p);
        const double hx = fld<F16>(A, 3, p), hy = fld<F16>(A, 4, p), hz = fld<F16>(A, 5, p);
        const bool fx = frozen_at(A, 0, i, j, k), fy = frozen_at(A, 1, i, j, k), fz = frozen_at(A, 2, i, j, k);
        const double epx = eps_of<F16, LOSSY>(A, 0, p, fx), epy = eps_of<F16, LOSSY>(A, 1, p, fy),
                     epz = eps_of<F16, LOSSY>(A, 2, p, fz);
        // curl of H at the E positions (backward differences, as in the E update)
        const double chx = (hz - fld<F16>(A, 5, pjm)) - (hy - fld<F16>(A, 4, pkm));
        const double chy = (hx - fld<F16>(A, 3, pkm)) - (hz - fld<F16>(A, 5, pim));
        const double chz = (hy - fld<F16>(A, 4, pim)) - (hx - fld<F16>(A, 3, pjm));
        if (!fx) { s[1] += epx * ex * ex; cpl += ex * chx; }
        if (!fy) { s[1] += epy * ey * ey; cpl += ey * chy; }
        if (!fz) { s[1] += epz * ez * ez; cpl += ez * chz; }
        s[2] += hx * hx + hy * hy + hz * hz;
        // backward divergence of eps E at node (i, j, k), nodes off the PEC walls
        const bool interior = !((A.pec[0] && i == 0) || (A.pec[1] && j == 0) || (A.pec[2] && k == 0));
        double de = 0.0;
        if (interior) {
            const int im = i == 0 ? A.nx - 1 : i - 1, jm = j == 0 ? A.ny - 1 : j - 1, km = k == 0 ? A.nz - 1 : k - 1;
            const bool fxm = frozen_at(A, 0, im, j, k), fym = frozen_at(A, 1, i, jm, k), fzm = frozen_at(A, 2, i, j, km);
            de = ((epx * ex - eps_of<F16, LOSSY>(A, 0, pim, fxm) * fld<F16>(A, 0, pim)) +
                  (epy * ey - eps_of<F16, LOSSY>(A, 1, pjm, fym) * fld<F16>(A, 1, pjm))) +
                 (epz * ez - eps_of<F16, LOSSY>(A, 2, pkm, fzm) * fld<F16>(A, 2, pkm));
            s[3] += fabs(de);
            s[4] += de * de;
        }
        // forward divergence of H at every cell
        const double dh = ((fld<F16>(A, 3, pip) - hx) + (fld<F16>(A, 4, pjp) - hy)) + (fld<F16>(A, 5, pkp) - hz);
        s[5] += fabs(dh);
        s[6] += dh * dh;
        if (A.div_e) A.div_e[p] = de;
        if (A.div_h) A.div_h[p] = dh;
    }
    s[0] = cpl;
    // block sums in a fixed tree order
#pragma unroll
    for (int q = 0; q < FDTD_INV_COUNT; ++q) {
        red[threadIdx.x] = s[q];
        __syncthreads();
        for (int w = kRedThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) A.part[(size_t)blockIdx.x * kPart + q] = red[0];
        __syncthreads();
    }
}

// Add the partial records of nblk blocks in a fixed order; out[0] becomes Q.
__global__ __launch_bounds__(kRedThreads) void invariants_finish(const double* part, int nblk, double cH, double* out)
{
    __shared__ double red[kRedThreads];
    for (int q = 0; q < FDTD_INV_COUNT; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kRedThreads) v += part[(size_t)b * kPart + q];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = kRedThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = red[0];
        __syncthreads();
    }
    // Q = eps|E|^2 + |H|^2 + cH * coupling (out[0] held the coupling sum)
    if (threadIdx.x == 0) out[0] = (out[1] + out[2]) + cH * out[0];
}

}  // namespace

size_t invariants_scratch_doubles() { return kInvScratchDoubles; }

size_t invariants_sums_offset() { return (size_t)kInvBlocks * kPart; }

// Launch the reduction on ctx's stream: the partial records in `part`
// (kInvBlocks * kPart doubles, device memory), the FDTD_INV_COUNT final sums
// at `out` (device memory).  div_e / div_h: device arrays of ncell doubles,
// or null.
int invariants_launch(fdtd_ctx* ctx, double* part, double* out, double* div_e, double* div_h)
{
    InvArgs A;
    memset(&A, 0, sizeof(A));
    const bool h16 = ctx->storage == FDTD_FP16_STORAGE;
    const bool lossy = ctx->ca[0] != nullptr;
    for (int q = 0; q < 6; ++q) {
        A.f[q] = ctx->field[q];
        A.f16[q] = ctx->field16[q];
        A.sc[q] = ldexpf(1.0f, ctx->fexp[q]);
    }
    for (int q = 0; q < 3; ++q) {
        A.cE[q] = ctx->coef[q];
        A.c16[q] = ctx->coef16[q];
        A.ca[q] = ctx->ca[q];
    }
    A.nx = ctx->nx;
    A.ny = ctx->ny;
    A.nz = ctx->nz;
    for (int d = 0; d < 3; ++d) A.pec[d] = ctx->cfg.bc[d] == FDTD_BC_PEC;
    A.cH = (double)ctx->cH;
    A.part = part;
    A.div_e = div_e;
    A.div_h = div_h;
    using Kern = void (*)(InvArgs);
    const Kern k = h16 ? (lossy ? invariants_kernel<true, true> : invariants_kernel<true, false>)
                       : (lossy ? invariants_kernel<false, true> : invariants_kernel<false, false>);
    hipLaunchKernelGGL(k, dim3(kInvBlocks), dim3(kRedThreads), 0, ctx->stream, A);
    hipLaunchKernelGGL(invariants_finish, dim3(1), dim3(kRedThreads), 0, ctx->stream, (const double*)part,
                       kInvBlocks, (double)ctx->cH, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "launch(invariants)");
    return FDTD_OK;
}

}  // namespace fdtd

// Scratch of the allocation-free entry point (fdtd_invariants_noalloc): the
// reduction's partial records followed by its final sums, 64 KiB.  Every GPU
// the library runs on holds its own copy until the process ends; host code
// never uses this name as an address (on the host it is a stand-in), only
// the per-device address looked up below.
static __device__ __align__(256) double scratch[fdtd::kInvScratchDoubles];

namespace fdtd {

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices];  // device address of `scratch`, per device

}  // namespace

int invariants_scratch_init(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return FDTD_OK;  // the entry point refuses
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FDTD_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return FDTD_EHIP;
    }
    g_scratch_ptr[device] = static_cast<double*>(p);
    return FDTD_OK;
}

double* invariants_scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace fdtd
