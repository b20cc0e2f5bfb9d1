// Reverse-time adjoint of the Yee update: gradient of a frequency-domain
// monitor objective with respect to the permittivity (the inverse-design use
// the paper motivates in Section 1).
//
// Forward step n, as linear maps of the state (sources are an additive term
// independent of the permittivity):
//     E^n       = E^{n-1} + cE (.) CH(H^{n-1/2})     (Eq. 1 and permutations)
//     H^{n+1/2} = H^{n-1/2} - cH CE(E^n)
// with CH the backward-difference curl of the E half-step and CE the
// forward-difference curl of the H half-step; the two are transposes of each
// other on the periodic-index grid (CE^T = CH).  Reverse step n, for the
// adjoint fields lE, lH (both zero after the last step):
//     lE += dJ/dE^n               (monitor samples of step n)
//     lE -= cH CH(lH)             (transpose of the H half-step)
//     g  += lE (.) CH(H^{n-1/2})  (dJ/dcE, design box only)
//     lH += CE(cE (.) lE)         (transpose of the E half-step)
// and dJ/deps = -g cE / eps = -g cE^2 dx / dt.
//
// With conductivity the E half-step is E^n = A (.) E^{n-1} + B (.) CH(H^{n-1/2})
// (A the per-step decay, B the curl coefficient, both per cell: the
// semi-implicit conductive update).  The reverse step then decays the adjoint
// E by A before the new terms are added, weights the transposed curl by B,
// and keeps a second sum gA += lE (.) E^{n-1} for dJ/dA.  With sigma held
// fixed, dA/deps = (1 - A) B dx / dt and dB/deps = -B^2 dx / dt, so
//     dJ/deps = (dx / dt) B ((1 - A) gA - B gB),
// gB being the sum g above (zero where B is pinned to 0).
//
// The run is cut into segments of S steps.  The forward run stores the six
// fields at the start of every segment but the last, and records the last
// segment's CH(H^{n-1/2}) (and E^{n-1} with conductivity) over the design box
// as it goes; the reverse sweep runs that segment's reverse steps at once,
// then, for each earlier segment, recomputes it from its checkpoint to record
// the same history and runs its reverse steps.  When the whole history fits
// in device memory, S = N: one segment, no checkpoint and no recompute.  The monitor
// transform and the gradient accumulate in FP64; the adjoint fields are FP32.
#include "fdtd_internal.h"

#include <math.h>

#include <algorithm>

namespace {

constexpr int kBX = 64;  // threads along z
constexpr int kBY = 4;   // threads along y

struct Box {
    int lo[3];
    int n[3];
    __host__ __device__ long long cells() const { return (long long)n[0] * n[1] * n[2]; }
};

__device__ __forceinline__ void box_cell(const Box& b, long long q, int& i, int& j, int& k)
{
    k = b.lo[2] + (int)(q % b.n[2]);
    const long long r = q / b.n[2];
    j = b.lo[1] + (int)(r % b.n[1]);
    i = b.lo[0] + (int)(r / b.n[1]);
}

// F += E(r) (cr + i ci) over the monitor box; F interleaves re, im.
__global__ void adj_dft_kernel(const float* __restrict__ E, Box b, int ny, int nz, double cr,
                               double ci, double* __restrict__ F)
{
    const long long nb = b.cells();
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nb;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const double e = (double)E[((long long)i * ny + j) * nz + k];
        F[2 * q] += e * cr;
        F[2 * q + 1] += e * ci;
    }
}

// lE(r) += dJ/dE^n(r) = 2 Re(conj(F(r)) (cr + i ci)) over the monitor box.
__global__ void adj_src_kernel(float* __restrict__ lE, Box b, int ny, int nz,
                               const double* __restrict__ F, double cr, double ci)
{
    const long long nb = b.cells();
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nb;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const long long p = ((long long)i * ny + j) * nz + k;
        lE[p] = (float)((double)lE[p] + 2.0 * (F[2 * q] * cr + F[2 * q + 1] * ci));
    }
}

// out[c][q] = CH(H)_c at the design-box cells (backward differences, the
// E half-step's curl, with the grid's periodic index arithmetic); with
// conductivity also out[3 + c][q] = E_c there.
template <bool LOSSY>
__global__ void adj_curl_box_kernel(const float* __restrict__ Hx, const float* __restrict__ Hy,
                                    const float* __restrict__ Hz, const float* __restrict__ Ex,
                                    const float* __restrict__ Ey, const float* __restrict__ Ez,
                                    Box b, int nx, int ny, int nz, float* __restrict__ out)
{
    const long long nb = b.cells();
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nb;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const int im = i == 0 ? nx - 1 : i - 1, jm = j == 0 ? ny - 1 : j - 1,
                  km = k == 0 ? nz - 1 : k - 1;
        auto at = [&](int a, int c, int d) { return ((long long)a * ny + c) * nz + d; };
        const long long p = at(i, j, k);
        out[q] = (Hz[p] - Hz[at(i, jm, k)]) - (Hy[p] - Hy[at(i, j, km)]);
        out[nb + q] = (Hx[p] - Hx[at(i, j, km)]) - (Hz[p] - Hz[at(im, j, k)]);
        out[2 * nb + q] = (Hy[p] - Hy[at(im, j, k)]) - (Hx[p] - Hx[at(i, jm, k)]);
        if (LOSSY) {
            out[3 * nb + q] = Ex[p];
            out[4 * nb + q] = Ey[p];
            out[5 * nb + q] = Ez[p];
        }
    }
}

// g[c][q] += lE_c(r) * ch[c][q] over the design box; with conductivity also
// g[3 + c][q] += lE_c(r) * ch[3 + c][q] (the recorded E^{n-1}).
template <bool LOSSY>
__global__ void adj_grad_kernel(const float* __restrict__ lEx, const float* __restrict__ lEy,
                                const float* __restrict__ lEz, Box b, int ny, int nz,
                                const float* __restrict__ ch, double* __restrict__ g)
{
    const long long nb = b.cells();
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nb;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const long long p = ((long long)i * ny + j) * nz + k;
        g[q] += (double)lEx[p] * (double)ch[q];
        g[nb + q] += (double)lEy[p] * (double)ch[nb + q];
        g[2 * nb + q] += (double)lEz[p] * (double)ch[2 * nb + q];
        if (LOSSY) {
            g[3 * nb + q] += (double)lEx[p] * (double)ch[3 * nb + q];
            g[4 * nb + q] += (double)lEy[p] * (double)ch[4 * nb + q];
            g[5 * nb + q] += (double)lEz[p] * (double)ch[5 * nb + q];
        }
    }
}

// dJ/deps_c = -g_c cE_c^2 dx / dt over the design box (0 where cE is pinned);
// with conductivity (ca non-null, cE then being B)
// dJ/deps_c = (dx / dt) B ((1 - A) gA_c - B gB_c).  With iso the three
// components' derivatives are added in double into one block (one
// permittivity per cell driving all three components).
template <bool LOSSY>
__global__ void adj_eps_kernel(const double* __restrict__ g, const float* __restrict__ cEx,
                               const float* __restrict__ cEy, const float* __restrict__ cEz,
                               const float* __restrict__ cax, const float* __restrict__ cay,
                               const float* __restrict__ caz, Box b, int ny, int nz, double dx_dt,
                               int iso, float* __restrict__ out)
{
    const long long nb = b.cells();
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nb;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_cell(b, q, i, j, k);
        const long long p = ((long long)i * ny + j) * nz + k;
        const float* ce[3] = {cEx, cEy, cEz};
        const float* ca[3] = {cax, cay, caz};
        double tot = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double v = (double)ce[c][p];
            double d = -g[c * nb + q] * v * v * dx_dt;
            if (LOSSY) d += (1.0 - (double)ca[c][p]) * v * dx_dt * g[(3 + c) * nb + q];
            if (v == 0.0) d = 0.0;
            tot += d;
            if (!iso) out[c * nb + q] = (float)d;
        }
        if (iso) out[q] = (float)tot;
    }
}

// lE -= cH CH(lH): the transpose of the H half-step; with conductivity the
// adjoint E first decays, lE = A (.) lE - cH CH(lH) (the transpose of the
// previous reverse step's E half-step, carried here so that one pass over lE
// does both).  Same layout as the plain E kernel: one (j, k) column per
// thread, streaming along x.
template <bool LOSSY>
__global__ __launch_bounds__(kBX* kBY) void adj_E_kernel(
    float* __restrict__ Ex, float* __restrict__ Ey, float* __restrict__ Ez,
    const float* __restrict__ Hx, const float* __restrict__ Hy, const float* __restrict__ Hz,
    const float* __restrict__ cax, const float* __restrict__ cay, const float* __restrict__ caz,
    float cH, int nx, int ny, int nz, int xchunk)
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
        const float dx_ = (hz - Hz[b + row_jm]) - (hy - Hy[b + row_km]);
        const float dy_ = (hx - Hx[b + row_km]) - (hz - hz_im);
        const float dz_ = (hy - hy_im) - (hx - Hx[b + row_jm]);
        if (LOSSY) {
            Ex[p] = cax[p] * Ex[p] - cH * dx_;
            Ey[p] = cay[p] * Ey[p] - cH * dy_;
            Ez[p] = caz[p] * Ez[p] - cH * dz_;
        } else {
            Ex[p] -= cH * dx_;
            Ey[p] -= cH * dy_;
            Ez[p] -= cH * dz_;
        }
        hy_im = hy;
        hz_im = hz;
    }
}

// lH += CE(cE (.) lE): the transpose of the E half-step (forward differences
// of the coefficient-weighted adjoint E).
__global__ __launch_bounds__(kBX* kBY) void adj_H_kernel(
    const float* __restrict__ Ex, const float* __restrict__ Ey, const float* __restrict__ Ez,
    const float* __restrict__ cEx, const float* __restrict__ cEy, const float* __restrict__ cEz,
    float* __restrict__ Hx, float* __restrict__ Hy, float* __restrict__ Hz, int nx, int ny, int nz,
    int xchunk)
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
    float wy_c = cEy[i0 * plane + row] * Ey[i0 * plane + row];
    float wz_c = cEz[i0 * plane + row] * Ez[i0 * plane + row];
    for (int i = i0; i < i1; ++i) {
        const long long b = (long long)i * plane;
        const long long p = b + row;
        const long long bp = (long long)(i == nx - 1 ? 0 : i + 1) * plane;
        const float wy_ip = cEy[bp + row] * Ey[bp + row], wz_ip = cEz[bp + row] * Ez[bp + row];
        const float wx = cEx[p] * Ex[p];
        const float wz_jp = cEz[b + row_jp] * Ez[b + row_jp], wx_jp = cEx[b + row_jp] * Ex[b + row_jp];
        const float wy_kp = cEy[b + row_kp] * Ey[b + row_kp], wx_kp = cEx[b + row_kp] * Ex[b + row_kp];
        Hx[p] += (wz_jp - wz_c) - (wy_kp - wy_c);
        Hy[p] += (wx_kp - wx) - (wz_ip - wz_c);
        Hz[p] += (wy_ip - wy_c) - (wx_jp - wx);
        wy_c = wy_ip;
        wz_c = wz_ip;
    }
}

int box_grid(long long cells) { return (int)std::max<long long>(1, std::min<long long>((cells + 255) / 256, 4096)); }

void column_grid(const fdtd_ctx* ctx, dim3* grid, int* xchunk)
{
    const int gx = (ctx->nz + kBX - 1) / kBX;
    const int gy = (ctx->ny + kBY - 1) / kBY;
    long long base = (long long)gx * gy;
    long long nchunks = (8192 + base - 1) / base;
    nchunks = std::max<long long>(1, std::min<long long>(nchunks, ctx->nx));
    *xchunk = (int)((ctx->nx + nchunks - 1) / nchunks);
    *grid = dim3(gx, gy, (ctx->nx + *xchunk - 1) / *xchunk);
}

// Device buffers of one adjoint call, freed on every exit path.
struct Work {
    float* ckpt = nullptr;   // checkpoints of segments 0..nseg-2, then the final state
    float* lam = nullptr;    // 6 adjoint fields
    double* F = nullptr;     // monitor transform, re/im
    float* hist = nullptr;   // S x (3 or 6) x design cells: CH(H^{n-1/2}) (and E^{n-1})
    double* g = nullptr;     // (3 or 6) x design cells: dJ/dcE (and dJ/dA)
    float* out = nullptr;    // 3 x design cells (host destination only)
    ~Work()
    {
        for (void* p : {(void*)ckpt, (void*)lam, (void*)F, (void*)hist, (void*)g, (void*)out})
            if (p) (void)hipFree(p);
    }
};

}  // namespace

namespace fdtd {

int adjoint_run(fdtd_ctx* ctx, fdtd_adjoint_spec* spec, float* grad_eps, int where)
{
    if (!spec || spec->struct_size != sizeof(fdtd_adjoint_spec))
        return fail(ctx, FDTD_EINVAL, "adjoint: spec is NULL or struct_size does not match");
    if (!grad_eps || (where != FDTD_HOST && where != FDTD_DEVICE))
        return fail(ctx, FDTD_EINVAL, "adjoint: grad_eps is NULL or where is invalid");
    if (ctx->storage != FDTD_FP32)
        return fail(ctx, FDTD_EUNSUPPORTED, "adjoint: needs FP32 storage");
    if (spec->mon_comp < FDTD_EX || spec->mon_comp > FDTD_EZ)
        return fail(ctx, FDTD_EINVAL, "adjoint: the monitored component must be Ex, Ey or Ez");
    if (spec->isotropic != 0 && spec->isotropic != 1)
        return fail(ctx, FDTD_EINVAL, "adjoint: isotropic must be 0 or 1");
    if (spec->nsteps < 1 || spec->nsteps > (int64_t(1) << 31) || spec->checkpoint_every < 0)
        return fail(ctx, FDTD_EINVAL, "adjoint: nsteps must be in [1, 2^31], checkpoint_every >= 0");
    const int n3[3] = {ctx->nx, ctx->ny, ctx->nz};
    Box mon, des;
    for (int a = 0; a < 3; ++a) {
        if (spec->mon_lo[a] < 0 || spec->mon_hi[a] > n3[a] || spec->mon_lo[a] >= spec->mon_hi[a] ||
            spec->des_lo[a] < 0 || spec->des_hi[a] > n3[a] || spec->des_lo[a] >= spec->des_hi[a])
            return fail(ctx, FDTD_EINVAL, "adjoint: monitor and design boxes must be non-empty and inside the grid");
        mon.lo[a] = spec->mon_lo[a];
        mon.n[a] = spec->mon_hi[a] - spec->mon_lo[a];
        des.lo[a] = spec->des_lo[a];
        des.n[a] = spec->des_hi[a] - spec->des_lo[a];
    }
    const int64_t N = spec->nsteps;
    const size_t nc = (size_t)ctx->ncell;
    const long long nmon = mon.cells(), ndes = des.cells();
    const bool lossy = ctx->ca[0] != nullptr;
    const int nrec = lossy ? 6 : 3;  // recorded design-box arrays per step
    const size_t step_hist = (size_t)nrec * (size_t)ndes * sizeof(float);
    int64_t S = spec->checkpoint_every;
    if (S == 0) {
        // automatic: the whole history when it takes at most half the free
        // device memory, else a checkpoint every 200 steps
        size_t free_b = 0, total_b = 0;
        (void)hipSetDevice(ctx->device);
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            free_b = 0;
        }
        S = (double)N * (double)step_hist <= 0.5 * (double)free_b ? N : 200;
    }
    S = std::min<int64_t>(S, N);
    const int64_t nseg = (N + S - 1) / S;
    const int64_t last0 = (nseg - 1) * S;  // steps done when the last segment starts
    const int64_t nckpt = nseg > 1 ? nseg : 0;  // nseg - 1 checkpoints and the final state

    // sizes in double first: a request this large cannot be met, and the
    // size_t products below must not wrap
    if ((double)nckpt * 6.0 * (double)nc * sizeof(float) + (double)S * (double)step_hist > 4.0e18)
        return fail(ctx, FDTD_ENOMEM, "adjoint working memory: request too large");

    Work w;
    hipError_t e;
    if ((nckpt && (e = hipMalloc(&w.ckpt, (size_t)nckpt * 6 * nc * sizeof(float))) != hipSuccess) ||
        (e = hipMalloc(&w.lam, 6 * nc * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&w.F, 2 * (size_t)nmon * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&w.hist, (size_t)S * step_hist)) != hipSuccess ||
        (e = hipMalloc(&w.g, nrec * (size_t)ndes * sizeof(double))) != hipSuccess ||
        (where == FDTD_HOST && (e = hipMalloc(&w.out, 3 * (size_t)ndes * sizeof(float))) != hipSuccess)) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, std::string("adjoint working memory: ") + hipGetErrorString(e));
    }
    hipStream_t st = ctx->stream;
    auto copy_state = [&](float* dst_base, bool to_ckpt) -> hipError_t {
        for (int c = 0; c < 6; ++c) {
            float* ck = dst_base + c * nc;
            hipError_t r = to_ckpt ? hipMemcpyAsync(ck, ctx->field[c], nc * sizeof(float), hipMemcpyDeviceToDevice, st)
                                   : hipMemcpyAsync(ctx->field[c], ck, nc * sizeof(float), hipMemcpyDeviceToDevice, st);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    };
    const double dt = ctx->cfg.dt;
    auto phase = [&](int64_t n, double* cr, double* ci) {
        const double th = spec->omega * (double)n * dt;
        *cr = cos(th);
        *ci = -sin(th);
    };
    const int64_t s0 = ctx->step_count;
    const int comp = spec->mon_comp;

    // ---- forward run with the monitor transform and the checkpoints
    if ((e = hipMemsetAsync(w.F, 0, 2 * (size_t)nmon * sizeof(double), st)) != hipSuccess)
        return hip_fail(ctx, e, "adjoint: clear transform");
    for (int64_t n = 1; n <= N; ++n) {
        if (n - 1 < last0) {
            if ((n - 1) % S == 0 && (e = copy_state(w.ckpt + (size_t)((n - 1) / S) * 6 * nc, true)) != hipSuccess)
                return hip_fail(ctx, e, "adjoint: checkpoint");
        } else {
            // last segment: CH(H^{n-1/2}) (and E^{n-1}) recorded before step n
            hipLaunchKernelGGL((lossy ? adj_curl_box_kernel<true> : adj_curl_box_kernel<false>),
                               dim3(box_grid(ndes)), dim3(256), 0, st, ctx->field[3], ctx->field[4],
                               ctx->field[5], ctx->field[0], ctx->field[1], ctx->field[2], des, ctx->nx,
                               ctx->ny, ctx->nz, w.hist + (size_t)(n - 1 - last0) * nrec * ndes);
        }
        int rc = plain_step(ctx, 1);
        if (rc) return rc;
        double cr, ci;
        phase(n, &cr, &ci);
        hipLaunchKernelGGL(adj_dft_kernel, dim3(box_grid(nmon)), dim3(256), 0, st, ctx->field[comp], mon,
                           ctx->ny, ctx->nz, cr, ci, w.F);
    }
    if (nckpt && (e = copy_state(w.ckpt + (size_t)(nseg - 1) * 6 * nc, true)) != hipSuccess)
        return hip_fail(ctx, e, "adjoint: final state");
    std::vector<double> Fh(2 * (size_t)nmon);
    if ((e = hipMemcpyAsync(Fh.data(), w.F, Fh.size() * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "adjoint: read transform");
    double J = 0.0;
    for (long long q = 0; q < nmon; ++q) J += Fh[2 * q] * Fh[2 * q] + Fh[2 * q + 1] * Fh[2 * q + 1];

    // ---- reverse sweep, one checkpointed segment at a time
    float* lE[3] = {w.lam, w.lam + nc, w.lam + 2 * nc};
    float* lH[3] = {w.lam + 3 * nc, w.lam + 4 * nc, w.lam + 5 * nc};
    if ((e = hipMemsetAsync(w.lam, 0, 6 * nc * sizeof(float), st)) != hipSuccess ||
        (e = hipMemsetAsync(w.g, 0, nrec * (size_t)ndes * sizeof(double), st)) != hipSuccess)
        return hip_fail(ctx, e, "adjoint: clear");
    dim3 grid;
    int xchunk;
    column_grid(ctx, &grid, &xchunk);
    const dim3 block(kBX, kBY);
    int64_t recomputed = 0;
    for (int64_t m = nseg - 1; m >= 0; --m) {
        const int64_t n0 = m * S;  // steps done at the checkpoint
        const int64_t len = std::min<int64_t>(S, N - n0);
        // the last segment's history was recorded by the forward run
        if (m < nseg - 1) {
            if ((e = copy_state(w.ckpt + (size_t)m * 6 * nc, false)) != hipSuccess)
                return hip_fail(ctx, e, "adjoint: restore checkpoint");
            ctx->step_count = s0 + n0;
        }
        for (int64_t l = 0; m < nseg - 1 && l < len; ++l) {
            // CH(H^{n-1/2}) (and E^{n-1}) for step n = n0 + l + 1, before that step runs
            hipLaunchKernelGGL((lossy ? adj_curl_box_kernel<true> : adj_curl_box_kernel<false>),
                               dim3(box_grid(ndes)), dim3(256), 0, st, ctx->field[3], ctx->field[4],
                               ctx->field[5], ctx->field[0], ctx->field[1], ctx->field[2], des, ctx->nx,
                               ctx->ny, ctx->nz, w.hist + (size_t)l * nrec * ndes);
            if (l + 1 < len) {
                int rc = plain_step(ctx, 1);
                if (rc) return rc;
                ++recomputed;
            }
        }
        for (int64_t l = len - 1; l >= 0; --l) {
            const int64_t n = n0 + l + 1;
            double cr, ci;
            phase(n, &cr, &ci);
            // lE = A lE - cH CH(lH), then the monitor samples of step n
            hipLaunchKernelGGL((lossy ? adj_E_kernel<true> : adj_E_kernel<false>), grid, block, 0, st,
                               lE[0], lE[1], lE[2], lH[0], lH[1], lH[2], ctx->ca[0], ctx->ca[1],
                               ctx->ca[2], ctx->cH, ctx->nx, ctx->ny, ctx->nz, xchunk);
            hipLaunchKernelGGL(adj_src_kernel, dim3(box_grid(nmon)), dim3(256), 0, st, lE[comp], mon, ctx->ny,
                               ctx->nz, (const double*)w.F, cr, ci);
            hipLaunchKernelGGL((lossy ? adj_grad_kernel<true> : adj_grad_kernel<false>),
                               dim3(box_grid(ndes)), dim3(256), 0, st, lE[0], lE[1], lE[2], des, ctx->ny,
                               ctx->nz, (const float*)(w.hist + (size_t)l * nrec * ndes), w.g);
            hipLaunchKernelGGL(adj_H_kernel, grid, block, 0, st, lE[0], lE[1], lE[2], ctx->coef[0],
                               ctx->coef[1], ctx->coef[2], lH[0], lH[1], lH[2], ctx->nx, ctx->ny, ctx->nz,
                               xchunk);
        }
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(ctx, e, "launch(adjoint sweep)");
    }

    // ---- the state after the forward run (still in place with one
    // segment), and the gradient
    if (nckpt && (e = copy_state(w.ckpt + (size_t)(nseg - 1) * 6 * nc, false)) != hipSuccess)
        return hip_fail(ctx, e, "adjoint: restore final state");
    ctx->step_count = s0 + N;
    float* dst = where == FDTD_DEVICE ? grad_eps : w.out;
    hipLaunchKernelGGL((lossy ? adj_eps_kernel<true> : adj_eps_kernel<false>), dim3(box_grid(ndes)),
                       dim3(256), 0, st, (const double*)w.g, ctx->coef[0], ctx->coef[1], ctx->coef[2],
                       ctx->ca[0], ctx->ca[1], ctx->ca[2], des, ctx->ny, ctx->nz,
                       ctx->cfg.dx / ctx->cfg.dt, (int)spec->isotropic, dst);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(ctx, e, "launch(adjoint gradient)");
    const size_t nblocks = spec->isotropic ? 1 : 3;
    if (where == FDTD_HOST &&
        (e = hipMemcpyAsync(grad_eps, w.out, nblocks * (size_t)ndes * sizeof(float), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(ctx, e, "adjoint: copy gradient");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "adjoint: synchronize");
    spec->objective = J;
    spec->recomputed_steps = recomputed;
    return FDTD_OK;
}

}  // namespace fdtd
