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

#include <algorithm>
#include <new>

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

// ---- fused step: one launch per step, from (E, H) into other arrays
//
// A block of kFY + 1 wavefronts (one y row each) x 64 lanes (along z) streams
// along x over a chunk of planes.  It owns kFY rows x 64 lanes of columns,
// so every wavefront access is one aligned 256-byte run.  H' of the owned
// cells also needs E' of the +y and +z neighbours.  The extra wavefront
// computes E' of the next block's first row and, on its lanes 0..kFY-1, Ex'
// and Ey' of the cell after each owned row (the next tile's first cell) --
// both again from the inputs, as the neighbouring block does for its own
// cells.  (Tiles of 63 lanes with lane 63 as the halo need no extra cells,
// but their unaligned rows straddle cache lines and ran at half the rate.)
// For each plane i the block
// computes E' (sources included), stages it in LDS, and then H' of plane
// i - 1 from E' of planes i - 1 and i; one plane past the chunk supplies the
// chunk's last H'.  The inputs are only read and the outputs are other
// arrays, so blocks never see each other's results.  Same operations, in the
// same order, as the E half-step, the source additions (in table order) and
// the H half-step of the two-launch step.  Algorithmic traffic: E, H and cE
// in, E and H out -- 60 B per cell update.
//
// The loads of plane i + 1 are issued before the work on plane i, and the
// barrier between the LDS write and the LDS reads waits for LDS traffic only,
// so they stay in flight across it.  Blocks are numbered so that each XCD
// (workgroups are dealt to the eight XCDs in turn) takes a contiguous range
// of (z, y, x-chunk) tiles: neighbouring tiles, which share the cache lines
// of their edge columns, then meet in one L2.
constexpr int kFY = 7;   // owned rows per block
constexpr int kFZ = 64;  // owned lanes per wavefront
constexpr int kXCD = 8;  // XCDs of the device

__device__ __forceinline__ void fused_lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <bool LOSSY>
__global__ __launch_bounds__(64 * (kFY + 1)) void plain_fused_kernel(
    const float* __restrict__ Ex, const float* __restrict__ Ey, const float* __restrict__ Ez,
    const float* __restrict__ Hx, const float* __restrict__ Hy, const float* __restrict__ Hz,
    float* __restrict__ oEx, float* __restrict__ oEy, float* __restrict__ oEz,
    float* __restrict__ oHx, float* __restrict__ oHy, float* __restrict__ oHz,
    const float* __restrict__ cEx, const float* __restrict__ cEy, const float* __restrict__ cEz,
    const float* __restrict__ cax, const float* __restrict__ cay, const float* __restrict__ caz,
    float cH, int nx, int ny, int nz, int gz, int gy, int ntiles, int xchunk,
    const fdtd::DevSource* __restrict__ src, int nsrc, long long step, const long long* step_in,
    long long* step_out)
{
    // a replayed graph passes the step through device words: read from
    // step_in, the next one written to step_out (a different word, so no
    // block of this launch reads what it writes)
    if (step_in) {
        step = *step_in;
        if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) *step_out = step + 1;
    }
    // E' of the last three planes (x, y, z components): a plane is read in
    // the iteration after it is written and overwritten two iterations
    // later, so one barrier per plane separates every write from the reads
    // of the buffer's previous contents
    __shared__ float st[3][3][kFY + 1][64];
    __shared__ float sth[3][2][kFY];  // Ex', Ey' of the cell after each owned row
    // tile of this block: launch order dealt round the XCDs, tile order
    // contiguous per XCD (the launch has a multiple of kXCD blocks)
    const int per_xcd = (int)(gridDim.x / kXCD);
    const int tile = (int)(blockIdx.x % kXCD) * per_xcd + (int)(blockIdx.x / kXCD);
    if (tile >= ntiles) return;  // whole block: before any barrier
    const int tz = tile % gz, ty = (tile / gz) % gy, tx = tile / (gz * gy);
    const int L = threadIdx.x, R = threadIdx.y;
    const int k0 = tz * kFZ, j0 = ty * kFY;
    const int i0 = tx * xchunk;
    const int i1 = min(nx, i0 + xchunk);
    const int k = (k0 + L) % nz, j = (j0 + R) % ny;  // halo and spare lanes wrap
    const bool own = R < kFY && j0 + R < ny && k0 + L < nz;
    const int km = k == 0 ? nz - 1 : k - 1;
    const int jm = j == 0 ? ny - 1 : j - 1;
    // lane r < kFY of the extra wavefront: Ex', Ey' at (row r, z = kh), whose
    // -z neighbour is the last lane of row r (needed when that lane is owned)
    const bool halo = R == kFY && L < kFY && k0 + 63 < nz;
    const int kh = (k0 + 64) % nz, khm = (k0 + 63) % nz;
    const int jr = (j0 + L) % ny;
    const int jrm = jr == 0 ? ny - 1 : jr - 1;
    const long long rowh = (long long)jr * nz + kh;
    const long long rowh_jm = (long long)jrm * nz + kh;
    const long long rowh_km = (long long)jr * nz + khm;
    const long long plane = (long long)ny * nz;
    const long long row = (long long)j * nz + k;
    const long long row_jm = (long long)jm * nz + k;
    const long long row_km = (long long)j * nz + km;
    const int im0 = i0 == 0 ? nx - 1 : i0 - 1;
    float hy_im = Hy[im0 * plane + row];
    float hz_im = Hz[im0 * plane + row];
    float hz_im_h = halo ? Hz[im0 * plane + rowh] : 0.f;  // Hz(i - 1) at the halo cell
    // inputs of one plane at this lane's cell (and at its halo cell)
    struct In {
        float hx, hy, hz, hz_jm, hx_jm, hy_km, hx_km, cx, cy, cz, ex, ey, ez, ax, ay, az;
        float h_ex, h_ey, h_cx, h_cy, h_hx, h_hy, h_hz, h_hz_jm, h_hx_km, h_hy_km, h_ax, h_ay;
    };
    auto load = [&](int ii) {
        const long long b = (long long)ii * plane;
        const long long p = b + row;
        In v{};
        v.hx = Hx[p];
        v.hy = Hy[p];
        v.hz = Hz[p];
        v.hz_jm = Hz[b + row_jm];
        v.hx_jm = Hx[b + row_jm];
        v.hy_km = Hy[b + row_km];
        v.hx_km = Hx[b + row_km];
        v.cx = cEx[p];
        v.cy = cEy[p];
        v.cz = cEz[p];
        v.ex = Ex[p];
        v.ey = Ey[p];
        v.ez = Ez[p];
        if (LOSSY) {
            v.ax = cax[p];
            v.ay = cay[p];
            v.az = caz[p];
        }
        if (halo) {
            const long long q = b + rowh;
            v.h_ex = Ex[q];
            v.h_ey = Ey[q];
            v.h_cx = cEx[q];
            v.h_cy = cEy[q];
            v.h_hx = Hx[q];
            v.h_hy = Hy[q];
            v.h_hz = Hz[q];
            v.h_hz_jm = Hz[b + rowh_jm];
            v.h_hx_km = Hx[b + rowh_km];
            v.h_hy_km = Hy[b + rowh_km];
            if (LOSSY) {
                v.h_ax = cax[q];
                v.h_ay = cay[q];
            }
        }
        return v;
    };
    In cur = load(i0);
    float pex = 0.f, pey = 0.f, pez = 0.f;  // E' of the previous plane
    float phx = 0.f, phy = 0.f, phz = 0.f;  // H of the previous plane
    for (int i = i0; i <= i1; ++i) {
        const int ii = i == nx ? 0 : i;
        In nxt = cur;
        if (i < i1) nxt = load(i + 1 == nx ? 0 : i + 1);
        float ex = cur.ex, ey = cur.ey, ez = cur.ez;
        if (LOSSY) {
            ex = cur.ax * ex;
            ey = cur.ay * ey;
            ez = cur.az * ez;
        }
        ex = (ex + cur.cx * (cur.hz - cur.hz_jm)) - cur.cx * (cur.hy - cur.hy_km);
        ey = (ey + cur.cy * (cur.hx - cur.hx_km)) - cur.cy * (cur.hz - hz_im);
        ez = (ez + cur.cz * (cur.hy - hy_im)) - cur.cz * (cur.hx - cur.hx_jm);
        // the halo cell's Ex', Ey'
        float ex_h = 0.f, ey_h = 0.f;
        if (halo) {
            ex_h = LOSSY ? cur.h_ax * cur.h_ex : cur.h_ex;
            ey_h = LOSSY ? cur.h_ay * cur.h_ey : cur.h_ey;
            ex_h = (ex_h + cur.h_cx * (cur.h_hz - cur.h_hz_jm)) - cur.h_cx * (cur.h_hy - cur.h_hy_km);
            ey_h = (ey_h + cur.h_cy * (cur.h_hx - cur.h_hx_km)) - cur.h_cy * (cur.h_hz - hz_im_h);
        }
        // point sources of this step on plane ii (the table and the plane
        // are the same for the whole block), in table order per cell
        for (int q = 0; q < nsrc; ++q) {
            if (src[q].i != ii) continue;
            const long long m = step - src[q].first;
            if (m < 0 || m >= src[q].len) continue;
            const int c = src[q].comp;
            if (src[q].j == j && src[q].k == k) {
                const float w = src[q].wave[m];
                ex = c == 0 ? ex + w : ex;
                ey = c == 1 ? ey + w : ey;
                ez = c == 2 ? ez + w : ez;
            }
            if (halo && src[q].j == jr && src[q].k == kh) {
                const float w = src[q].wave[m];
                ex_h = c == 0 ? ex_h + w : ex_h;
                ey_h = c == 1 ? ey_h + w : ey_h;
            }
        }
        const int bcur = (i - i0) % 3;
        st[bcur][0][R][L] = ex;
        st[bcur][1][R][L] = ey;
        st[bcur][2][R][L] = ez;
        if (halo) {
            sth[bcur][0][L] = ex_h;
            sth[bcur][1][L] = ey_h;
        }
        fused_lds_barrier();
        if (i > i0 && own) {
            // H' of plane i - 1: E' there (registers and LDS) and on plane i
            const int pb = (i - i0 + 2) % 3;
            const float ez_jp = st[pb][2][R + 1][L], ex_jp = st[pb][0][R + 1][L];
            const int l1 = min(L + 1, 63);
            const float ey_kp = L == 63 ? sth[pb][1][R] : st[pb][1][R][l1];
            const float ex_kp = L == 63 ? sth[pb][0][R] : st[pb][0][R][l1];
            const float nhx = (phx - cH * (ez_jp - pez)) + cH * (ey_kp - pey);
            const float nhy = (phy - cH * (ex_kp - pex)) + cH * (ez - pez);
            const float nhz = (phz - cH * (ey - pey)) + cH * (ex_jp - pex);
            const long long po = (long long)(i - 1) * plane + row;
            oEx[po] = pex;
            oEy[po] = pey;
            oEz[po] = pez;
            oHx[po] = nhx;
            oHy[po] = nhy;
            oHz[po] = nhz;
        }
        pex = ex;
        pey = ey;
        pez = ez;
        phx = cur.hx;
        phy = cur.hy;
        phz = cur.hz;
        hy_im = cur.hy;
        hz_im = cur.hz;
        hz_im_h = cur.h_hz;
        cur = nxt;
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

// One step loop of a plain scheme replayed as a HIP graph: kGraphSteps steps
// of kernel nodes, captured once on a private stream and replayed with one
// launch per kGraphSteps steps.  Kernels that need the step number (the
// sources) read it from a device counter that the graph itself advances.
// The graph is rebuilt whenever an argument its kernels were captured with
// changes (arrays, sources, scales, scheme).
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    std::vector<const void*> key;
};

namespace {

constexpr int kGraphSteps = 16;  // steps per replay (even: the fused scheme's two field sets alternate)

__global__ void set_step_kernel(long long* p, long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        p[0] = v;
        p[1] = v;
    }
}

// Everything the captured kernels take: a replay is valid while it is unchanged.
std::vector<const void*> graph_key(const fdtd_ctx* ctx, int scheme)
{
    std::vector<const void*> k;
    k.push_back((const void*)(intptr_t)scheme);
    k.push_back((const void*)(intptr_t)ctx->storage);
    for (int c = 0; c < 6; ++c) {
        k.push_back(ctx->field[c]);
        k.push_back(ctx->alt[c]);
        k.push_back(ctx->field16[c]);
        k.push_back((const void*)(intptr_t)ctx->fexp[c]);
    }
    for (int c = 0; c < 3; ++c) {
        k.push_back(ctx->coef[c]);
        k.push_back(ctx->coef16[c]);
        k.push_back(ctx->ca[c]);
    }
    k.push_back(ctx->dev_sources);
    k.push_back((const void*)(intptr_t)ctx->dev_sources_n);
    k.push_back(ctx->d_step);
    return k;
}

// Queue n steps of the two-launch plain scheme on st.  Direct launches (stepp
// null) start at ctx->step_count and skip the sources kernel on steps no
// source reaches; under capture (stepp set) every step has a sources node
// that reads and advances *stepp.
int queue_plain(fdtd_ctx* ctx, hipStream_t st, int64_t n, long long* stepp)
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
    for (int64_t q = 0; q < n; ++q) {
        const int64_t s = ctx->step_count + q;
        PendingTiming t;
        if (!stepp) timing_begin(ctx, FDTD_KERNEL_PLAIN_E, &t);
        if (h16)
            hipLaunchKernelGGL((plain_E_kernel<false, F16Store>), grid, block, 0, st, f16[0], f16[1],
                               f16[2], f16[3], f16[4], f16[5], c16[0], c16[1], c16[2], nullptr, nullptr,
                               nullptr, ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        else if (ctx->ca[0])
            hipLaunchKernelGGL((plain_E_kernel<true, F32Store>), grid, block, 0, st, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->coef[0], ctx->coef[1], ctx->coef[2], ctx->ca[0], ctx->ca[1],
                               ctx->ca[2], ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        else
            hipLaunchKernelGGL((plain_E_kernel<false, F32Store>), grid, block, 0, st, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->coef[0], ctx->coef[1], ctx->coef[2], nullptr, nullptr, nullptr,
                               ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        if (!stepp) timing_end(ctx, &t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(plain E)");
        if (stepp ? ctx->dev_sources_n > 0 : sources_active(ctx, s)) {
            int rc = launch_sources(ctx, s, st, stepp);
            if (rc) return rc;
        }
        if (!stepp) timing_begin(ctx, FDTD_KERNEL_PLAIN_H, &t);
        if (h16)
            hipLaunchKernelGGL(plain_H_kernel<F16Store>, grid, block, 0, st, f16[0], f16[1], f16[2],
                               f16[3], f16[4], f16[5], ctx->cH, ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        else
            hipLaunchKernelGGL(plain_H_kernel<F32Store>, grid, block, 0, st, ctx->field[0],
                               ctx->field[1], ctx->field[2], ctx->field[3], ctx->field[4], ctx->field[5],
                               ctx->cH, ctx->nx, ctx->ny, ctx->nz, xchunk, sc);
        if (!stepp) timing_end(ctx, &t);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(plain H)");
    }
    return FDTD_OK;
}

// Queue n steps of the fused plain scheme on st (n even under capture, so
// the graph ends on the field set it started from).  Direct launches trade
// ctx->field and ctx->alt after every step; a capture leaves them as they
// were (it passes the step through the device words stepp[0] and stepp[1]).
int queue_fused(fdtd_ctx* ctx, hipStream_t st, int64_t n, long long* stepp)
{
    const int gz = (ctx->nz + kFZ - 1) / kFZ;
    const int gy = (ctx->ny + kFY - 1) / kFY;
    // enough blocks to fill the CUs several times over, with long x runs
    const long long base = (long long)gz * gy;
    long long nchunks = std::max<long long>(1, std::min<long long>((4096 + base - 1) / base, ctx->nx));
    const int xchunk = (int)((ctx->nx + nchunks - 1) / nchunks);
    const long long ntiles = base * ((ctx->nx + xchunk - 1) / xchunk);
    if (ntiles > (1LL << 30)) return fail(ctx, FDTD_EUNSUPPORTED, "fused plain step: grid too large");
    const dim3 grid((unsigned)((ntiles + kXCD - 1) / kXCD * kXCD));  // a multiple of kXCD
    const dim3 block(64, kFY + 1);
    const bool lossy = ctx->ca[0] != nullptr;
    const bool srcs = ctx->dev_sources_n > 0;
    float* in[6];
    float* out[6];
    for (int c = 0; c < 6; ++c) {
        in[c] = ctx->field[c];
        out[c] = ctx->alt[c];
    }
    for (int64_t q = 0; q < n; ++q) {
        const long long* sin = (stepp && srcs) ? stepp + (q & 1) : nullptr;
        long long* sout = (stepp && srcs) ? stepp + ((q + 1) & 1) : nullptr;
        PendingTiming t;
        if (!stepp) timing_begin(ctx, FDTD_KERNEL_PLAIN_FUSED, &t);
        hipLaunchKernelGGL((lossy ? plain_fused_kernel<true> : plain_fused_kernel<false>), grid, block, 0,
                           st, in[0], in[1], in[2], in[3], in[4], in[5], out[0], out[1], out[2],
                           out[3], out[4], out[5], ctx->coef[0], ctx->coef[1], ctx->coef[2], ctx->ca[0],
                           ctx->ca[1], ctx->ca[2], ctx->cH, ctx->nx, ctx->ny, ctx->nz, gz, gy,
                           (int)ntiles, xchunk, (const DevSource*)ctx->dev_sources, ctx->dev_sources_n,
                           (long long)(ctx->step_count + q), sin, sout);
        if (!stepp) timing_end(ctx, &t);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "launch(fused plain step)");
        for (int c = 0; c < 6; ++c) std::swap(in[c], out[c]);
    }
    if (!stepp && (n & 1))
        for (int c = 0; c < 6; ++c) std::swap(ctx->field[c], ctx->alt[c]);
    return FDTD_OK;
}

// (Re)capture the graph of kGraphSteps steps of `scheme` when its key changed.
int ensure_graph(fdtd_ctx* ctx, int scheme)
{
    hipError_t e;
    if (!ctx->d_step) {
        if ((e = hipMalloc(&ctx->d_step, 2 * sizeof(long long))) != hipSuccess) {
            (void)hipGetLastError();
            ctx->d_step = nullptr;
            return fail(ctx, FDTD_ENOMEM, "step graph: counter allocation failed");
        }
    }
    if (!ctx->graph) {
        ctx->graph = new (std::nothrow) StepGraph();
        if (!ctx->graph) return fail(ctx, FDTD_ENOMEM, "step graph: host allocation failed");
    }
    StepGraph* G = ctx->graph;
    std::vector<const void*> key = graph_key(ctx, scheme);
    if (G->exec && G->key == key) return FDTD_OK;
    release_step_graph_exec(G);
    if (!G->cap && (e = hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(ctx, e, "step graph: capture stream");
    if ((e = hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(ctx, e, "step graph: begin capture");
    const int rc = scheme == FDTD_SCHEME_PLAIN_FUSED ? queue_fused(ctx, G->cap, kGraphSteps, ctx->d_step)
                                                     : queue_plain(ctx, G->cap, kGraphSteps, ctx->d_step);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(G->cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "step graph: end capture");
    G->graph = g;
    if ((e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        G->exec = nullptr;
        return hip_fail(ctx, e, "step graph: instantiate");
    }
    G->key = key;
    return FDTD_OK;
}

// Advance n steps: whole graphs of kGraphSteps steps where the option allows
// (and per-kernel timing is off), direct launches for the rest.
int run_steps(fdtd_ctx* ctx, int64_t nsteps, int scheme)
{
    const bool fused = scheme == FDTD_SCHEME_PLAIN_FUSED;
    int64_t reps = (ctx->use_graphs && !ctx->profile) ? nsteps / kGraphSteps : 0;
    if (reps > 0) {
        int rc = ensure_graph(ctx, scheme);
        if (rc) return rc;
        hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->d_step,
                           (long long)ctx->step_count);
        hipError_t e = hipGetLastError();
        for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(ctx->graph->exec, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "step graph: launch");
        ctx->step_count += reps * kGraphSteps;  // (an even count: the field sets are where they were)
    }
    const int64_t rest = nsteps - reps * kGraphSteps;
    if (rest > 0) {
        int rc = fused ? queue_fused(ctx, ctx->stream, rest, nullptr) : queue_plain(ctx, ctx->stream, rest, nullptr);
        if (rc) return rc;
        ctx->step_count += rest;
    }
    return FDTD_OK;
}

}  // namespace

void release_step_graph_exec(StepGraph* G)
{
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    G->exec = nullptr;
    G->graph = nullptr;
    G->key.clear();
}

void release_step_graph(fdtd_ctx* ctx)
{
    if (ctx->graph) {
        release_step_graph_exec(ctx->graph);
        if (ctx->graph->cap) (void)hipStreamDestroy(ctx->graph->cap);
        delete ctx->graph;
        ctx->graph = nullptr;
    }
    if (ctx->d_step) (void)hipFree(ctx->d_step);
    ctx->d_step = nullptr;
}

int plain_step(fdtd_ctx* ctx, int64_t nsteps) { return run_steps(ctx, nsteps, FDTD_SCHEME_PLAIN); }

int plain_fused_prepare(fdtd_ctx* ctx)
{
    if (ctx->storage != FDTD_FP32)
        return fail(ctx, FDTD_EUNSUPPORTED, "fused plain step: needs FP32 storage");
    const size_t bytes = (size_t)ctx->ncell * sizeof(float);
    for (int c = 0; c < 6; ++c)
        if (!ctx->alt[c]) {
            hipError_t e = hipMalloc(&ctx->alt[c], bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                ctx->alt[c] = nullptr;
                return fail(ctx, FDTD_ENOMEM, "fused plain step: second field set does not fit");
            }
        }
    return FDTD_OK;
}

int plain_fused_step(fdtd_ctx* ctx, int64_t nsteps)
{
    int rc = plain_fused_prepare(ctx);
    if (rc) return rc;
    return run_steps(ctx, nsteps, FDTD_SCHEME_PLAIN_FUSED);
}

}  // namespace fdtd
