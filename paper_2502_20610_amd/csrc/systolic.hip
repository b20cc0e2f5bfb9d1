// Systolic scheme: one persistent launch per fdtd_step() call.
//
// Method (paper, Sections 3 and 4): the grid is covered by subdomain tiles
// that stay resident on chip for a band of K steps.  Every step a tile moves
// one cell along the x-y-z-t diagonal, so every dependency between tiles
// points one way (upwind = +x, +y, +z); a tile only exchanges the faces of its
// subdomain with its neighbours, through device memory, and waits on its
// seven upwind neighbours' progress counters instead of a grid-wide barrier.
// E is updated before H in every step (caption of Fig. 7), and the update
// equations are exactly those of the plain scheme, so the result is the same
// FP32 value bit for bit.
//
// MI355X mapping (one workgroup = one tile):
//   * z: 16 slots on the 16 lanes of a DPP row; the +-1 z neighbour is a
//     row_ror:1 / row_ror:15 operand modifier of the consuming VALU op;
//   * y: 4 rows per wavefront x NW wavefronts = 4*NW slots; the +-1 y
//     neighbour goes through LDS;
//   * x: 16 slots in registers per lane (12 or 20 for the 11- and 19-wide
//     tiles; the 19-wide one holds each cell's material index instead of its
//     three coefficients); moving the tile one cell along x is a compile-time
//     renaming (results of register j are written to j-1), so the x
//     neighbour is a plain register operand.
//   Each axis holds W+1 slots for W updated cells: the extra slot is the
//   layer below the tile (H needed by the E half-step), then receives the
//   layer above it from the upwind neighbours (E needed by the H half-step,
//   then the state of the cells that enter the tile).  Slots are addressed
//   modulo 16 on y and z, so cells never move between lanes.
//
// Faces: after each half-step a tile publishes the first layer of its
// subdomain (E and H; the z face also the coefficients, or the index) into
// per-ticket face rings, one per face orientation, laid out so that every
// face is one contiguous block per component.  On grids without periodic
// axes a step publishes one progress level, once its stores have completed
// behind the next half-step's work; periodic rings, whose tiles wait on each
// other in a cycle, publish after each half-step.  A consumer assembles its forward shell
// from up to seven upwind producers (edges and the corner come from the
// diagonal neighbours).  The field arrays are read only when a band starts
// and written only when it ends, so within a band every hand-off keeps full
// precision whatever the arrays store.  A ring slot is reused R tickets
// later, after its occupant's consumers have finished with it.
//
// Schedule: tickets (band, tile) in topological order (bands in order; in a
// band, tiles by depth below the most upwind corner).  Workgroups take
// tickets from an atomic counter; every wait targets an earlier ticket or a
// tile of the same periodic ring group (which must be resident together),
// so the schedule cannot deadlock.  Waits are bounded: on expiry the kernel
// raises the error word and drains.
//
// On PEC axes cells outside the grid are ghosts that read as +0, which
// reproduces the closed box of the periodic-index definition; on periodic
// axes the tiles form rings and positions wrap.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <vector>

#include "fdtd_internal.h"
#include "plan.h"

namespace fdtd {

namespace {

constexpr int PX = 16, PZ = 16;         // slots along x (registers) and z (lanes)
constexpr int WX = PX - 1, WZ = PZ - 1; // updated cells along x and z
constexpr int WX_LOSSY = 11;              // updated cells along x with conductivity
constexpr int WX_WIDE = 19;               // updated cells along x of the wide tile
constexpr unsigned kOOB = 0xFFFFFFF0u;  // buffer offset that reads 0 / drops stores
constexpr int kErrTimeout = 2;          // error-word bit: a bounded wait expired

// longest band: the per-band source samples are staged in LDS
constexpr int kMaxBand = 64;


// One simulation of a launch (a launch advances one or several independent
// simulations; every ticket names its simulation).
struct SimArgs {
    float* f[6];
    const float* cE[3];
    const float* ca[3];  // conductive decay per cell (conductive variant only)
    float cH;
    int nx, ny, nz;
    unsigned esize;    // bytes per stored element (4, or 2 with FP16 storage)
    const int* band;   // per band: alo ahi blo bhi clo chi tix_off pad (tix_off into the launch's table)
    long long step0;
    const DevSource* src;
    int nsrc;
    int per[3];  // periodic axis: tiles form a ring, positions wrap
    int L[3];    // tiles of the ring on a periodic axis
    int wr[3];   // updated cells of the ring's last (ragged) tile
    int K;       // steps per band of this simulation
    float sc[6], isc[6];  // FP16 storage: field scale 2^e_c and its inverse
    const unsigned* mid;  // material index per cell (material variant only)
    const float* mtab;    // material table: kMaxMaterials x (cEx, cEy, cEz)
};

struct SysArgs {
    const SimArgs* sims;
    const int* tsim;   // simulation of each ticket; null when there is one
    const int4* tickets;  // (band, a, b, c)
    int nt;
    const int* tix;    // ticket index of (band, tile)
    unsigned* progress;  // per ticket: last completed half-step level
    float* ring[6];  // face rings: x, y, z faces (E, H); z-, x-, y-face coefficients
    unsigned ring_bytes[6];
    int R, Kmax;   // ring slots; the longest band (the ring's slot stride)
    int nsteps;
    unsigned* counter;
    int* error;
    long long spin_limit;
};

// A simulation record read word by word into scalar registers (the record is
// the same for every lane; the compiler cannot see that from a global load).
__device__ __forceinline__ SimArgs load_sim(const SimArgs* p)
{
    static_assert(sizeof(SimArgs) % 4 == 0, "record of whole words");
    SimArgs s;
    const int* src = reinterpret_cast<const int*>(p);
    int* dst = reinterpret_cast<int*>(&s);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(SimArgs) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return s;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// Cache policy of the accesses to data shared between workgroups (field
// arrays, face ring): with kDev = 16 (the "sc1" bit, device scope) every load
// and store is coherent across the XCDs by itself, so publishing only has to
// wait for the stores to complete and waiting only has to observe the flag.
// With 0 the accesses are cached normally and the flag store/load carry
// agent-scope release/acquire fences (L2 write-back / invalidate).
template <int POL>
__device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, POL));
}

template <int POL>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, POL);
}

// FP16 storage: a binary16 element read as FP32, and an FP32 value stored
// rounded to binary16 (round to nearest even).
template <int POL>
__device__ __forceinline__ float bld16(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return (float)__builtin_bit_cast(_Float16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, POL));
}

template <int POL>
__device__ __forceinline__ void bst16(__amdgpu_buffer_rsrc_t r, unsigned off, float v)
{
    // the empty asm keeps the conversion a plain v_cvt_f16_f32 (a preceding
    // multiply folded into v_fma_mix with a +0 addend would turn -0 into +0)
    asm volatile("" : "+v"(v));
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, (int)off, 0, POL);
}

// Value of the lane (zs - 1) mod 16 / (zs + 1) mod 16 of the same DPP row.
__device__ __forceinline__ float from_zm(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x121, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_zp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x12F, 0xF, 0xF, false));
}

template <typename T>
__device__ __forceinline__ unsigned lds_offset(T* p)
{
    return (unsigned)(unsigned long long)(__attribute__((address_space(3))) T*)(p);
}

// Asynchronous load of one dword per lane from a buffer straight into LDS at
// lds + 4 * lane (out-of-range offsets write 0).  Issued as inline assembly
// so that the compiler does not hold later LDS accesses of unrelated arrays
// behind it; the kernel itself waits (vmcnt(0) and a barrier) before it reads
// the destination.  M0 carries the LDS address; nothing else in this kernel
// uses M0, and every such load sets it first.
template <bool DEV>
__device__ __forceinline__ void dma_dword(__amdgpu_buffer_rsrc_t desc, unsigned lds, unsigned voff)
{
    lds = __builtin_amdgcn_readfirstlane(lds);
    if (DEV)
        asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, 0 offen sc1 lds"
                     :: "s"(lds), "v"(voff), "s"(desc) : "memory");
    else
        asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, 0 offen lds"
                     :: "s"(lds), "v"(voff), "s"(desc) : "memory");
}

// Uniform words read through the scalar data cache (every lane has the same
// address, and the value lands in scalar registers).  Each load completes
// inside its asm statement.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned sload(const void* p)
{
    unsigned v;
    asm volatile("s_load_dword %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(p) : "memory");
    return v;
}
__device__ __forceinline__ v4i sload4(const void* p)
{
    v4i v;
    asm volatile("s_load_dwordx4 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(p) : "memory");
    return v;
}
__device__ __forceinline__ const float* sload_ptr(const void* p)
{
    v2i v;
    asm volatile("s_load_dwordx2 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(p) : "memory");
    return (const float*)(((unsigned long long)(unsigned)v[1] << 32) | (unsigned)v[0]);
}

// A band's record: tile ranges (a0, a1, b0, b1) and (c0, c1, first ticket
// index, -), read through the scalar data cache (the plan does not change
// while the kernel runs), so that testing neighbours against it takes one
// scalar round trip and no vector memory operation.
struct BandRec {
    v4i r0, r1;
};
__device__ __forceinline__ BandRec load_band(const int* bi)
{
    return BandRec{sload4(bi), sload4(bi + 4)};
}
__device__ __forceinline__ int band_has(const BandRec& B, int a, int b, int c)
{
    return a >= B.r0[0] && a <= B.r0[1] && b >= B.r0[2] && b <= B.r0[3] && c >= B.r1[0] && c <= B.r1[1];
}

// An LDS address made opaque at this point of the program, so that the
// per-component destinations derived from it are formed where they are used
// instead of being kept live (in scalar registers) across the step loop.
__device__ __forceinline__ unsigned lds_here(unsigned base)
{
    asm volatile("" : "+s"(base));
    return base;
}

// Workgroup barrier for LDS traffic only: waits for this wavefront's LDS
// operations, not for its outstanding global loads (__syncthreads() would
// also drain those, which would stall on the prefetched faces).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Tile coordinate v + (-1, 0 or +1) on an axis: wrapped onto the ring of a
// periodic axis.
template <bool PER>
__device__ __forceinline__ int wrap_tile(const SimArgs& P, int d, int v)
{
    if (!PER || !P.per[d]) return v;
    return v >= P.L[d] ? v - P.L[d] : (v < 0 ? v + P.L[d] : v);
}

// Grid position (o + tau) + k on an axis, k in [-1, 16]: U = o + tau (tile
// frame, unbounded), Uw = U mod n (kept only on periodic axes, n >= 16).
// Returns false for ghost positions outside a PEC axis.
template <bool PER>
__device__ __forceinline__ bool axis_pos(int U, int Uw, int n, bool per, int k, int& p)
{
    if (PER && per) {
        int q = Uw + k;
        q = q >= n ? q - n : q;
        p = q < 0 ? q + n : q;
        return true;
    }
    p = U + k;
    return (unsigned)p < (unsigned)n;
}

// Ticket index of tile (a, b, c) of the band whose record is B (the tile
// must be in the band: band_has).
__device__ __forceinline__ int ticket_of(const SysArgs& A, const BandRec& B, int a, int b, int c)
{
    return A.tix[B.r1[2] + ((a - B.r0[0]) * (B.r0[3] - B.r0[2] + 1) + (b - B.r0[2])) * (B.r1[1] - B.r1[0] + 1) +
                 (c - B.r1[0])];
}

// Ticket indices of the tiles (a, b, c) + s * (d & 1, (d >> 1) & 1, (d >> 2) & 1),
// s = +1 (upwind corner) or -1 (downwind), in the band whose record is B: lane
// d = lane & 7 of each wavefront looks up one direction, so that the eight
// lookups cost one round trip instead of eight dependent ones.  Every lane
// returns its own direction's ticket, or -1 when the band lacks that tile;
// readlane(v, d) gives direction d.
template <bool PER>
__device__ __forceinline__ int corner_tickets(const SysArgs& A, const SimArgs& P, const BandRec& B, int a,
                                              int b, int c, int s)
{
    const int d = (int)(threadIdx.x & 7);
    const int ua = wrap_tile<PER>(P, 0, a + s * (d & 1)), ub = wrap_tile<PER>(P, 1, b + s * ((d >> 1) & 1)),
              uc = wrap_tile<PER>(P, 2, c + s * ((d >> 2) & 1));
    return band_has(B, ua, ub, uc) ? ticket_of(A, B, ua, ub, uc) : -1;
}

// Set the tile's progress counter (release): every wavefront has completed
// the global stores the new level covers, and passed a barrier since.
template <bool DEV>
__device__ __forceinline__ void set_flag(const SysArgs& A, int me, unsigned v)
{
    if (threadIdx.x == 0) {
        if (!DEV) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(A.progress + me, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Make this workgroup's global stores visible at device scope, then set the
// tile's progress counter.
template <bool DEV>
__device__ __forceinline__ void publish(const SysArgs& A, int me, unsigned v)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    set_flag<DEV>(A, me, v);
}


// Complete this workgroup's outstanding loads into LDS and make them visible
// to every wavefront.
__device__ __forceinline__ void complete_loads()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// Complete every vector memory operation of this wavefront except the last N
// it issued, then a workgroup barrier.  The vector memory counter retires in
// issue order (loads, stores and loads into LDS alike), so with N = the number
// of stores issued since a group of loads into LDS, those loads have landed
// and every earlier store has completed, while the N recent stores may still
// be in flight.  N must not exceed the operations actually issued since.
template <int N>
__device__ __forceinline__ void complete_all_but()
{
    static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" :: "n"(N) : "memory");
}

// Barrier of the progress waits.  With device-scope accesses (DEV) only the
// LDS words and the execution order need it: the polled counters are used in
// registers, and the data they release is read after the barrier with
// device-scope loads, so outstanding global operations (a box load, a
// half-step's face stores) can stay in flight.  Otherwise a full barrier.
template <bool DEV>
__device__ __forceinline__ void wait_barrier()
{
    if (DEV)
        lds_barrier();
    else
        __syncthreads();
}

// Wait until every listed tile's counter is >= target (acquire).  Lanes
// 0..n-1 of the first wavefront poll one counter each.  Returns false (on
// every thread) if a wait expired or another workgroup raised the error.
template <bool DEV>
__device__ __forceinline__ bool wait_tiles(const SysArgs& A, const int (&idx)[8], int n,
                                           unsigned target, int* s_abort, unsigned* s_min)
{
    const int tid = threadIdx.x;
    unsigned v = 0xFFFFFFFFu;  // (lanes that poll nothing)
    if (tid < n) {
        int my = idx[0];
#pragma unroll
        for (int k = 1; k < 8; ++k)
            if (tid == k) my = idx[k];
        unsigned* p = A.progress + my;
        long long it = 0;
        while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target) {
            if (++it > A.spin_limit) {
                atomicOr(A.error, kErrTimeout);
                *s_abort = 1;
                break;
            }
            if ((it & 255) == 0 && (__hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout)) {
                *s_abort = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!DEV) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // The lowest progress seen bounds every later wait of this ticket: lane 0
    // of the first wavefront writes the minimum over the polling lanes.  (The
    // workgroup reads *s_min right after this function's barrier, into a
    // register; successive calls alternate between two words, so the next
    // call's barrier separates that read from the next write to the word.)
    if (s_min && tid < 64) {
        unsigned m = v;
#pragma unroll
        for (int k = 1; k < 8; ++k) m = min(m, (unsigned)__builtin_amdgcn_readlane((int)v, k));
        if (tid == 0) *s_min = m;
    }
    wait_barrier<DEV>();
    return *s_abort == 0;
}

// The ticket's waits before its box load, as one poll: each lane of the first
// wavefront with my >= 0 waits until tile my's counter is >= target (acquire).
// Lanes 1..7 are the upwind neighbours' (target 0: one read); the minimum of
// what they read goes to *s_min.  Returns false (on every thread) if a wait
// expired or another workgroup raised the error.
template <bool DEV>
__device__ __forceinline__ bool wait_lanes(const SysArgs& A, int my, unsigned target, int* s_abort,
                                           unsigned* s_min)
{
    const int tid = threadIdx.x;
    unsigned v = 0xFFFFFFFFu;  // (lanes that poll nothing)
    if (tid < 64 && my >= 0) {
        unsigned* p = A.progress + my;
        long long it = 0;
        while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target) {
            if (++it > A.spin_limit) {
                atomicOr(A.error, kErrTimeout);
                *s_abort = 1;
                break;
            }
            if ((it & 255) == 0 && (__hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout)) {
                *s_abort = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!DEV) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (tid < 64) {
        unsigned m = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 1; k < 8; ++k) m = min(m, (unsigned)__builtin_amdgcn_readlane((int)v, k));
        if (tid == 0) *s_min = m;
    }
    wait_barrier<DEV>();
    return *s_abort == 0;
}

template <int NW, bool DEV, bool PER, bool LOSSY, bool F16, bool MAT, int XW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void systolic_kernel(SysArgs A)
{
    // XW: updated cells of the tile along x (registers): 15; 11 with
    // conductivity (which frees the registers of the per-cell decay ca) or
    // when asked for; 19 with material indices held in registers
    static_assert(XW == WX || XW == WX_LOSSY || XW == WX_WIDE, "tile widths 15, 11, 19");
    static_assert(!LOSSY || XW == WX_LOSSY, "conductive grids: the 11-wide tile");
    static_assert(!(XW == WX_LOSSY && F16), "11-wide tile: FP32 storage only");
    // MAT: the coefficients enter as per-cell material indices into a table
    // (lossless grids).  IDR (the wide tile): the registers hold each cell's
    // index instead of its three coefficients, and the z face carries it;
    // otherwise the z face carries the values themselves.
    static_assert(!(MAT && LOSSY), "material indices: lossless grids only");
    constexpr bool IDR = XW == WX_WIDE;
    static_assert(!IDR || MAT, "19-wide tile: material indices");
    constexpr int SP = DEV ? 16 : 0;  // cache policy of shared-data accesses
    constexpr int PY = 4 * NW;
    constexpr int WY = PY - 1;
    static_assert(PY == 16, "face staging assumes 16 slots on y and z");
    constexpr int PXk = XW + 1;  // x slots in registers
    constexpr int WXk = XW;
    // staged components: E, H, then cb (cE; with IDR the index), and ca
    // with conductivity
    constexpr int NQA = LOSSY ? 12 : (IDR ? 7 : 9);
    // rows of the y and z faces (one per x slot): whole groups of four, a
    // wavefront's rows; each wavefront handles NG groups (w, w + NW, ...)
    constexpr int YR = (PXk + 3) & ~3;
    constexpr int NG = (YR / 4 + NW - 1) / NW;
    constexpr int FR = YR > 16 ? YR : 16;  // rows of a y or z face block on its ring
    // y-neighbour exchange, two components per half-step
    __shared__ float xch[2][WXk][PY][PZ];
    // incoming faces of the next box: x face [comp][y slot][z slot], y face
    // [comp][x][z slot], z face [comp][x][y slot] (with material indices the
    // x and y faces stage E, H and the index)
    constexpr int NQS = MAT ? 7 : NQA;
    __shared__ float xst[NQS][PY][PZ];
    __shared__ float yst[NQS][YR][PZ];
    __shared__ float4 s_tab[MAT ? kMaxMaterials : 1];  // material table (cEx, cEy, cEz, -)
    __shared__ __attribute__((aligned(16))) float zst[NQA][YR][PY];
    // outgoing faces of the first layer, one half-step's components at a
    // time (E; then H and the coefficients): y face [comp][x][z slot], z face
    // [comp][x][y slot] (with FP16 storage the y face carries the
    // coefficients as well)
    constexpr int NQY = (F16 && !MAT) ? 9 : 6;
    __shared__ float ytr[NQY - 3][YR][PZ];
    __shared__ __attribute__((aligned(16))) float ztr[NQA - 3][YR][PY];
    __shared__ int s_ticket;
    __shared__ int s_abort;
    __shared__ unsigned s_up[2];  // lower bound of the upwind neighbours' progress (alternate calls)
    // point sources kept in LDS (more are read from memory; the wide tile
    // keeps fewer, for its LDS budget)
    constexpr int kLdsSrc = IDR ? 8 : 16;
    __shared__ int s_src[kLdsSrc][4];        // comp, i, j, k
    __shared__ long long s_srcw[kLdsSrc][2]; // first, len
    __shared__ const float* s_srcp[kLdsSrc];
    __shared__ float s_wv[kLdsSrc][kMaxBand];  // their samples for the steps of the current band
    __shared__ unsigned s_srcmask;             // LDS-cached sources this ticket may reach

    const int tid = threadIdx.x;
    // wavefront index, wave-uniform (kept in a scalar register)
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = (tid >> 4) & 3;   // row within the wavefront
    const int ys = tid >> 4;        // y slot: 4 rows per wavefront, NW wavefronts
    const int zs = tid & 15;        // z slot: lane within the DPP row
    if (tid == 0) s_abort = 0;
    // Face rings, one per face orientation: per (slot, local step) the x
    // face holds E and H as [comp][dy][dz] (the producer's own slots), the y
    // face E and H as [comp][x register][dz], the z face E and H as
    // [comp][x register][next-box y slot], and a fourth ring the z face's
    // coefficients (cE, and ca; with IDR the index) in the same layout.  Every ring holds at most
    // six components per (slot, step), which keeps each within the 32-bit
    // offsets of a buffer descriptor on large grids.
    const __amdgpu_buffer_rsrc_t rrx = make_rsrc(A.ring[0], A.ring_bytes[0]);
    const __amdgpu_buffer_rsrc_t rry = make_rsrc(A.ring[1], A.ring_bytes[1]);
    const __amdgpu_buffer_rsrc_t rrz = make_rsrc(A.ring[2], A.ring_bytes[2]);
    const __amdgpu_buffer_rsrc_t rrc = make_rsrc(A.ring[3], A.ring_bytes[3]);
    // FP16 storage: the x and y faces' coefficients travel on rings too (the
    // coefficient arrays are binary16, which the LDS loads cannot convert)
    const __amdgpu_buffer_rsrc_t rrxc = make_rsrc(A.ring[4], A.ring_bytes[4]);
    const __amdgpu_buffer_rsrc_t rryc = make_rsrc(A.ring[5], A.ring_bytes[5]);
    constexpr unsigned ES = F16 ? 2u : 4u;         // bytes per stored field element
    // floats per component of an x face block (16 x 16) and of a y or z
    // face block (FR x 16), the blocks of a (slot, local step) and the bytes
    // per component
    constexpr unsigned rcx = PY * 16u, rcyz = FR * 16u;
    constexpr unsigned step_fx = 6u * rcx, step_fyz = 6u * rcyz;        // E and H
    constexpr unsigned step_c = (unsigned)(NQA - 6) * rcyz;             // the z face's coefficients
    constexpr unsigned step_c3x = 3u * rcx, step_c3y = 3u * rcyz;       // rrxc, rryc
    constexpr unsigned cbx = rcx * 4u, cbyz = rcyz * 4u;
    // Lazy publishing (grids with no periodic axis): a level goes out once
    // its stores have completed in the shadow of later work.  The global
    // stores each half-step issues after its prefetch: the x face (3, with
    // FP16 storage also its 3 coefficients), then the y and z faces.
    constexpr bool LAZY = !PER;
    constexpr int kStoresE = 3 + NG * (3 + 3);
    constexpr int kStoresH = 3 + ((F16 && !MAT) ? 3 : 0) + NG * ((NQY - 3) + (NQA - 3));

    float E[3][PXk], H[3][PXk], C[3][PXk];  // (C unused with IDR)
    unsigned ID[IDR ? PXk : 1];              // material index per cell (IDR)
    float CA[LOSSY ? 3 : 1][PXk];  // conductive decay per cell (unused when lossless)

    int staged_sim = -1, staged_band = -1;  // what the LDS copies below hold
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            // a raised timeout bit (another workgroup's wait expired) drains
            // the grid; the bad-permittivity bit does not stop the update (it
            // is reported at the next synchronising call, as for the plain
            // scheme)
            const int err = __hip_atomic_load(A.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_ticket = (err & kErrTimeout) ? A.nt : (int)atomicAdd(A.counter, 1u);
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_ticket);  // wave-uniform
        if (t >= A.nt || s_abort) break;

        const int4 tk = A.tickets[t];
        const int bnd = tk.x, a = tk.y, b = tk.z, c = tk.w;
        const int t0_ = bnd;  // band index; its steps follow once the record is read
        // this ticket's simulation: arrays, sizes, sources, boundaries
        const int simi = A.tsim ? __builtin_amdgcn_readfirstlane(A.tsim[t]) : 0;
        const SimArgs P = load_sim(A.sims + simi);
        // The LDS copies of the sources, of their samples for the band and of
        // the material table depend on the simulation and the band only: they
        // are kept from this workgroup's previous ticket when both are the same.
        const bool restage = simi != staged_sim || bnd != staged_band;
        staged_sim = simi;
        staged_band = bnd;
        const int t0 = t0_ * P.K;
        const int t1 = min(A.nsteps, t0 + P.K);
        const BandRec bi = load_band(P.band + 8 * bnd);
        const unsigned plane = (unsigned)P.ny * (unsigned)P.nz;
        const bool perx = PER && P.per[0], pery = PER && P.per[1], perz = PER && P.per[2];
        // Field and coefficient descriptors start at the first x-plane the
        // ticket can touch: on a PEC x axis every position it reads or writes
        // lies in [ox + t0, ox + t1 + 16), so offsets stay far below the
        // 32-bit limit even for arrays of 4 GiB.  A periodic x axis wraps over
        // the whole array, which it addresses from its start (such grids are
        // limited to arrays below 4 GiB).
        const int xlo = perx ? 0 : max(0, a * WXk + t0);
        const unsigned long long ebase = (unsigned long long)xlo * plane;
        const unsigned rbytes = (unsigned)min(((unsigned long long)P.nx * plane - ebase) * ES,
                                              0xFFFFFF00ull);
        __amdgpu_buffer_rsrc_t rf[6], rc[3];
#pragma unroll
        for (int q = 0; q < 6; ++q) rf[q] = make_rsrc((const char*)P.f[q] + ebase * ES, rbytes);
#pragma unroll
        for (int q = 0; q < 3; ++q) rc[q] = make_rsrc((const char*)P.cE[q] + ebase * ES, rbytes);
        __amdgpu_buffer_rsrc_t rid;
        if (MAT)
            rid = make_rsrc((const char*)P.mid + ebase * 4ull,
                            (unsigned)min(((unsigned long long)P.nx * plane - ebase) * 4ull, 0xFFFFFF00ull));
        __amdgpu_buffer_rsrc_t rca[3];
        if (LOSSY) {
#pragma unroll
            for (int q = 0; q < 3; ++q) rca[q] = make_rsrc((const char*)P.ca[q] + ebase * 4ull, rbytes);
        }
        const float cH = P.cH;
        if (restage) {
            if (tid < min(P.nsrc, kLdsSrc)) {
                const DevSource sq = P.src[tid];
                s_src[tid][0] = sq.comp;
                s_src[tid][1] = sq.i;
                s_src[tid][2] = sq.j;
                s_src[tid][3] = sq.k;
                s_srcw[tid][0] = sq.first;
                s_srcw[tid][1] = sq.len;
                s_srcp[tid] = sq.wave;
            }
            if (MAT)
                for (int i = tid; i < kMaxMaterials; i += 64 * NW)
                    s_tab[i] = make_float4(P.mtab[3 * i], P.mtab[3 * i + 1], P.mtab[3 * i + 2], 0.f);
            __syncthreads();
        }
        const int me = t;  // progress counters are per ticket
        const int ox = a * WXk, oy = b * WY, oz = c * WZ;

        // upwind neighbours that exist in this band, and the ring slot of
        // each (d: bit 0 = +x, bit 1 = +y, bit 2 = +z; -1 when absent): lane
        // d (mod 8) of every wavefront holds direction d's slot in slv, which
        // a lane's choice of producer reads back with a cross-lane permute.
        // (Not an array: a per-lane choice among the elements of an array can
        // become a load from scratch memory, whose wait would drain the
        // vector memory counter in every half-step.)
        int ups[8];
        int nup = 0;
        const int upv = corner_tickets<PER>(A, P, bi, a, b, c, 1);
        const int slv = upv >= 0 ? upv % A.R : -1;
        const int su4 = __builtin_amdgcn_readlane(slv, 4);  // the z face's producer (wavefront-uniform)
#pragma unroll
        for (int d = 1; d < 8; ++d) {
            const int pi = __builtin_amdgcn_readlane(upv, d);
            if (pi >= 0) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k == nup) ups[k] = pi;
                ++nup;
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k >= nup) ups[k] = me;

        // The waits before the box load, as one poll by the first wavefront:
        // lanes 8..15 wait for the band start (this tile and its upwind
        // neighbours finished the previous band), lanes 16..23 for the ring
        // slot's reuse (its previous occupant has finished writing it and the
        // occupant's consumers, its downwind neighbours, have finished reading
        // it), and lanes 1..7 read the upwind progress once.  The lookups of
        // the three lists are independent loads, in flight together.
        const int slot = t % A.R;
        const int lane8 = tid & 7, lgrp = (tid & 63) >> 3;
        int bv = -1, cv = -1;
        unsigned pend = 0u;
        if (bnd > 0) bv = corner_tickets<PER>(A, P, load_band(P.band + 8 * (bnd - 1)), a, b, c, 1);
        if (t >= A.R) {
            const int4 pk = A.tickets[t - A.R];
            const SimArgs PP = load_sim(A.sims + (A.tsim ? __builtin_amdgcn_readfirstlane(A.tsim[t - A.R]) : 0));
            pend = 2u * (unsigned)min(A.nsteps, (pk.x + 1) * PP.K);
            const int cd = corner_tickets<PER>(A, PP, load_band(PP.band + 8 * pk.x), pk.y, pk.z, pk.w, -1);
            cv = lane8 ? cd : t - A.R;
        }
        int myw = -1;
        unsigned tgw = 0u;
        if (lgrp == 0) {
            myw = lane8 ? upv : -1;
        } else if (lgrp == 1) {
            myw = bv;
            tgw = 2u * (unsigned)t0;
        } else if (lgrp == 2) {
            myw = cv;
            tgw = pend;
        }
        if (!wait_lanes<DEV>(A, myw, tgw, &s_abort, &s_up[0])) break;
        // updated cells per axis (the last tile of a periodic ring is ragged),
        // the lanes that take the forward y and z faces, and the tile frame
        // origin modulo n on periodic axes
        const int wxr = (perx && a == P.L[0] - 1) ? P.wr[0] : WXk;
        const int wyr = (pery && b == P.L[1] - 1) ? P.wr[1] : WY;
        const int wzr = (perz && c == P.L[2] - 1) ? P.wr[2] : WZ;
        const int fy = (wyr + 1) & (PY - 1), fz = (wzr + 1) & (PZ - 1);
        int Xw = 0, Yw = 0, Zw = 0;
        if (perx) Xw = (ox + t0 + 1) % P.nx;
        if (pery) Yw = (oy + t0 + 1) % P.ny;
        if (perz) Zw = (oz + t0 + 1) % P.nz;

        // ---- load the slot box of step t0 + 1 (lower corner o + t0); the
        //      loads stay in flight through the scalar and LDS work below
        {
            const int by = oy + t0, bz = oz + t0;
            int y, z;
            const bool oky = axis_pos<PER>(by + 1, Yw, P.ny, pery, ((ys - by) & (PY - 1)) - 1, y);
            const bool okz = axis_pos<PER>(bz + 1, Zw, P.nz, perz, ((zs - bz) & (PZ - 1)) - 1, z);
            const bool okyz = oky && okz;
            const unsigned yz = (unsigned)y * (unsigned)P.nz + (unsigned)z;
#pragma unroll
            for (int j = 0; j < PXk; ++j) {
                int x;
                const bool okx = axis_pos<PER>(ox + t0 + 1, Xw, P.nx, perx, j - 1, x);
                const unsigned off = (okyz && okx) ? ((unsigned)(x - xlo) * plane + yz) * ES : kOOB;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (F16) {
                        E[q][j] = bld16<SP>(rf[q], off) * P.sc[q];
                        H[q][j] = bld16<SP>(rf[3 + q], off) * P.sc[3 + q];
                        if (!MAT) C[q][j] = bld16<0>(rc[q], off);
                    } else {
                        E[q][j] = bld<SP>(rf[q], off);
                        H[q][j] = bld<SP>(rf[3 + q], off);
                        if (!MAT) C[q][j] = bld<0>(rc[q], off);
                    }
                    if (LOSSY) CA[q][j] = bld<0>(rca[q], off);
                }
                if (MAT) {
                    // (an index out of the grid reads 0: the (+0, +0, +0) entry; the
                    // index array holds 4 bytes per cell whatever the field storage)
                    const unsigned ioff = (F16 && off != kOOB) ? off * 2u : off;
                    const unsigned id = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(rid, (int)ioff, 0, 0) &
                                        (unsigned)(kMaxMaterials - 1);
                    if (IDR) {
                        ID[j] = id;
                    } else {
                        const float4 t4 = s_tab[id];
                        C[0][j] = t4.x;
                        C[1][j] = t4.y;
                        C[2][j] = t4.z;
                    }
                }
            }
        }
        // (a register copy, the same in every wavefront: every wavefront takes
        // the same branch at each progress check)
        unsigned up_reg = __builtin_amdgcn_readfirstlane(s_up[0]);
        int upar = 1;  // the word of s_up the next wait writes
        // consumers of this tile's x, y and z faces in this band
        const int has_xc = band_has(bi, wrap_tile<PER>(P, 0, a - 1), b, c);
        const int has_yc = band_has(bi, a, wrap_tile<PER>(P, 1, b - 1), c);
        const int has_consumer = band_has(bi, a, b, wrap_tile<PER>(P, 2, c - 1));

        // ---- the band's samples of the LDS-cached sources (step tau reads
        //      sample step0 + tau - 1 - first; the range test is repeated at use)
        {
            const int nl = min(P.nsrc, kLdsSrc);
            for (int i = restage ? tid : nl * kMaxBand; i < nl * kMaxBand; i += 64 * NW) {
                const int q = i / kMaxBand, l = i % kMaxBand;
                const long long m = P.step0 + t0 + l - s_srcw[q][0];
                s_wv[q][l] = (l < t1 - t0 && m >= 0 && m < s_srcw[q][1]) ? s_srcp[q][m] : 0.f;
            }
            // Sources that can fall inside this tile during the band: on a PEC
            // axis the cell is inside B_tau for tau in [p - o - w + 1, p - o];
            // periodic axes are not narrowed.  The test at use stays exact.
            if (tid == 0) s_srcmask = 0u;
            lds_barrier();
            if (tid < nl) {
                int lo = t0 + 1, hi = t1;
                const int p3[3] = {s_src[tid][1], s_src[tid][2], s_src[tid][3]};
                const int o3[3] = {ox, oy, oz}, w3[3] = {wxr, wyr, wzr};
                const bool per3[3] = {perx, pery, perz};
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (!per3[d]) {
                        lo = max(lo, p3[d] - o3[d] - w3[d] + 1);
                        hi = min(hi, p3[d] - o3[d]);
                    }
                // and the waveform covers some of those steps
                const long long first = s_srcw[tid][0], len = s_srcw[tid][1];
                lo = (int)max((long long)lo, first + 1 - P.step0);
                hi = (int)min((long long)hi, first + len - P.step0);
                if (lo <= hi) atomicOr(&s_srcmask, 1u << tid);
            }
        }
        lds_barrier();  // (s_srcmask and the samples are complete)

        // The box has landed before the step loop (a wait the compiler sees:
        // left to its own accounting, loads still in flight at the loop's
        // entry would make it drain the vector memory counter inside the
        // loop on every step).
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)

        // (s_srcmask is complete: the barrier above)
        const unsigned srcmask = __builtin_amdgcn_readfirstlane(s_srcmask);
        bool aborted = false;
        for (int tau = t0 + 1; tau <= t1; ++tau) {
            const int ls = tau - t0 - 1;
            const int by = oy + tau - 1, bz = oz + tau - 1;
            const int dy = (ys - by) & (PY - 1);  // 0: layer below the tile; 1..WY: inside
            const int dz = (zs - bz) & (PZ - 1);
            const int Ux = ox + tau, Uy = oy + tau, Uz = oz + tau;  // frame origin of B_tau
            int y, z;
            const bool oky = axis_pos<PER>(Uy, Yw, P.ny, pery, dy - 1, y);
            const bool okz0 = axis_pos<PER>(Uz, Zw, P.nz, perz, dz - 1, z);
            const bool inB = dy >= 1 && dz >= 1 && dy <= wyr && dz <= wzr;
            const bool okyz = oky && okz0;
            const unsigned yz = (unsigned)y * (unsigned)P.nz + (unsigned)z;
            // offset of this lane's cell at x = Ux + k
            auto off_at = [&](int k) -> unsigned {
                int x;
                const bool okx = axis_pos<PER>(Ux, Xw, P.nx, perx, k, x);
                return (okyz && okx) ? ((unsigned)(x - xlo) * plane + yz) * ES : kOOB;
            };
            // coordinates of this lane in the next box (after the one-cell move)
            const int dy1 = (dy - 1) & (PY - 1), dz1 = (dz - 1) & (PZ - 1);
            int y1, z1;
            const bool oky1 = axis_pos<PER>(Uy, Yw, P.ny, pery, dy1, y1);
            const bool okz1 = axis_pos<PER>(Uz, Zw, P.nz, perz, dz1, z1);
            const bool okyz1 = oky1 && okz1;
            const unsigned yz1 = (unsigned)y1 * (unsigned)P.nz + (unsigned)z1;
            // (slot, local step) index of this tile's faces, and of a producer's
            const unsigned sls = (unsigned)slot * (unsigned)A.Kmax + (unsigned)ls;
            auto sls_of = [&](int sl) { return (unsigned)sl * (unsigned)A.Kmax + (unsigned)ls; };
            // the forward y and z planes of the next box
            int yf, zf, zl;
            const bool oky_f = axis_pos<PER>(Uy, Yw, P.ny, pery, wyr, yf);
            const bool okz_f = axis_pos<PER>(Uz, Zw, P.nz, perz, wzr, zf);
            // z of DPP lane zs in the next box, for the y-face loads
            const bool okz_l = axis_pos<PER>(Uz, Zw, P.nz, perz, (zs - oz - tau) & (PZ - 1), zl);
            (void)zf;

            // Issue the loads of the next box's forward shell for components
            // [Q0, Q0 + NQ) (0..2 = E, 3..5 = H, 6..8 = cE, 9..11 = ca; with
            // material indices 6 = the index) straight into LDS: E and H from
            // the producers' face rings, the coefficients from their arrays
            // (or rings).  Wavefront w loads rows 4w..4w+3 of the x face and
            // the row groups w, w + NW, ... of the y and z faces.
            auto prefetch = [&](auto q0c, auto nqc) {
                constexpr int Q0 = decltype(q0c)::value, NQ = decltype(nqc)::value;
                // x face: rows of the wavefront are y slots, lanes are z
                // slots.  The next box's slots dy1 < wyr, dz1 < wzr are the +x
                // neighbour's cells (its slots dy1 + 1, dz1 + 1); dy1 == wyr
                // (dz1 == wzr) is the first row (column) of the neighbour
                // further along +y (+z).
                int xf;
                const bool okxf = axis_pos<PER>(Ux, Xw, P.nx, perx, wxr, xf);
                const unsigned oxf = (okyz1 && okxf) ? ((unsigned)(xf - xlo) * plane + yz1) * 4u : kOOB;
                const bool fwy = dy1 == wyr, fwz = dz1 == wzr;
                const int sx = __builtin_amdgcn_ds_bpermute((1 | (fwy ? 2 : 0) | (fwz ? 4 : 0)) << 2, slv);
                const bool okxr = okyz1 && okxf && dy1 <= wyr && dz1 <= wzr && sx >= 0;
                const unsigned xin = (unsigned)(fwy ? 1 : dy1 + 1) * 16u + (unsigned)(fwz ? 1 : dz1 + 1);
                const unsigned oxr = (sls_of(sx) * step_fx + xin) * 4u;
                const unsigned oxc = (sls_of(sx) * step_c3x + xin) * 4u;
                const unsigned lxb = lds_offset(&xst[0][4 * w][0]);
#pragma unroll
                for (int q = Q0; q < Q0 + NQ; ++q) {
                    const unsigned lx = lds_here(lxb) + (unsigned)q * (unsigned)sizeof(xst[0]);
                    if (q < 6)
                        dma_dword<DEV>(rrx, lx, okxr ? oxr + (unsigned)q * cbx : kOOB);
                    else if (MAT) {
                        if (q == 6) dma_dword<false>(rid, lx, oxf);  // the material index (one word per cell)
                    } else if (q < 9 && F16)
                        dma_dword<DEV>(rrxc, lx, okxr ? oxc + (unsigned)(q - 6) * cbx : kOOB);
                    else if (q < 9)
                        dma_dword<false>(rc[q - 6], lx, oxf);
                    else if (LOSSY)
                        dma_dword<false>(rca[q - 9], lx, oxf);
                }
                // y face: rows are x registers, lanes are z slots; the +y
                // neighbour's (or, on the forward z lane, the +y+z
                // neighbour's) first y row.  z face: rows are x registers,
                // lanes are y slots, from the +z neighbour's ring slot.
                const bool fwzl = dz1 == wzr;
                const int sy = __builtin_amdgcn_ds_bpermute((2 | (fwzl ? 4 : 0)) << 2, slv);
                int yr;
                const bool okzy = su4 >= 0 && okz_f && zs < WY && axis_pos<PER>(Uy, Yw, P.ny, pery, zs, yr);
#pragma unroll
                for (int k = 0; k < NG; ++k) {
                    const int g = w + NW * k;  // wavefront-uniform
                    if (g >= YR / 4) break;
                    const int j = 4 * g + r;
                    int x;
                    const bool okx = j < WXk && axis_pos<PER>(Ux, Xw, P.nx, perx, j, x);
                    const unsigned oyf = (oky_f && okz_l && okx)
                                             ? (((unsigned)(x - xlo) * (unsigned)P.ny + (unsigned)yf) * (unsigned)P.nz + (unsigned)zl) * 4u
                                             : kOOB;
                    const bool okyr = oky_f && okz_l && okx && dz1 <= wzr && sy >= 0;
                    const unsigned yin = (unsigned)j * 16u + (unsigned)(fwzl ? 1 : dz1 + 1);
                    const unsigned oyr = (sls_of(sy) * step_fyz + yin) * 4u;
                    const unsigned oyc = (sls_of(sy) * step_c3y + yin) * 4u;
                    const bool okz = okzy && okx;
                    const unsigned ozf = (sls_of(su4) * step_fyz + (unsigned)j * 16u + (unsigned)zs) * 4u;
                    const unsigned ozc = (sls_of(su4) * step_c + (unsigned)j * 16u + (unsigned)zs) * 4u;
                    const unsigned lyb = lds_offset(&yst[0][4 * g][0]);
                    const unsigned lzb = lds_offset(&zst[0][4 * g][0]);
#pragma unroll
                    for (int q = Q0; q < Q0 + NQ; ++q) {
                        const unsigned ly = lds_here(lyb) + (unsigned)q * (unsigned)sizeof(yst[0]);
                        const unsigned lz = lds_here(lzb) + (unsigned)q * (unsigned)sizeof(zst[0]);
                        if (q < 6) {
                            dma_dword<DEV>(rry, ly, okyr ? oyr + (unsigned)q * cbyz : kOOB);
                            dma_dword<DEV>(rrz, lz, okz ? ozf + (unsigned)q * cbyz : kOOB);
                        } else {
                            if (MAT) {
                                if (q == 6) dma_dword<false>(rid, ly, oyf);
                            } else if (q < 9 && F16)
                                dma_dword<DEV>(rryc, ly, okyr ? oyc + (unsigned)(q - 6) * cbyz : kOOB);
                            else if (q < 9)
                                dma_dword<false>(rc[q - 6], ly, oyf);
                            else if (LOSSY)
                                dma_dword<false>(rca[q - 9], ly, oyf);
                            dma_dword<DEV>(rrc, lz, okz ? ozc + (unsigned)(q - 6) * cbyz : kOOB);
                        }
                    }
                }
            };
            // Write the staged first-layer faces for components [Q0, Q0+NQ)
            // (z face: [Q0, Q0+NQZ)), staged in LDS from slot 0 on, to memory,
            // after a barrier that makes the LDS writes visible.  Wavefront w
            // writes the row groups w, w + NW, ... (every wavefront issues the
            // same number of stores: rows past the face are dropped, their
            // LDS reads clamped).
            auto store_faces = [&](auto q0c, auto nqc, auto nqzc) {
                constexpr int Q0 = decltype(q0c)::value, NQ = decltype(nqc)::value;
                constexpr int NQZ = decltype(nqzc)::value;
                lds_barrier();
                const int dzl = (zs - oz - tau + 1) & (PZ - 1);
#pragma unroll
                for (int k = 0; k < NG; ++k) {
                    const int j = 4 * (w + NW * k) + r;
                    const int jl = min(j, YR - 1);
                    // y face (the first y row) as [x register][dz]
                    const bool oky_ = has_yc && j < WXk;
                    const unsigned oy_ = (sls * step_fyz + (unsigned)j * 16u + (unsigned)dzl) * 4u;
                    const unsigned oyc_ = (sls * step_c3y + (unsigned)j * 16u + (unsigned)dzl) * 4u;
#pragma unroll
                    for (int q = Q0; q < Q0 + NQ; ++q) {
                        if (q < 6)
                            bst<SP>(rry, oky_ ? oy_ + (unsigned)q * cbyz : kOOB, ytr[q - Q0][jl][zs]);
                        else
                            bst<SP>(rryc, oky_ ? oyc_ + (unsigned)(q - 6) * cbyz : kOOB, ytr[q - Q0][jl][zs]);
                    }
                    // z face as [x register][y slot] (dropped offsets when
                    // there is no consumer: no branch)
                    const bool okz_ = has_consumer && j < WXk;
                    const unsigned oz_ = (sls * step_fyz + (unsigned)j * 16u + (unsigned)zs) * 4u;
                    const unsigned oc_ = (sls * step_c + (unsigned)j * 16u + (unsigned)zs) * 4u;
#pragma unroll
                    for (int q = Q0; q < Q0 + NQZ; ++q) {
                        if (q < 6)
                            bst<SP>(rrz, okz_ ? oz_ + (unsigned)q * cbyz : kOOB, ztr[q - Q0][jl][zs]);
                        else
                            bst<SP>(rrc, okz_ ? oc_ + (unsigned)(q - 6) * cbyz : kOOB, ztr[q - Q0][jl][zs]);
                    }
                }
            };
            auto ensure_up = [&](unsigned level) -> bool {
                if (up_reg >= level) return true;
                const bool ok = wait_tiles<DEV>(A, ups, nup, level, &s_abort, &s_up[upar]);
                up_reg = __builtin_amdgcn_readfirstlane(s_up[upar]);
                upar ^= 1;
                return ok;
            };

            // Before the tile's first cell crosses the lower wall of a PEC
            // axis its box holds ghosts only (+0, loaded out of range), and no
            // grid cell depends on what an update would make of them (the
            // grid cells they touch are PEC-tangential E, whose coefficient
            // is 0): the step skips the updates and the faces (consumers read
            // those positions as ghosts) and keeps the waits and the forward
            // shells, the last of which carry the first grid cells in.  With
            // every register +0, the skipped one-slot renaming changes nothing.
            // (Only in the variant for grids with no periodic axis: the
            // periodic variant, short of registers already, would spill.)
            const bool skip = !PER && (ox + tau + WXk - 1 < 0 || oy + tau + WY - 1 < 0 || oz + tau + WZ - 1 < 0);
            // offset of this lane's cell in the x face ring block
            const unsigned ox_ = (sls * step_fx + (unsigned)dy * 16u + (unsigned)dz) * 4u;

            // ================= E half-step (H frame: register j <-> x = ox+tau-1+j)
            const bool earlyE = up_reg >= 2u * (unsigned)tau - 1u;
            if (earlyE) prefetch(std::integral_constant<int, 0>(), std::integral_constant<int, 3>());
            if (!skip) {
#pragma unroll
                for (int j = 1; j < PXk; ++j) {
                    xch[0][j - 1][ys][zs] = H[2][j];
                    xch[1][j - 1][ys][zs] = H[0][j];
                }
                lds_barrier();
                {
                    const int ysm = (ys - 1) & (PY - 1);
#pragma unroll
                    for (int j = 1; j < PXk; ++j) {
                        const float hz_ym = xch[0][j - 1][ysm][zs];
                        const float hx_ym = xch[1][j - 1][ysm][zs];
                        const float hy_zm = from_zm(H[1][j]);
                        const float hx_zm = from_zm(H[0][j]);
                        // with conductivity the old E decays by ca first (ca = 1
                        // reproduces the lossless update)
                        const float e0 = LOSSY ? CA[0][j] * E[0][j] : E[0][j];
                        const float e1 = LOSSY ? CA[1][j] * E[1][j] : E[1][j];
                        const float e2 = LOSSY ? CA[2][j] * E[2][j] : E[2][j];
                        float c0, c1, c2;
                        if (IDR) {
                            const float4 t4 = s_tab[ID[j]];
                            c0 = t4.x;
                            c1 = t4.y;
                            c2 = t4.z;
                        } else {
                            c0 = C[0][j];
                            c1 = C[1][j];
                            c2 = C[2][j];
                        }
                        const float ex = (e0 + c0 * (H[2][j] - hz_ym)) - c0 * (H[1][j] - hy_zm);
                        const float ey = (e1 + c1 * (H[0][j] - hx_zm)) - c1 * (H[2][j] - H[2][j - 1]);
                        const float ez = (e2 + c2 * (H[1][j] - H[1][j - 1])) - c2 * (H[0][j] - hx_ym);
                        E[0][j - 1] = ex;
                        E[1][j - 1] = ey;
                        E[2][j - 1] = ez;
                        if (IDR) ID[j - 1] = ID[j];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            if (!IDR) C[q][j - 1] = C[q][j];
                            if (LOSSY) CA[q][j - 1] = CA[q][j];
                        }
                    }
                }
            }
            // now E and C registers j <-> x = ox+tau+j (j < WXk); j = WXk stale

            // point sources of this step on cells of the tile (registers are
            // only ever indexed with compile-time constants, so they stay in
            // VGPRs)
            // (the LDS-cached and the remaining sources are read in separate loops
            // so that neither becomes a generic-address load)
#define FDTD_APPLY_SOURCE(comp, si, sj, sk, first, len, sample)                                        \
    {                                                                                               \
        const long long m = P.step0 + tau - 1 - (first);                                            \
        int px = (si) - (perx ? Xw : Ux), py = (sj) - (pery ? Yw : Uy), pz = (sk) - (perz ? Zw : Uz); \
        px += (perx && px < 0) ? P.nx : 0;                                                          \
        py += (pery && py < 0) ? P.ny : 0;                                                          \
        pz += (perz && pz < 0) ? P.nz : 0;                                                          \
        if (m >= 0 && m < (len) && (unsigned)px < (unsigned)wxr && (unsigned)py < (unsigned)wyr &&  \
            (unsigned)pz < (unsigned)wzr) {                                                         \
            const float wv = (sample);                                                              \
            const int lx = (dy == py + 1 && dz == pz + 1) ? px : -1;                                \
            if ((comp) == 0) {                                                                      \
                _Pragma("unroll") for (int j = 0; j < WXk; ++j) E[0][j] = lx == j ? E[0][j] + wv : E[0][j]; \
            } else if ((comp) == 1) {                                                               \
                _Pragma("unroll") for (int j = 0; j < WXk; ++j) E[1][j] = lx == j ? E[1][j] + wv : E[1][j]; \
            } else {                                                                                \
                _Pragma("unroll") for (int j = 0; j < WXk; ++j) E[2][j] = lx == j ? E[2][j] + wv : E[2][j]; \
            }                                                                                       \
        }                                                                                           \
    }
            {
                for (unsigned msk = srcmask; msk; msk &= msk - 1u) {
                    const int q = __builtin_ctz(msk);
                    FDTD_APPLY_SOURCE(s_src[q][0], s_src[q][1], s_src[q][2], s_src[q][3], s_srcw[q][0],
                                      s_srcw[q][1], s_wv[q][ls]);
                }
                for (int q = kLdsSrc; q < P.nsrc; ++q) {
                    // (scalar loads: nothing of this rare loop is left on the
                    // vector memory counter, which the prefetch waits use)
                    const DevSource* sp = P.src + q;
                    const v4i h = sload4(sp);         // comp, i, j, k
                    const v4i fl = sload4(&sp->len);  // len, first
                    const long long len = (long long)(((unsigned long long)(unsigned)fl[1] << 32) | (unsigned)fl[0]);
                    const long long first = (long long)(((unsigned long long)(unsigned)fl[3] << 32) | (unsigned)fl[2]);
                    const float* wave = sload_ptr(&sp->wave);
                    // (the sample's index is clamped into the waveform: the
                    // load sits under a uniform branch but must never stray)
                    FDTD_APPLY_SOURCE(h[0], h[1], h[2], h[3], first, len,
                                      __builtin_bit_cast(float, sload(wave + min(max(m, 0ll), len - 1))));
                }
            }
#undef FDTD_APPLY_SOURCE

            if (!skip) {
                // E of the first x layer of the tile (every lane: slot [dy][dz])
#pragma unroll
                for (int q = 0; q < 3; ++q) bst<SP>(rrx, has_xc ? ox_ + (unsigned)q * cbx : kOOB, E[q][0]);
                if (dy == 1) {
#pragma unroll
                    for (int j = 0; j < WXk; ++j)
#pragma unroll
                        for (int q = 0; q < 3; ++q) ytr[q][j][zs] = E[q][j];
                }
                if (dz == 1) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int j = 0; j < WXk; ++j) ztr[q][j][dy1] = E[q][j];
                }
                store_faces(std::integral_constant<int, 0>(), std::integral_constant<int, 3>(), std::integral_constant<int, 3>());
                // (lazy: the early prefetch lands; this half-step's stores may fly on)
                if (LAZY && earlyE) complete_all_but<kStoresE>();
            } else if (LAZY && earlyE) {
                complete_all_but<0>();
            }
            if (!LAZY) {
                // publish (which also completes an early prefetch); a late
                // prefetch waits for the upwind neighbours only after this
                // tile's own flag is out, since on a periodic ring they wait
                // on it in turn
                publish<DEV>(A, me, 2u * (unsigned)tau - 1u);
                if (!earlyE) {
                    if (!ensure_up(2u * (unsigned)tau - 1u)) {
                        aborted = true;
                        break;
                    }
                    prefetch(std::integral_constant<int, 0>(), std::integral_constant<int, 3>());
                    complete_loads();
                }
            } else {
                // Without periodic axes no tile waits on a tile downwind of it,
                // so the level of the previous step (2 tau - 2) is published
                // here, once its stores have completed behind this half-step's
                // work, and the E level of this step is not published on its
                // own (the next full level covers it).
                if (!earlyE) {
                    if (!ensure_up(2u * (unsigned)tau - 1u)) {
                        aborted = true;
                        break;
                    }
                    prefetch(std::integral_constant<int, 0>(), std::integral_constant<int, 3>());
                    complete_loads();
                }
                if (tau > t0 + 1) set_flag<DEV>(A, me, 2u * (unsigned)tau - 2u);
            }

            // forward shell's E^tau into the registers
            if (dy == fy) {
#pragma unroll
                for (int j = 0; j < WXk; ++j)
#pragma unroll
                    for (int q = 0; q < 3; ++q) E[q][j] = yst[q][j][zs];
            } else if (dz == fz) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int j = 0; j < WXk; ++j) E[q][j] = zst[q][j][dy1];
            }
            if (!PER || wxr == WXk) {
#pragma unroll
                for (int q = 0; q < 3; ++q) E[q][WXk] = xst[q][ys][zs];
            } else {
                // ragged tile of a periodic ring: the x face enters at slot wxr
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float v = xst[q][ys][zs];
#pragma unroll
                    for (int j = 0; j < WXk; ++j) E[q][j] = j == wxr ? v : E[q][j];
                }
            }

            // ================= H half-step (E frame: register j <-> x = ox+tau+j)
            const bool earlyH = tau < t1 && up_reg >= 2u * (unsigned)tau;
            if (earlyH) prefetch(std::integral_constant<int, 3>(), std::integral_constant<int, NQA - 3>());
            if (!skip) {
#pragma unroll
                for (int j = 0; j < WXk; ++j) {
                    xch[0][j][ys][zs] = E[2][j];
                    xch[1][j][ys][zs] = E[0][j];
                }
                lds_barrier();
                {
                    const int ysp = (ys + 1) & (PY - 1);
#pragma unroll
                    for (int j = 0; j < WXk; ++j) {
                        const float ez_yp = xch[0][j][ysp][zs];
                        const float ex_yp = xch[1][j][ysp][zs];
                        const float ey_zp = from_zp(E[1][j]);
                        const float ex_zp = from_zp(E[0][j]);
                        const float hx = (H[0][j + 1] - cH * (ez_yp - E[2][j])) + cH * (ey_zp - E[1][j]);
                        const float hy = (H[1][j + 1] - cH * (ex_zp - E[0][j])) + cH * (E[2][j + 1] - E[2][j]);
                        const float hz = (H[2][j + 1] - cH * (E[1][j + 1] - E[1][j])) + cH * (ex_yp - E[0][j]);
                        H[0][j] = hx;
                        H[1][j] = hy;
                        H[2][j] = hz;
                    }
                }
                // now H registers j <-> x = ox+tau+j as well

                // H (and, on the z face, the coefficients) of the first layer
#pragma unroll
                for (int q = 0; q < 3; ++q) bst<SP>(rrx, has_xc ? ox_ + (unsigned)(3 + q) * cbx : kOOB, H[q][0]);
                if (F16 && !MAT) {
                    const unsigned oxc_ = (sls * step_c3x + (unsigned)dy * 16u + (unsigned)dz) * 4u;
#pragma unroll
                    for (int q = 0; q < 3; ++q) bst<SP>(rrxc, has_xc ? oxc_ + (unsigned)q * cbx : kOOB, C[q][0]);
                }
                if (dy == 1) {
#pragma unroll
                    for (int j = 0; j < WXk; ++j)
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            ytr[q][j][zs] = H[q][j];
                            if (F16 && !MAT) ytr[3 + q][j][zs] = C[q][j];
                        }
                }
                if (dz == 1) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int j = 0; j < WXk; ++j) {
                            ztr[q][j][dy1] = H[q][j];
                            if (IDR) {
                                if (q == 0) ztr[3][j][dy1] = __builtin_bit_cast(float, ID[j]);
                            } else {
                                ztr[3 + q][j][dy1] = C[q][j];
                            }
                            if (LOSSY) ztr[6 + q][j][dy1] = CA[q][j];
                        }
                }
                store_faces(std::integral_constant<int, 3>(), std::integral_constant<int, NQY - 3>(),
                            std::integral_constant<int, NQA - 3>());
                // (lazy: the early prefetch lands; the level 2 tau goes out in
                // the next step's E half)
                if (LAZY && earlyH) complete_all_but<kStoresH>();
            } else if (LAZY && earlyH) {
                complete_all_but<0>();
            }
            if (tau == t1 && inB) {
                // band end: the whole subdomain goes back to the field arrays
#pragma unroll
                for (int j = 0; j < WXk; ++j) {
                    const unsigned o = j < wxr ? off_at(j) : kOOB;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if (F16) {
                            bst16<SP>(rf[q], o, E[q][j] * P.isc[q]);
                            bst16<SP>(rf[3 + q], o, H[q][j] * P.isc[3 + q]);
                        } else {
                            bst<SP>(rf[q], o, E[q][j]);
                            bst<SP>(rf[3 + q], o, H[q][j]);
                        }
                    }
                }
            }
            if (!LAZY || tau == t1)
                publish<DEV>(A, me, 2u * (unsigned)tau);
            else
                asm volatile("" ::: "memory");  // (keeps memory accesses on their side, as publish does)
            if (tau == t1) break;
            // Past a PEC wall: once the box of the next step lies wholly past
            // the upper wall of a PEC axis (the tile only moves further out),
            // nothing the tile would compute reaches a grid cell, and its
            // consumers read those positions as ghosts (+0, out-of-range
            // loads).  The band-end level releases everything that waits on
            // it: its consumers, the next occupant of its ring slot and its
            // own next band.  (publish completes every load in flight.)
            if ((!perx && ox + tau + 1 >= P.nx) || (!pery && oy + tau + 1 >= P.ny) ||
                (!perz && oz + tau + 1 >= P.nz)) {
                publish<DEV>(A, me, 2u * (unsigned)t1);
                break;
            }
            if (!earlyH) {
                if (!ensure_up(2u * (unsigned)tau)) {
                    aborted = true;
                    break;
                }
                prefetch(std::integral_constant<int, 3>(), std::integral_constant<int, NQA - 3>());
                complete_loads();
            }

            // forward shell's H^(tau+1/2) and coefficients (or indices) into
            // the registers
            auto tab = [&](unsigned id, int q) -> float {
                const float4 t4 = s_tab[id];
                return q == 0 ? t4.x : (q == 1 ? t4.y : t4.z);
            };
            if (dy == fy) {
#pragma unroll
                for (int j = 0; j < WXk; ++j) {
                    const unsigned id = MAT ? (__builtin_bit_cast(unsigned, yst[6][j][zs]) & (unsigned)(kMaxMaterials - 1)) : 0u;
                    if (IDR) ID[j] = id;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        H[q][j] = yst[3 + q][j][zs];
                        if (!IDR) C[q][j] = MAT ? tab(id, q) : yst[6 + q][j][zs];
                        if (LOSSY) CA[q][j] = yst[9 + q][j][zs];
                    }
                }
            } else if (dz == fz) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int j = 0; j < WXk; ++j) {
                        H[q][j] = zst[3 + q][j][dy1];
                        if (IDR) {
                            if (q == 0) ID[j] = __builtin_bit_cast(unsigned, zst[6][j][dy1]) & (unsigned)(kMaxMaterials - 1);
                        } else {
                            C[q][j] = zst[6 + q][j][dy1];
                        }
                        if (LOSSY) CA[q][j] = zst[9 + q][j][dy1];
                    }
            }
            const unsigned xid = MAT ? (__builtin_bit_cast(unsigned, xst[6][ys][zs]) & (unsigned)(kMaxMaterials - 1)) : 0u;
            if (!PER || wxr == WXk) {
                if (IDR) ID[WXk] = xid;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    H[q][WXk] = xst[3 + q][ys][zs];
                    if (!IDR) C[q][WXk] = MAT ? tab(xid, q) : xst[6 + q][ys][zs];
                    if (LOSSY) CA[q][WXk] = xst[9 + q][ys][zs];
                }
            } else {
                if (IDR) {
#pragma unroll
                    for (int j = 0; j < WXk; ++j) ID[j] = j == wxr ? xid : ID[j];
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float vh = xst[3 + q][ys][zs], vc = (MAT && !IDR) ? tab(xid, q) : (IDR ? 0.f : xst[6 + q][ys][zs]);
                    const float va = LOSSY ? xst[9 + q][ys][zs] : 0.f;
#pragma unroll
                    for (int j = 0; j < WXk; ++j) {
                        H[q][j] = j == wxr ? vh : H[q][j];
                        if (!IDR) C[q][j] = j == wxr ? vc : C[q][j];
                        if (LOSSY) CA[q][j] = j == wxr ? va : CA[q][j];
                    }
                }
            }
            if (PER) {
                Xw = (perx && Xw == P.nx - 1) ? 0 : Xw + 1;
                Yw = (pery && Yw == P.ny - 1) ? 0 : Yw + 1;
                Zw = (perz && Zw == P.nz - 1) ? 0 : Zw + 1;
            }
        }
        if (aborted) break;
    }
}

// A member of a batched launch takes the shared launch's timeout bit into its
// own error word (keeping its own bits).
__global__ void or_timeout(int* dst, const int* src)
{
    if (threadIdx.x == 0) {
        const int v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout;
        if (v) atomicOr(dst, v);
    }
}

__global__ void fill_u32(unsigned* p, unsigned v, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

constexpr int kNW = 4;  // wavefronts per tile: tile = 15 x 15 x 15 updated cells

}  // namespace

// Host-side plan of one context's call (plan::Plan) and the launch resources
// of the launches it leads.
struct SystolicState {
    plan::Plan pl;
    uint64_t version = 0;       // bumped whenever the plan is rebuilt
    // launch resources (used when this context leads a launch)
    int4* d_tickets = nullptr;
    int* d_tsim = nullptr;
    int* d_tix = nullptr;
    int* d_band = nullptr;
    SimArgs* d_sims = nullptr;
    unsigned* d_progress = nullptr;
    float* d_ring = nullptr;
    unsigned* d_counter = nullptr;
    SimArgs* h_sims = nullptr;     // pinned staging of the per-simulation records
    hipEvent_t sims_done = nullptr;  // the last upload from h_sims has completed
    size_t cap_tickets = 0, cap_tsim = 0, cap_tix = 0, cap_band = 0, cap_sims = 0, cap_prog = 0;
    int R = 0;
    size_t ring_bytes = 0;
    int sm_count = 0;
    // the uploaded launch plan: which contexts (and plan versions) it covers
    std::vector<const fdtd_ctx*> up_ctx;
    std::vector<uint64_t> up_ver;
    int up_nt = 0, up_D = 1, up_group = 1;
    std::vector<size_t> up_band_off;  // per simulation: offset of its band records
};

namespace {

static_assert(sizeof(plan::Ticket) == sizeof(int4), "tickets upload as int4");

void free_launch(SystolicState* s)
{
    for (void* p : {(void*)s->d_tickets, (void*)s->d_tsim, (void*)s->d_tix, (void*)s->d_band,
                    (void*)s->d_sims, (void*)s->d_progress, (void*)s->d_ring, (void*)s->d_counter})
        if (p) (void)hipFree(p);
    if (s->sims_done) (void)hipEventSynchronize(s->sims_done);
    if (s->h_sims) (void)hipHostFree(s->h_sims);
    if (s->sims_done) (void)hipEventDestroy(s->sims_done);
    s->d_tickets = nullptr;
    s->d_tsim = nullptr;
    s->d_tix = nullptr;
    s->d_band = nullptr;
    s->d_sims = nullptr;
    s->d_progress = nullptr;
    s->d_ring = nullptr;
    s->d_counter = nullptr;
    s->h_sims = nullptr;
    s->sims_done = nullptr;
    s->cap_tickets = s->cap_tsim = s->cap_tix = s->cap_band = s->cap_sims = s->cap_prog = 0;
    s->R = 0;
    s->ring_bytes = 0;
    s->up_ctx.clear();
    s->up_ver.clear();
}

// updated cells along x of a tile of this context: conductive grids use the
// narrower register tile that leaves room for the per-cell decay
// (a lossless FP32 context may ask for the narrow tile too, or for the
// 19-wide one, which needs material indices: FDTD_OPT_TILE_X; without a
// request the launch picks 19 when its members allow it, else 15)
int tile_x(const fdtd_ctx* c)
{
    if (c->ca[0]) return WX_LOSSY;
    if (c->tile_wx == WX_WIDE || c->tile_wx == WX) return c->tile_wx;
    if (c->tile_wx == WX_LOSSY && c->storage == FDTD_FP32) return WX_LOSSY;
    return c->auto_wx == WX_WIDE ? WX_WIDE : WX;  // (the last launch's default)
}

void tile_of(const fdtd_ctx* c, int W[3])
{
    W[0] = tile_x(c);
    W[1] = 4 * kNW - 1;
    W[2] = WZ;
}

void axes_of(const fdtd_ctx* c, int N[3], int per[3])
{
    N[0] = c->nx;
    N[1] = c->ny;
    N[2] = c->nz;
    for (int d = 0; d < 3; ++d) per[d] = c->cfg.bc[d] == FDTD_BC_PERIODIC;
}

// The plan of one context: tiles per band, tickets in topological order.
int build_plan(fdtd_ctx* ctx, SystolicState* s, int nsteps, int K)
{
    int N[3], per[3], W[3];
    axes_of(ctx, N, per);
    tile_of(ctx, W);
    std::string err;
    plan::Order order;
    // FDTD_SYSTOLIC_ORDER="wx,wy,wz[,axis,slab]" overrides the dequeue order
    // (weights of the depth key; optional slabs along one axis)
    if (const char* o = getenv("FDTD_SYSTOLIC_ORDER")) {
        int v[5] = {1, 1, 1, -1, 0};
        const int n = sscanf(o, "%d,%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3], &v[4]);
        if (n >= 3) {
            for (int d = 0; d < 3; ++d) order.w[d] = v[d];
            if (n == 5) {
                order.slab_axis = v[3];
                order.slab = v[4];
            }
        }
    }
    if (!plan::build(N, per, W, nsteps, K, &s->pl, &err, order)) return fail(ctx, FDTD_EUNSUPPORTED, err);
    // unique across contexts, so a launch plan is never mistaken for the plan
    // of another context that happens to reuse an address
    static std::atomic<uint64_t> g_version{0};
    s->version = ++g_version;
    return FDTD_OK;
}

// Band length (steps per residency) for a launch over the contexts cs.  An
// explicit option wins; otherwise the cost model plan::band_cost picks it
// (over several grids, the cell-weighted mean; a batched launch asks per
// grid).
int default_band(fdtd_ctx* const* cs, int n, int64_t nsteps)
{
    if (cs[0]->band_steps > 0) return (int)std::min<int64_t>(std::min(cs[0]->band_steps, kMaxBand), nsteps);
    static const int cand[] = {8, 12, 16, 24, 32, 48, 64};
    int best = (int)std::min<int64_t>(nsteps, 32);
    double best_cost = 1e300;
    for (int K0 : cand) {
        const int K = (int)std::min<int64_t>(K0, nsteps);
        double cost = 0.0, cells = 0.0;
        for (int i = 0; i < n; ++i) {
            int N[3], per[3], W[3];
            axes_of(cs[i], N, per);
            tile_of(cs[i], W);
            cost += plan::band_cost(N, per, W, K) * (double)cs[i]->ncell;
            cells += (double)cs[i]->ncell;
        }
        cost /= cells;
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = K;
        }
        if (K0 >= nsteps) break;
    }
    return best;
}

template <typename T>
int ensure_buffer(fdtd_ctx* ctx, T** p, size_t* cap, size_t n, const char* what)
{
    n = std::max<size_t>(n, 1);
    if (*cap >= n && *p) return FDTD_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, std::string("systolic ") + what + ": " + hipGetErrorString(e));
    }
    *cap = n;
    return FDTD_OK;
}

// Upload the launch plan of the contexts cs (one or several simulations) to
// the lead state L.  Tickets are merged by (band start step, simulation), each
// simulation's tickets keeping their own order: every wait of a ticket still
// targets an earlier ticket of its simulation or its own ring group, ring
// groups stay contiguous, and a producer stays close to its consumers (the
// face ring stays as shallow as for the simulation alone), while the next
// simulation's tickets fill the workgroups a simulation's band tail leaves
// idle.
int upload_plan(fdtd_ctx* lead, SystolicState* L, fdtd_ctx* const* cs, int n)
{
    bool same = (int)L->up_ctx.size() == n && L->d_tickets;
    for (int i = 0; i < n && same; ++i) same = L->up_ctx[i] == cs[i] && L->up_ver[i] == cs[i]->sys->version;
    if (same) return FDTD_OK;
    L->up_ctx.clear();
    L->up_ver.clear();
    std::vector<const plan::Plan*> plans(n);
    for (int i = 0; i < n; ++i) plans[i] = &cs[i]->sys->pl;
    plan::Merged m;
    std::string err;
    if (!plan::merge(plans.data(), n, &m, &err)) return fail(lead, FDTD_EUNSUPPORTED, err);
    const size_t nt = m.tickets.size();
    int rc;
    if ((rc = ensure_buffer(lead, &L->d_tickets, &L->cap_tickets, nt, "tickets")) ||
        (rc = ensure_buffer(lead, &L->d_tsim, &L->cap_tsim, nt, "ticket simulations")) ||
        (rc = ensure_buffer(lead, &L->d_tix, &L->cap_tix, m.tix.size(), "tile table")) ||
        (rc = ensure_buffer(lead, &L->d_band, &L->cap_band, m.band.size(), "band table")) ||
        (rc = ensure_buffer(lead, &L->d_progress, &L->cap_prog, nt, "progress counters")))
        return rc;
    hipError_t e;
    if ((e = hipMemcpy(L->d_tickets, m.tickets.data(), nt * sizeof(int4), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(L->d_tsim, m.tsim.data(), nt * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(L->d_tix, m.tix.data(), m.tix.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(L->d_band, m.band.data(), m.band.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(lead, e, "systolic plan upload");
    for (int i = 0; i < n; ++i) {
        L->up_ctx.push_back(cs[i]);
        L->up_ver.push_back(cs[i]->sys->version);
    }
    L->up_nt = (int)nt;
    L->up_D = m.D;
    L->up_group = m.group;
    L->up_band_off = m.band_off;
    return FDTD_OK;
}

// One persistent launch advancing the contexts cs[0..n) by nsteps each, on
// cs[0]'s stream (the others' streams wait for it and it for them).
// kcap: the longest band an automatic choice may take (lowered when the face
// rings of a longer band would not fit their 32-bit offsets).
// With run = false the launch is only prepared: plans built and uploaded,
// rings and counters allocated, nothing queued.
int launch(fdtd_ctx* const* cs, int n, int64_t nsteps, int kcap = kMaxBand, bool run = true)
{
    fdtd_ctx* lead = cs[0];
    if (nsteps > (int64_t(1) << 24)) return fail(lead, FDTD_EINVAL, "systolic: at most 2^24 steps per call");
    // one kernel variant per launch: all members conductive or none, and
    // all with the same storage format
    const bool lossy = lead->ca[0] != nullptr;
    const bool h16 = lead->storage == FDTD_FP16_STORAGE;
    for (int i = 1; i < n; ++i) {
        if ((cs[i]->ca[0] != nullptr) != lossy)
            return fail(lead, FDTD_EUNSUPPORTED, "systolic batch: conductive and lossless grids cannot share a launch");
        if ((cs[i]->storage == FDTD_FP16_STORAGE) != h16)
            return fail(lead, FDTD_EUNSUPPORTED, "systolic batch: FP32 and FP16 storage cannot share a launch");
        if (tile_x(cs[i]) != tile_x(lead))
            return fail(lead, FDTD_EUNSUPPORTED, "systolic batch: every member needs the same tile width");
    }
    // synchronisation variant: device-scope accesses (default) or cached
    // accesses with agent-scope fences (FDTD_SYSTOLIC_SYNC=fence)
    const char* sync_env = getenv("FDTD_SYSTOLIC_SYNC");
    const bool dev = !(sync_env && strcmp(sync_env, "fence") == 0);
    // The default tile width: 19 when every member can hold material indices
    // in registers (lossless grids with at most 256 coefficient triples whose
    // periodic x axes, if any, have 20 cells or more), else 15.  A
    // member that asked for a width keeps it (and a batch still needs one
    // width for all).
    bool wide_ok = !lossy && dev;
    for (int i = 0; i < n && wide_ok; ++i)
        wide_ok = cs[i]->use_mat && cs[i]->nmat > 0 && cs[i]->mat_id &&
                  !(cs[i]->cfg.bc[0] == FDTD_BC_PERIODIC && cs[i]->nx < WX_WIDE + 1);
    for (int i = 0; i < n; ++i) cs[i]->auto_wx = wide_ok ? WX_WIDE : WX;
    // band length per simulation: the lead's option for all, else each
    // simulation's own choice of the cost model
    int Kmax = 1;
    for (int i = 0; i < n; ++i) {
        if (!cs[i]->sys) {
            cs[i]->sys = new (std::nothrow) SystolicState();
            if (!cs[i]->sys) return fail(lead, FDTD_ENOMEM, "systolic: host allocation failed");
        }
        SystolicState* si = cs[i]->sys;
        const int K = lead->band_steps > 0 ? default_band(cs, 1, nsteps)
                                           : std::min(kcap, default_band(cs + i, 1, nsteps));
        Kmax = std::max(Kmax, K);
        if (si->pl.nsteps != (int)nsteps || si->pl.K != K || si->pl.wx != tile_x(cs[i])) {
            int rc = build_plan(cs[i], si, (int)nsteps, K);
            if (rc) return rc == FDTD_OK ? rc : fail(lead, rc, cs[i]->err);
        }
    }
    SystolicState* L = lead->sys;
    int rc = upload_plan(lead, L, cs, n);
    if (rc) return rc;
    bool anyper = false;
    for (int i = 0; i < n; ++i) anyper = anyper || cs[i]->sys->pl.per[0] || cs[i]->sys->pl.per[1] || cs[i]->sys->pl.per[2];

    // material indices when every member has them (and allows them)
    bool mat = !lossy;
    for (int i = 0; i < n && mat; ++i) mat = cs[i]->use_mat && cs[i]->nmat > 0 && cs[i]->mat_id;
    // the tile width (every member shares it): 11 on a lossless FP32 grid
    // when asked for, 19 (indices in registers) with material indices
    const int wx = tile_x(lead);
    const bool narrow = !lossy && !h16 && wx == WX_LOSSY;
    const bool wide = wx == WX_WIDE;
    // (FP16 storage with material indices: device-scope synchronisation only;
    // the fence variant streams the binary16 coefficients)
    if (h16 && !dev) mat = false;
    if (wide && !(mat && dev))
        return fail(lead, FDTD_EUNSUPPORTED,
                    "systolic: the 19-wide tile needs material indices (at most 256 coefficient triples, "
                    "FDTD_OPT_MATERIAL_IDS) and device-scope synchronisation");
    // (a periodic x axis wraps positions once per access: it needs at least
    // as many cells as the tile has x slots)
    for (int i = 0; i < n; ++i)
        if (cs[i]->sys->pl.per[0] && cs[i]->nx < wx + 1)
            return fail(lead, FDTD_EUNSUPPORTED,
                        "systolic: a periodic x axis needs at least " + std::to_string(wx + 1) +
                            " cells with a " + std::to_string(wx) + "-wide tile");
    // variants: [sync][periodic][FP32, conductive, FP16 storage, FP32 with
    // material indices, the next two with the 11-wide tile, FP16 storage with
    // material indices, material indices with the 19-wide tile in FP32 and
    // FP16 storage (the last five: device-scope synchronisation only)]
    using Kern = void (*)(SysArgs);
#define FDTD_SYS_ROW(D, P)                                                                                  \
    {systolic_kernel<kNW, D, P, false, false, false, WX>, systolic_kernel<kNW, D, P, true, false, false, WX_LOSSY>, \
     systolic_kernel<kNW, D, P, false, true, false, WX>, systolic_kernel<kNW, D, P, false, false, true, WX>,       \
     D ? systolic_kernel<kNW, D, P, false, false, false, WX_LOSSY> : nullptr,                                   \
     D ? systolic_kernel<kNW, D, P, false, false, true, WX_LOSSY> : nullptr,                                    \
     D ? systolic_kernel<kNW, D, P, false, true, true, WX> : nullptr,                                           \
     D ? systolic_kernel<kNW, D, P, false, false, true, WX_WIDE> : nullptr,                                     \
     D ? systolic_kernel<kNW, D, P, false, true, true, WX_WIDE> : nullptr}
    static const Kern kernels[2][2][9] = {{FDTD_SYS_ROW(false, false), FDTD_SYS_ROW(false, true)},
                                          {FDTD_SYS_ROW(true, false), FDTD_SYS_ROW(true, true)}};
#undef FDTD_SYS_ROW
    const int var = wide ? (h16 ? 8 : 7) : h16 ? (mat ? 6 : 2) : (lossy ? 1 : (mat ? 3 : 0)) + (narrow ? (mat ? 2 : 4) : 0);
    const Kern kern = kernels[dev][anyper][var];
    if (!kern) return fail(lead, FDTD_EUNSUPPORTED, "systolic: the narrow tile needs device-scope synchronisation");
    hipError_t e;
    if (L->sm_count == 0) {
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, lead->device)) != hipSuccess) return hip_fail(lead, e, "hipGetDeviceProperties");
        L->sm_count = prop.multiProcessorCount;
    }
    int per_cu = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * kNW, 0)) != hipSuccess)
        return hip_fail(lead, e, "occupancy query");
    // every workgroup of the persistent grid must be resident at once
    const int capacity = std::max(1, per_cu) * L->sm_count;
    const int nt = L->up_nt;
    int grid = lead->workgroups > 0 ? std::min(lead->workgroups, capacity) : capacity;
    grid = std::max(1, std::min(grid, nt));
    // The tiles of a periodic ring wait on each other in a cycle that only
    // time breaks, so a whole ring group must be resident together.
    if (anyper && grid < L->up_group)
        return fail(lead, FDTD_EUNSUPPORTED,
                    "systolic: a periodic ring group of " + std::to_string(L->up_group) +
                        " tiles needs as many resident workgroups (grid " + std::to_string(grid) + ")");
    // Face ring: a slot is reused R tickets later, after its previous
    // occupant and that occupant's consumers have finished.  R = D + 2 * grid
    // keeps those long finished by the time the slot comes round again,
    // so the reuse wait never holds a workgroup in steady state; as grid is
    // at least one ring group, both lie in groups before the reuser's own.
    const int R = std::max(1, std::min(L->up_D + 2 * grid, nt));
    // four face rings in one allocation (x, y, z faces of E and H; the z
    // face's coefficients), each addressed with 32-bit offsets
    // (one component of an x face block is 16 x 16 words; of a y or z face
    // block, one row per x slot rounded up to four, at least 16, x 16)
    const size_t face = (size_t)(4 * kNW) * 16 * sizeof(float);
    const size_t face_yz = (size_t)std::max(16, (wx + 1 + 3) & ~3) * 16 * sizeof(float);
    const size_t rf6 = (size_t)R * Kmax * 6 * face_yz;
    // the z face's coefficients: cE (with conductivity ca too; with the wide
    // tile the index alone)
    const int ncz = lossy ? 6 : (wide ? 1 : 3);
    // (with FP16 storage the x and y faces' coefficients travel on rings of
    // their own, unless material indices replace them)
    const size_t rb[6] = {(size_t)R * Kmax * 6 * face, rf6, rf6, (size_t)R * Kmax * ncz * face_yz,
                          (h16 && !mat) ? (size_t)R * Kmax * 3 * face : 0,
                          (h16 && !mat) ? (size_t)R * Kmax * 3 * face_yz : 0};
    if (rf6 >= ((size_t)1 << 32) && lead->band_steps == 0 && Kmax > 1) {
        // an automatic band: take the longest one whose rings fit
        const size_t per_step = (size_t)R * 6 * face_yz;
        const int fit = (int)std::min<size_t>((((size_t)1 << 32) - 1) / per_step, (size_t)Kmax - 1);
        return launch(cs, n, nsteps, std::max(1, fit), run);
    }
    if (rf6 >= ((size_t)1 << 32))
        return fail(lead, FDTD_EUNSUPPORTED,
                    "systolic: face ring too large for 32-bit offsets (" + std::to_string(R) + " slots of " +
                        std::to_string(Kmax) + " steps); a shorter band (FDTD_OPT_BAND_STEPS) shrinks it");
    const size_t ring_bytes = rb[0] + rb[1] + rb[2] + rb[3] + rb[4] + rb[5];
    if (ring_bytes > L->ring_bytes || !L->d_ring) {
        if (L->d_ring) (void)hipFree(L->d_ring);
        L->d_ring = nullptr;
        L->ring_bytes = 0;
        if ((e = hipMalloc(&L->d_ring, ring_bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(lead, FDTD_ENOMEM, std::string("systolic face ring: ") + hipGetErrorString(e));
        }
        L->ring_bytes = ring_bytes;
    }
    L->R = R;
    if (!L->d_counter && (e = hipMalloc(&L->d_counter, sizeof(unsigned))) != hipSuccess) {
        (void)hipGetLastError();
        return fail(lead, FDTD_ENOMEM, "systolic: ticket counter");
    }
    if (!run) return FDTD_OK;
    // per-simulation records, through pinned staging
    if (!L->sims_done && (e = hipEventCreateWithFlags(&L->sims_done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(lead, e, "hipEventCreate");
    if ((e = hipEventSynchronize(L->sims_done)) != hipSuccess) return hip_fail(lead, e, "hipEventSynchronize");
    if ((size_t)n > L->cap_sims) {
        if (L->h_sims) (void)hipHostFree(L->h_sims);
        if (L->d_sims) (void)hipFree(L->d_sims);
        L->h_sims = nullptr;
        L->d_sims = nullptr;
        L->cap_sims = 0;
        if ((e = hipHostMalloc(&L->h_sims, n * sizeof(SimArgs), hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc(&L->d_sims, n * sizeof(SimArgs))) != hipSuccess) {
            (void)hipGetLastError();
            return fail(lead, FDTD_ENOMEM, "systolic: simulation records");
        }
        L->cap_sims = n;
    }
    for (int i = 0; i < n; ++i) {
        const fdtd_ctx* c = cs[i];
        SimArgs& P = L->h_sims[i];
        memset(&P, 0, sizeof(P));
        // (with FP16 storage the record holds the binary16 arrays: the
        // kernel only forms buffer descriptors from these addresses)
        for (int q = 0; q < 6; ++q) P.f[q] = h16 ? (float*)c->field16[q] : c->field[q];
        for (int q = 0; q < 3; ++q) P.cE[q] = h16 ? (const float*)c->coef16[q] : c->coef[q];
        for (int q = 0; q < 3; ++q) P.ca[q] = c->ca[q];
        for (int q = 0; q < 6; ++q) {
            P.sc[q] = ldexpf(1.0f, c->fexp[q]);
            P.isc[q] = ldexpf(1.0f, -c->fexp[q]);
        }
        P.cH = c->cH;
        P.nx = c->nx;
        P.ny = c->ny;
        P.nz = c->nz;
        P.esize = h16 ? 2u : 4u;
        P.band = L->d_band + L->up_band_off[i];
        P.step0 = c->step_count;
        P.src = c->dev_sources;
        P.nsrc = c->dev_sources_n;
        for (int d = 0; d < 3; ++d) {
            const int nd = d == 0 ? c->nx : (d == 1 ? c->ny : c->nz);
            const int W = d == 0 ? tile_x(c) : (d == 1 ? 4 * kNW - 1 : WZ);
            P.per[d] = c->sys->pl.per[d];
            P.L[d] = c->sys->pl.L[d];
            P.wr[d] = c->sys->pl.per[d] ? nd - W * (c->sys->pl.L[d] - 1) : W;
        }
        P.K = c->sys->pl.K;
        P.mid = mat ? c->mat_id : nullptr;
        P.mtab = mat ? c->mat_tab : nullptr;
    }
    hipStream_t st = lead->stream;
    // order the launch after each member's earlier work
    std::vector<hipEvent_t> evs;
    for (int i = 1; i < n; ++i) {
        if (cs[i]->stream == st) continue;
        hipEvent_t ev;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(lead, e, "hipEventCreate");
        evs.push_back(ev);
        if ((e = hipEventRecord(ev, cs[i]->stream)) != hipSuccess || (e = hipStreamWaitEvent(st, ev, 0)) != hipSuccess)
            break;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(L->d_sims, L->h_sims, n * sizeof(SimArgs), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(L->sims_done, st);
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    evs.clear();
    if (e != hipSuccess) return hip_fail(lead, e, "systolic launch set-up");
    hipLaunchKernelGGL(fill_u32, dim3(256), dim3(256), 0, st, L->d_progress, 0u, (long long)nt);
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, st, L->d_counter, 0u, 1LL);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(lead, e, "systolic reset");

    SysArgs A;
    memset(&A, 0, sizeof(A));
    A.sims = L->d_sims;
    A.tsim = n > 1 ? L->d_tsim : nullptr;
    A.tickets = L->d_tickets;
    A.nt = nt;
    A.tix = L->d_tix;
    A.progress = L->d_progress;
    size_t roff = 0;
    for (int f = 0; f < 6; ++f) {
        A.ring[f] = L->d_ring + roff / sizeof(float);
        A.ring_bytes[f] = (unsigned)rb[f];
        roff += rb[f];
    }
    A.R = R;
    A.Kmax = Kmax;
    A.nsteps = (int)nsteps;
    A.counter = L->d_counter;
    A.error = lead->dev_error;
    A.spin_limit = lead->spin_limit;
    PendingTiming t;
    timing_begin(lead, FDTD_KERNEL_SYSTOLIC, &t);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kNW), 0, st, A);
    timing_end(lead, &t);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(lead, e, "launch(systolic)");
    // members see a timeout of the shared launch in their own error word (their
    // own bits stay), and their streams continue after the launch
    for (int i = 1; i < n && e == hipSuccess; ++i) {
        hipLaunchKernelGGL(or_timeout, dim3(1), dim3(64), 0, st, cs[i]->dev_error, (const int*)lead->dev_error);
        e = hipGetLastError();
        if (e == hipSuccess && cs[i]->stream != st) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) == hipSuccess) {
                e = hipEventRecord(ev, st);
                if (e == hipSuccess) e = hipStreamWaitEvent(cs[i]->stream, ev, 0);
                (void)hipEventDestroy(ev);
            }
        }
    }
    if (e != hipSuccess) return hip_fail(lead, e, "systolic launch completion");
    for (int i = 0; i < n; ++i) {
        cs[i]->step_count += nsteps;
        cs[i]->sys_grid = grid;
        cs[i]->sys_ring_slots = R;
        cs[i]->sys_band = cs[i]->sys->pl.K;
        cs[i]->sys_tickets = nt;
    }
    return FDTD_OK;
}

}  // namespace

int systolic_supported(const fdtd_ctx* ctx, std::string* why)
{
    const int n[3] = {ctx->nx, ctx->ny, ctx->nz};
    for (int a = 0; a < 3; ++a)
        if (ctx->cfg.bc[a] == FDTD_BC_PERIODIC && n[a] < 16) {
            *why = "the systolic scheme needs at least 16 cells on a periodic axis";
            return 0;
        }
    // 32-bit buffer offsets: a ticket addresses at most kMaxBand + 16
    // x-planes from its own base on a PEC x axis, the whole array on a
    // periodic one
    const uint64_t es = ctx->storage == FDTD_FP16_STORAGE ? 2u : 4u;
    const uint64_t plane = (uint64_t)ctx->ny * ctx->nz;
    const bool perx = ctx->cfg.bc[0] == FDTD_BC_PERIODIC;
    const uint64_t span = perx ? (uint64_t)ctx->nx : std::min<uint64_t>(ctx->nx, kMaxBand + 16);
    if (span * plane * es > 0xFFFFFF00ull) {
        *why = perx ? "field arrays of 4 GiB or more need a PEC x axis on the systolic scheme"
                    : "an x-plane of this grid is too large for the systolic scheme's 32-bit offsets";
        return 0;
    }
    return 1;
}

int systolic_step(fdtd_ctx* ctx, int64_t nsteps)
{
    fdtd_ctx* one[1] = {ctx};
    return launch(one, 1, nsteps);
}

int systolic_step_batch(fdtd_ctx* const* ctxs, int n, int64_t nsteps) { return launch(ctxs, n, nsteps); }

int systolic_prepare(fdtd_ctx* ctx, int64_t nsteps)
{
    fdtd_ctx* one[1] = {ctx};
    return launch(one, 1, nsteps, kMaxBand, false);
}

void systolic_tile(const fdtd_ctx* ctx, int* wx, int* wy, int* wz)
{
    *wx = tile_x(ctx);
    *wy = 4 * kNW - 1;
    *wz = WZ;
}

void systolic_release(fdtd_ctx* ctx)
{
    if (!ctx->sys) return;
    free_launch(ctx->sys);
    delete ctx->sys;
    ctx->sys = nullptr;
}

}  // namespace fdtd
