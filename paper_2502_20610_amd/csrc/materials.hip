// Material indices of a lossless FP32 grid.
//
// The E update of Section 2 multiplies by the per-cell coefficients cE_c
// (the structural fields of Section 4).  Grids built from a few materials
// (boxes of a few permittivities, PEC walls) hold only a few distinct
// triples (cEx, cEy, cEz) per cell.  The systolic scheme then streams a
// 4-byte index per cell instead of the triple (12 bytes, or the 6 of
// binary16 with FP16 storage, which also had to travel on face rings) and
// looks the triple up in a table of at most kMaxMaterials entries: the
// coefficient values, and so every result, are the same bits as with the
// arrays.
//
// The distinct triples are found on the device in rounds.  Each round
// classifies every cell against the triples known so far (a hash table in
// LDS, keyed on the three bit patterns); cells that match get their index,
// and unmatched triples are reported, up to kCand distinct ones per round.
// The host adds the new triples and runs another round until every cell
// matches, or gives up once there are more than kMaxMaterials.  Entry 0 is always (+0, +0, +0):
// the value that positions outside the grid read.
#include <string.h>

#include <vector>

#include "fdtd_internal.h"

namespace fdtd {

namespace {

constexpr int kSlots = 1024;  // hash slots (at most kMaxMaterials used)
constexpr int kCand = 64;     // unmatched triples reported per round
constexpr int kThreads = 256;

__host__ __device__ inline unsigned slot_of(unsigned a, unsigned b, unsigned c)
{
    unsigned h = (a * 0x9E3779B1u) ^ (b * 0x85EBCA77u) ^ (c * 0xC2B2AE3Du);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 13;
    return h & (kSlots - 1);
}

// keys: kSlots x 3 words (the triple's bits), idx: kSlots entries (-1 empty).
// Cells that match get their index.  Unmatched triples are reported into a
// table of kCand slots keyed by a hash of the triple: each wavefront reports
// up to four distinct triples per launch (one atomic compare-and-swap each,
// no waiting), so a round finds up to kCand new triples; cand[0] is set when
// any cell did not match.  cand layout: [0] flag, [1 .. kCand] slot keys,
// then kCand triples.
// With H16 the coefficients are binary16 (FP16 storage) and the triple is
// that of their exact FP32 values.
template <bool H16>
__global__ __launch_bounds__(kThreads) void classify_kernel(const void* __restrict__ c0v,
                                                            const void* __restrict__ c1v,
                                                            const void* __restrict__ c2v, long long n,
                                                            const unsigned* __restrict__ keys,
                                                            const int* __restrict__ idx,
                                                            unsigned* __restrict__ ids,
                                                            unsigned* __restrict__ cand)
{
    __shared__ unsigned s_key[kSlots][3];
    __shared__ int s_idx[kSlots];
    auto bits = [&](const void* base, long long p) -> unsigned {
        if (H16) return __float_as_uint((float)__builtin_bit_cast(_Float16, ((const uint16_t*)base)[p]));
        return __float_as_uint(((const float*)base)[p]);
    };
    for (int i = threadIdx.x; i < kSlots; i += kThreads) {
        s_key[i][0] = keys[3 * i];
        s_key[i][1] = keys[3 * i + 1];
        s_key[i][2] = keys[3 * i + 2];
        s_idx[i] = idx[i];
    }
    __syncthreads();
    int reports = 0;  // wave-uniform: distinct triples this wavefront reported
    const long long nr = (n + kThreads - 1) / kThreads * kThreads;  // every lane runs every pass
    for (long long p0 = (long long)blockIdx.x * kThreads; p0 < nr; p0 += (long long)gridDim.x * kThreads) {
        const long long p = p0 + threadIdx.x;
        const bool in = p < n;
        unsigned a = 0, b = 0, c = 0;
        int found = -1;
        if (in) {
            a = bits(c0v, p);
            b = bits(c1v, p);
            c = bits(c2v, p);
            unsigned s = slot_of(a, b, c);
            // the table is at most a quarter full, so an empty slot ends every probe
            for (int probe = 0; probe < kSlots; ++probe) {
                const int id = s_idx[s];
                if (id < 0) break;
                if (s_key[s][0] == a && s_key[s][1] == b && s_key[s][2] == c) {
                    found = id;
                    break;
                }
                s = (s + 1) & (kSlots - 1);
            }
            ids[p] = found >= 0 ? (unsigned)found : 0u;
        }
        unsigned long long miss = __ballot(in && found < 0);
        if (miss && (threadIdx.x & 63) == __ffsll((long long)miss) - 1) cand[0] = 1u;
        while (miss && reports < 4) {
            const int lead = __ffsll((long long)miss) - 1;
            const unsigned ta = __shfl(a, lead, 64), tb = __shfl(b, lead, 64), tc = __shfl(c, lead, 64);
            if ((int)(threadIdx.x & 63) == lead) {
                const unsigned h = (slot_of(ta, tb, tc) * 0x9E3779B9u) | 1u;  // never 0 (free)
                const unsigned q = h % (unsigned)kCand;
                const unsigned prev = atomicCAS(&cand[1 + q], 0u, h);
                if (prev == 0u) {
                    unsigned* t = cand + 1 + kCand + 3 * q;
                    t[0] = ta;
                    t[1] = tb;
                    t[2] = tc;
                }
            }
            // lanes holding the same triple are covered by that report
            miss &= __ballot(!(a == ta && b == tb && c == tc));
            ++reports;
        }
    }
}

int grid_blocks(int64_t n)
{
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

}  // namespace

void release_material_ids(fdtd_ctx* ctx)
{
    if (ctx->mat_id) (void)hipFree(ctx->mat_id);
    if (ctx->mat_tab) (void)hipFree(ctx->mat_tab);
    ctx->mat_id = nullptr;
    ctx->mat_tab = nullptr;
    ctx->nmat = 0;
}

int build_material_ids(fdtd_ctx* ctx)
{
    ctx->nmat = 0;
    if (ctx->ca[0]) return FDTD_OK;  // lossless grids only
    hipError_t e;
    if (!ctx->mat_id && (e = hipMalloc(&ctx->mat_id, (size_t)ctx->ncell * sizeof(unsigned))) != hipSuccess) {
        (void)hipGetLastError();
        ctx->mat_id = nullptr;
        return FDTD_OK;  // no room: the per-cell arrays serve
    }
    if (!ctx->mat_tab && (e = hipMalloc(&ctx->mat_tab, kMaxMaterials * 3 * sizeof(float))) != hipSuccess) {
        (void)hipGetLastError();
        ctx->mat_tab = nullptr;
        return FDTD_OK;
    }
    unsigned* d_keys = nullptr;
    int* d_idx = nullptr;
    unsigned* d_cand = nullptr;
    const size_t ncand = 1 + kCand + 3 * kCand;  // flag, slot keys, triples
    const size_t scratch = kSlots * 3 * sizeof(unsigned) + kSlots * sizeof(int) + ncand * sizeof(unsigned);
    char* d_scratch = nullptr;
    if ((e = hipMalloc(&d_scratch, scratch)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FDTD_ENOMEM, "material table: scratch allocation failed");
    }
    d_keys = (unsigned*)d_scratch;
    d_idx = (int*)(d_keys + kSlots * 3);
    d_cand = (unsigned*)(d_idx + kSlots);

    std::vector<unsigned> tab(3, 0u);  // entry 0: (+0, +0, +0)
    std::vector<unsigned> keys(kSlots * 3), cand(ncand);
    const std::vector<unsigned> cand0(ncand, 0u);
    std::vector<int> idx(kSlots);
    bool ok = false;
    e = hipSuccess;
    for (int round = 0; round <= kMaxMaterials && e == hipSuccess; ++round) {
        const int nm = (int)tab.size() / 3;
        std::fill(idx.begin(), idx.end(), -1);
        std::fill(keys.begin(), keys.end(), 0u);
        for (int m = 0; m < nm; ++m) {
            unsigned s = slot_of(tab[3 * m], tab[3 * m + 1], tab[3 * m + 2]);
            while (idx[s] >= 0) s = (s + 1) & (kSlots - 1);
            idx[s] = m;
            for (int q = 0; q < 3; ++q) keys[3 * s + q] = tab[3 * m + q];
        }
        if ((e = hipMemcpyAsync(d_keys, keys.data(), keys.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                                ctx->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(d_idx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(d_cand, cand0.data(), ncand * sizeof(unsigned), hipMemcpyHostToDevice,
                                ctx->stream)) != hipSuccess)
            break;
        const bool h16 = ctx->storage == FDTD_FP16_STORAGE;
        const void* cs[3];
        for (int q = 0; q < 3; ++q) cs[q] = h16 ? (const void*)ctx->coef16[q] : (const void*)ctx->coef[q];
        hipLaunchKernelGGL(h16 ? classify_kernel<true> : classify_kernel<false>, dim3(grid_blocks(ctx->ncell)),
                           dim3(kThreads), 0, ctx->stream, cs[0], cs[1], cs[2], (long long)ctx->ncell, d_keys,
                           d_idx, ctx->mat_id, d_cand);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = hipMemcpyAsync(cand.data(), d_cand, cand.size() * sizeof(unsigned), hipMemcpyDeviceToHost,
                                ctx->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
            break;
        if (cand[0] == 0) {
            ok = true;
            break;
        }
        for (int i = 0; i < kCand && (int)tab.size() / 3 <= kMaxMaterials; ++i) {
            if (cand[1 + i] == 0) continue;  // slot not claimed
            const unsigned* t = &cand[1 + kCand + 3 * i];
            bool have = false;
            for (size_t m = 0; m < tab.size() / 3 && !have; ++m)
                have = tab[3 * m] == t[0] && tab[3 * m + 1] == t[1] && tab[3 * m + 2] == t[2];
            if (!have) tab.insert(tab.end(), t, t + 3);
        }
        if ((int)tab.size() / 3 > kMaxMaterials) break;  // too many: the per-cell arrays serve
    }
    if (ok && e == hipSuccess) {
        std::vector<unsigned> full(kMaxMaterials * 3, 0u);
        std::copy(tab.begin(), tab.end(), full.begin());
        e = hipMemcpyAsync(ctx->mat_tab, full.data(), full.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) ctx->nmat = (int)tab.size() / 3;
    }
    (void)hipFree(d_scratch);
    if (e != hipSuccess) return hip_fail(ctx, e, "material table");
    // too many materials: the per-cell arrays serve, the index array goes
    if (ctx->nmat == 0) release_material_ids(ctx);
    return FDTD_OK;
}

}  // namespace fdtd
