// Internal declarations shared by the translation units of libfdtd.so.
// Not part of the public ABI (see include/fdtd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fdtd.h"

namespace fdtd {

// One soft point source: E_comp[cell] += wave[s - first] during the step that
// starts at step count s.
struct SourceRec {
    int comp;
    int i, j, k;
    int64_t len;
    int64_t first;
    float* wave;  // device copy of the waveform
};

// Device-side source table entry (plain scheme and systolic kernel).
struct DevSource {
    int comp;
    int i, j, k;
    long long len;
    long long first;
    const float* wave;
};

struct PendingTiming {
    int kernel;
    hipEvent_t start, stop;
};

struct SystolicState;  // defined in systolic.hip
struct StepGraph;      // defined in plain.hip

}  // namespace fdtd

struct fdtd_ctx {
    fdtd_config cfg;
    int nx, ny, nz;
    int64_t ncell;
    int device;
    hipStream_t stream;
    bool own_stream;

    // FP32 storage: field and coef hold the arrays (field16/coef16 null).
    // FP16 storage: field16 and coef16 hold IEEE binary16 arrays (field and
    // coef null); field component c is stored as v * 2^-fexp[c].
    int storage;      // FDTD_FP32 or FDTD_FP16_STORAGE
    float* field[6];  // Ex Ey Ez Hx Hy Hz
    float* coef[3];   // cEx cEy cEz (cb, the curl coefficient, with conductivity)
    uint16_t* field16[6];
    uint16_t* coef16[3];
    int fexp[6];      // FP16 storage: power-of-two scale exponent per field component
    float* ca[3];     // E decay per step with conductivity; null when lossless
    float* alt[6];    // second field set of the fused plain step (allocated on first use)
    float cH;

    std::vector<fdtd::SourceRec> sources;
    fdtd::DevSource* dev_sources;  // device table, rebuilt when sources change
    int dev_sources_n;

    int64_t step_count;
    bool poisoned;
    std::string err;

    // options
    int scheme;
    int band_steps;
    int workgroups;
    int64_t spin_limit;
    bool profile;

    // kernel timing
    std::vector<fdtd::PendingTiming> pending;
    int64_t launches[FDTD_KERNEL_COUNT];
    double total_ms[FDTD_KERNEL_COUNT];

    int* dev_error;  // device error word: bit 0 bad eps, bit 1 watchdog timeout

    double* inv_scratch;  // partial sums of fdtd_invariants (allocated on first use)

    // material indices (lossless grids with at most kMaxMaterials
    // distinct coefficient triples): per-cell index into a table of
    // (cEx, cEy, cEz); nmat = 0 when the per-cell arrays are the only form
    uint32_t* mat_id;
    float* mat_tab;   // kMaxMaterials x 3 floats, entry 0 = (+0, +0, +0)
    int nmat;
    bool use_mat;     // FDTD_OPT_MATERIAL_IDS
    int tile_wx;      // FDTD_OPT_TILE_X: 0 (the launch's default), 11, 15 or 19
    int auto_wx;      // the default width of the last systolic launch (19 or 15; 0 before)
    bool tune_plain;  // FDTD_OPT_AUTOTUNE_PLAIN

    // plain schemes: step loops replayed as a HIP graph (FDTD_OPT_GRAPHS)
    bool use_graphs;
    fdtd::StepGraph* graph;
    long long* d_step;  // the step counter the graph advances (two words)

    fdtd::SystolicState* sys;
    int sys_grid;        // persistent workgroups of the last systolic launch
    int sys_ring_slots;  // face-ring slots of the last systolic launch
    int sys_band;        // steps per band of the last systolic launch
    int sys_tickets;     // tickets of the last systolic launch
};

namespace fdtd {

// Error helpers (set ctx->err, return the code).
int fail(fdtd_ctx* ctx, int code, const std::string& msg);
int hip_fail(fdtd_ctx* ctx, hipError_t e, const char* what);

// Timing wrappers around a launch on ctx->stream (no-ops when profiling is off).
void timing_begin(fdtd_ctx* ctx, int kernel, PendingTiming* t);
void timing_end(fdtd_ctx* ctx, PendingTiming* t);

// Plain scheme: advance n steps starting at ctx->step_count (plain.hip).
int plain_step(fdtd_ctx* ctx, int64_t nsteps);
// Fused plain scheme: one launch per step into the second field set, whose
// pointers then trade places with ctx->field (plain.hip).
int plain_fused_step(fdtd_ctx* ctx, int64_t nsteps);
// Allocate the fused step's second field set (plain.hip).
int plain_fused_prepare(fdtd_ctx* ctx);
// Free the captured step graph and its counter (plain.hip).
void release_step_graph_exec(StepGraph* g);
void release_step_graph(fdtd_ctx* ctx);

// Systolic scheme (systolic.hip).
int systolic_supported(const fdtd_ctx* ctx, std::string* why);
int systolic_step(fdtd_ctx* ctx, int64_t nsteps);
int systolic_step_batch(fdtd_ctx* const* ctxs, int n, int64_t nsteps);
// Build and upload the plan of a call of nsteps steps, allocate its rings.
int systolic_prepare(fdtd_ctx* ctx, int64_t nsteps);
void systolic_release(fdtd_ctx* ctx);
void systolic_tile(const fdtd_ctx* ctx, int* wx, int* wy, int* wz);

// Measured tile width and band length of the systolic scheme (autotune.hip).
int autotune_run(fdtd_ctx* ctx, int64_t nsteps, int64_t* tile_x, int64_t* band_steps);
// Read the device error word: FDTD_ETIMEOUT (and poison), FDTD_EINVAL for a
// pending bad-permittivity report (then cleared), else FDTD_OK.  Synchronous.
int device_error(fdtd_ctx* ctx);

// Reverse-time adjoint of a monitor objective (adjoint.hip).
int adjoint_run(fdtd_ctx* ctx, fdtd_adjoint_spec* spec, float* grad_eps, int where);

// Discrete invariants (invariants.hip): the reduction runs kInvBlocks blocks
// whose partial records, and then the FDTD_INV_COUNT final sums, live in a
// scratch area of invariants_scratch_doubles() doubles.
constexpr int kInvBlocks = 1024;
constexpr size_t kInvScratchDoubles = (size_t)kInvBlocks * 8 + 8;
size_t invariants_scratch_doubles();
// the final sums start at scratch + invariants_sums_offset()
size_t invariants_sums_offset();
// partial records at `part`, the final sums at `out` (both device memory)
int invariants_launch(fdtd_ctx* ctx, double* part, double* out, double* div_e, double* div_h);
// The allocation-free variant's scratch (a static device array of
// kInvScratchDoubles doubles in invariants.hip): look up its address on
// `device` (the current device) once, at context creation; then
// invariants_scratch_ptr(device) returns it (null if never looked up or
// device >= kMaxScratchDevices).
constexpr int kMaxScratchDevices = 64;
int invariants_scratch_init(int device);
double* invariants_scratch_ptr(int device);

// Material indices (materials.hip): find the distinct coefficient triples
// of a lossless context after its coefficients were built (FP32 values; the
// exact FP32 values of binary16 ones with FP16 storage); leaves nmat = 0
// when there are more than kMaxMaterials (or the context is conductive).
// release_material_ids frees them.
constexpr int kMaxMaterials = 256;
int build_material_ids(fdtd_ctx* ctx);
void release_material_ids(fdtd_ctx* ctx);

// Launch the source-injection kernel for the step that starts at step count s
// on stream st (ctx->stream for a direct launch); with stepp (a graph being
// captured) the kernel reads the step from *stepp and advances it instead.
int launch_sources(fdtd_ctx* ctx, int64_t s, hipStream_t st, long long* stepp = nullptr);

// True if any source is active in the step starting at step count s.
bool sources_active(const fdtd_ctx* ctx, int64_t s);

}  // namespace fdtd
