/*
 * fdtd.h -- C ABI of the MI355X (gfx950) systolic 3D Yee FDTD library, libfdtd.so.
 *
 * The library advances Maxwell's equations with the Yee leapfrog scheme of the
 * paper's Section 2, Eq. (1): for every cell, first the three E components are
 * updated from backward differences of H, e.g.
 *
 *     Ex = (Ex + cEx*(Hz - Hz[j-1])) - cEx*(Hy - Hy[k-1]),
 *
 * (Ey, Ez by cyclic permutation), then point sources are added, then the three
 * H components are updated from forward differences of the new E with
 * Faraday's sign, e.g. Hx = (Hx - cH*(Ez[j+1] - Ez)) + cH*(Ey[k+1] - Ey).
 * E is updated before H within a step as in the horizontal-bar scheme (caption
 * of Fig. 7).  cE_c = dt/(eps_c*dx) per component and cell (the "structural
 * fields" of Section 4), computed in double and rounded to float; cH = dt/dx
 * (mu = 1).  Units are normalised, c = eps0 = mu0 = 1, as in Eq. (1).  Every
 * arithmetic operation is a separately rounded FP32 operation, evaluated left
 * to right as written, with no fused multiply-add; the results are therefore
 * a single well-defined FP32 value per cell and step, independent of the
 * scheme that computes them.
 *
 * Schemes:
 *   FDTD_SCHEME_PLAIN    one kernel launch per half-step over the whole grid:
 *                        the naive implementation of Section 2 / Fig. 1.
 *   FDTD_SCHEME_SYSTOLIC one persistent launch per call: subdomain tiles stay
 *                        resident on chip for many steps, move one cell along
 *                        the x-y-z-t diagonal per step and exchange only their
 *                        boundary faces through device memory, synchronising
 *                        with neighbour flags (Sections 3 and 4).
 *   FDTD_SCHEME_PLAIN_FUSED one kernel launch per step over the whole grid:
 *                        E and H are read from one set of arrays and the new
 *                        step is written to a second set, allocated on first
 *                        use (six more arrays; the two sets then trade places
 *                        every step).  FP32 storage only (else
 *                        FDTD_EUNSUPPORTED from fdtd_step); conductivity is
 *                        covered.
 *
 * Layout: every field and coefficient array is C order [nx][ny][nz]
 * (z fastest), one array per component (Ex, Ey, Ez, Hx, Hy, Hz); FP32, or
 * IEEE binary16 inside the library with FP16 storage (the ABI always passes
 * FP32).
 *
 * FP16 storage (fdtd_config.storage = FDTD_FP16_STORAGE; Section 4 stores the
 * field values in 16-bit floating point): the device arrays hold binary16,
 * field component c as v * 2^-e_c (fdtd_set_field_scale, default e_c = 0)
 * and cE rounded from its FP32 value; every operation still computes in FP32
 * exactly as above.  A stored value is rounded once, to nearest even (the
 * scales are powers of two, so scaling is exact; out-of-range values become
 * +-inf or binary16 subnormals/zero).  Rounding happens where a value is
 * stored: on input (fdtd_set_fields), and
 *   - plain scheme: after every E half-step, after each source addition, and
 *     after every H half-step;
 *   - systolic scheme: once per band of K steps (and at the end of every
 *     call), for the whole grid; every exchange between tiles inside a band
 *     keeps FP32.
 * fdtd_read_fields returns the stored values times 2^e_c, exactly.  With FP16
 * storage, conductive materials and fdtd_adjoint return FDTD_EUNSUPPORTED. 
 *
 * Boundaries: indices are periodic on every axis; a PEC axis additionally
 * holds the two E components tangential to its planes at +0 on its index-0
 * plane (cE = 0 there), which closes a perfectly conducting wall at 0 == n.
 *
 * Conventions for every function:
 *   - returns FDTD_OK (0) or a negative FDTD_E* code; no exception or abort
 *     crosses the ABI; fdtd_last_error() gives a message for the last failure;
 *   - a context is not thread-safe; distinct contexts are independent;
 *   - `where` says where a caller pointer lives: FDTD_HOST (read or written
 *     before the call returns) or FDTD_DEVICE (a device pointer on the
 *     context's device, accessed in order on the context's stream: the caller
 *     keeps it alive until fdtd_synchronize());
 *   - the library owns every allocation it makes and frees it in
 *     fdtd_destroy();
 *   - after FDTD_EHIP or FDTD_ETIMEOUT the context is poisoned: every later
 *     call except fdtd_last_error/fdtd_destroy returns FDTD_ESTATE.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_ctx fdtd_ctx; /* opaque */

enum {
    FDTD_OK = 0,
    FDTD_EINVAL = -1,      /* bad argument (sizes, ranges, Courant, PEC source) */
    FDTD_ENOMEM = -2,      /* device or host allocation failed                  */
    FDTD_EHIP = -3,        /* a HIP runtime call failed (message has the string)*/
    FDTD_ESTATE = -4,      /* context poisoned, or call out of order            */
    FDTD_EUNSUPPORTED = -5,/* valid request this build does not implement       */
    FDTD_ETIMEOUT = -6     /* a bounded wait inside the systolic kernel expired */
};

enum { FDTD_BC_PEC = 0, FDTD_BC_PERIODIC = 1 };
enum { FDTD_SCHEME_PLAIN = 0, FDTD_SCHEME_SYSTOLIC = 1, FDTD_SCHEME_PLAIN_FUSED = 2 };
enum { FDTD_FP32 = 0, FDTD_FP16_STORAGE = 1 };
enum { FDTD_EX = 0, FDTD_EY = 1, FDTD_EZ = 2, FDTD_HX = 3, FDTD_HY = 4, FDTD_HZ = 5 };
enum { FDTD_HOST = 0, FDTD_DEVICE = 1 };

typedef struct {
    uint32_t struct_size;  /* = sizeof(fdtd_config); versions the struct          */
    int32_t nx, ny, nz;    /* cells per axis, each >= 1; nx*ny*nz <= 2^30         */
    double dt, dx;         /* time step and uniform cell size (dx = dy = dz),
                              both > 0, with dt*sqrt(3) < dx (Courant for eps>=1) */
    int32_t bc[3];         /* FDTD_BC_PEC or FDTD_BC_PERIODIC for x, y, z        */
    int32_t scheme;        /* FDTD_SCHEME_*                                      */
    int32_t storage;       /* FDTD_FP32 or FDTD_FP16_STORAGE                     */
    int32_t device;        /* HIP device ordinal                                 */
    void* stream;          /* hipStream_t to run on; NULL = a stream the library
                              creates (default priority) and destroys           */
} fdtd_config;

/* Create a simulation: validates cfg (FDTD_EINVAL before any HIP call),
 * allocates the six field arrays and the three coefficient arrays on the
 * device, zero-fills the fields and sets eps = 1 everywhere.  On success
 * *out receives the context; on failure *out is NULL. */
int fdtd_create(const fdtd_config* cfg, fdtd_ctx** out);

/* Free everything the context owns.  NULL is accepted.  Waits for the
 * context's outstanding work first. */
int fdtd_destroy(fdtd_ctx* ctx);

/* Set the per-cell permittivity of each E component (the structural fields
 * of Section 4): three arrays of nx*ny*nz floats, each >= 1 and finite (else
 * FDTD_EINVAL, checked on host input; device input is checked on the
 * device and reported at the next synchronising call).  The library
 * computes cE_c = (float)(dt / ((double)eps_c * dx)) and zeroes it on the
 * index-0 planes of PEC axes tangential to component c.  The arrays are
 * copied; the caller keeps ownership.  The library also looks for the
 * distinct triples (cEx, cEy, cEz) of the grid (on the device, a few passes
 * over the coefficients, synchronising the stream; with FP16 storage the
 * triples of their binary16 values): with at most 256 of them (entry 0
 * being (+0, +0, +0)) it keeps a 4-byte material index per cell, which the
 * systolic scheme streams in place of the three coefficients (the bits it
 * multiplies by are the same). */
int fdtd_set_materials(fdtd_ctx* ctx, const float* eps_x, const float* eps_y,
                       const float* eps_z, int where);

/* Set permittivity and conductivity (the permittivity and conductivity
 * structural fields of Section 4): six arrays of nx*ny*nz floats, eps >= 1,
 * sigma >= 0, all finite (else FDTD_EINVAL as for fdtd_set_materials).  The
 * E half-step becomes the semi-implicit conductive update
 *     E_c = (ca_c * E_c + cb_c * d1) - cb_c * d2,
 *     h = sigma dt / (2 eps), ca = (1 - h) / (1 + h), cb = (dt / (eps dx)) / (1 + h),
 * all in IEEE double, rounded to FP32 (ca = 1, cb = 0 on PEC-tangential
 * index-0 entries); sigma = 0 gives the lossless update bit for bit.  Both
 * schemes run it (the systolic tile is then 11 cells wide along x, since ca
 * travels with the tile as three more per-cell coefficients);
 * fdtd_step_batch refuses (FDTD_EUNSUPPORTED) a batch that mixes
 * conductive and lossless contexts; fdtd_adjoint differentiates the
 * conductive update with respect to eps, sigma held fixed.  A later
 * fdtd_set_materials makes the context lossless again. */
int fdtd_set_lossy_materials(fdtd_ctx* ctx, const float* eps_x, const float* eps_y,
                             const float* eps_z, const float* sigma_x, const float* sigma_y,
                             const float* sigma_z, int where);

/* FP16 storage only (else FDTD_EINVAL): set the power-of-two scale of each
 * field component, component c being stored as v * 2^-exp2[c], exp2[c] in
 * [-30, 30].  The current field values are re-encoded under the new scales
 * (exact while they stay within the binary16 range).  Choosing e_c near
 * log2 of a component's peak magnitude keeps it away from binary16's
 * overflow (65504) and subnormal (< 6.1e-5) ranges. */
int fdtd_set_field_scale(fdtd_ctx* ctx, const int32_t exp2[6]);

/* Set the components selected by comp_mask (bit c = component c) from
 * src[c] (nx*ny*nz floats each; src entries for unselected components are
 * ignored and may be NULL).  The fields are E^n and H^(n+1/2) of the current
 * step count.  PEC-tangential E entries on index-0 planes are forced to +0. */
int fdtd_set_fields(fdtd_ctx* ctx, uint32_t comp_mask, const float* const src[6], int where);

/* Add a soft point source on E component comp (FDTD_EX..FDTD_EZ) at cell
 * (i, j, k): in the step that starts at step count s, after the E half-step,
 * E_comp[i][j][k] += waveform[s - first_step] for 0 <= s - first_step < len.
 * The waveform is copied.  FDTD_EINVAL if the cell is out of range or lies on
 * a PEC-frozen entry.  Returns the source id (>= 0) on success. */
int fdtd_add_source(fdtd_ctx* ctx, int comp, int32_t i, int32_t j, int32_t k,
                    const float* waveform, int64_t len, int64_t first_step, int where);

/* Advance nsteps (>= 0) full Yee steps.  Asynchronous: work is queued on the
 * context's stream.  The systolic scheme never falls back to another scheme;
 * configurations it does not cover return FDTD_EUNSUPPORTED: a periodic axis
 * of fewer than 16 cells, a periodic x axis with arrays of 4 GiB or more, a
 * periodic ring group (the tiles that differ only along periodic axes) larger
 * than the resident grid, or an explicit band whose face rings would not fit
 * 32-bit offsets.  A systolic launch on a grid with periodic axes needs each
 * ring group resident at once; other persistent launches running at the same
 * time on other streams (another context's systolic step, say) can hold the
 * workgroup slots it needs, and then it waits until they finish or until its
 * spin limit expires (FDTD_ETIMEOUT).  Launches on grids without periodic
 * axes make progress with any residency. */
int fdtd_step(fdtd_ctx* ctx, int64_t nsteps);

/* Prepare a later fdtd_step(ctx, nsteps): with the systolic scheme, build the
 * launch plan of a call of exactly nsteps steps (the (band, tile) tickets in
 * their topological order and the band tables of Section 3's diagonal
 * traversal), upload it with blocking copies, and allocate its face rings
 * and progress counters; with the fused plain scheme, allocate the second
 * field set; with the plain scheme, nothing.  No step runs and the state is
 * unchanged.  fdtd_step keeps the plan of its last call length (and the
 * largest rings so far), so repeated calls of one length never rebuild or
 * reallocate; this call moves that work ahead of a first call (say, out of
 * a timed region).  A change of the materials' kind (lossless or
 * conductive) or of the band option rebuilds the plan at the next call.
 * Errors as for fdtd_step (FDTD_EUNSUPPORTED for a grid the systolic scheme
 * does not cover, FDTD_ENOMEM if the rings do not fit). */
int fdtd_prepare(fdtd_ctx* ctx, int64_t nsteps);

/* Advance n independent contexts (grids of any sizes and boundaries, their
 * own materials and sources) by nsteps each in ONE persistent systolic launch
 * over a shared queue of subdomain tickets (the paper's tile traversal of
 * Section 3 extended over several simulations).  The result of each context
 * is bit-identical to fdtd_step on it alone; the systolic scheme is used
 * whatever each context's scheme option.  The launch runs on ctxs[0]'s
 * stream, after the work already queued on every member's stream, and every
 * member's stream continues after it.  Launch options (band steps, grid,
 * spin limit) are ctxs[0]'s; a wait timeout is reported by every member.
 * FDTD_EINVAL: NULL/empty list, n > 65536, a context listed twice, contexts
 * on different devices, nsteps < 0; FDTD_EUNSUPPORTED: a member the systolic
 * scheme does not cover, or a periodic ring group larger than the resident
 * grid. */
int fdtd_step_batch(fdtd_ctx* const* ctxs, int n, int64_t nsteps);

/* Copy the components selected by comp_mask into dst[c].  A host destination
 * synchronises the stream before returning; a device destination is written
 * in stream order. */
int fdtd_read_fields(fdtd_ctx* ctx, uint32_t comp_mask, float* const dst[6], int where);

/* Wait for all work queued on the context's stream; reports a watchdog
 * timeout of the systolic kernel as FDTD_ETIMEOUT. */
int fdtd_synchronize(fdtd_ctx* ctx);

/* Number of completed steps since creation (queued steps count as done);
 * -1 for a NULL context. */
int64_t fdtd_current_step(const fdtd_ctx* ctx);

/* Message describing the last failure of this context (never NULL).  With a
 * NULL context, the message of the last failed fdtd_create on this thread. */
const char* fdtd_last_error(const fdtd_ctx* ctx);

/* ---- discrete invariants (FP64 reductions on the device) ----------------
 *
 * The update of Section 2 (Eq. (1) and its cyclic permutations, E before H)
 * with the coefficients the context applies is
 *     E^{n+1} = E^n + cE (.) C_h H^{n+1/2},  H^{n+3/2} = H^{n+1/2} - cH C_e E^{n+1},
 * C_h the backward-difference curl of the E half-step, C_e = C_h^T the
 * forward-difference curl of the H half-step.  It keeps, exactly in exact
 * arithmetic,
 *   - the leapfrog energy Q = sum eps|E|^2 + sum |H|^2 + cH sum E . (C_h H)
 *     of a lossless box, eps_c = cH / cE_c being the permittivity the
 *     coefficients encode (cH (1 + ca) / (2 cb) with conductivity, where Q
 *     decays instead);
 *   - without sources, the backward divergence of eps E at every node whose
 *     index is >= 1 along each PEC axis, and the forward divergence of H at
 *     every cell.
 * The sums skip the E entries frozen by PEC walls (read as eps E = 0 in the
 * divergence).  Index arithmetic is periodic as in the update. */
enum {
    FDTD_INV_ENERGY = 0,      /* Q                                             */
    FDTD_INV_E_ENERGY = 1,    /* sum eps |E|^2                                 */
    FDTD_INV_H_ENERGY = 2,    /* sum |H|^2                                     */
    FDTD_INV_DIVE_L1 = 3,     /* sum over nodes off the PEC walls of |div eps E| */
    FDTD_INV_DIVE_L2SQ = 4,   /* the same sum of (div eps E)^2                 */
    FDTD_INV_DIVH_L1 = 5,     /* sum over all cells of |div H|                 */
    FDTD_INV_DIVH_L2SQ = 6,   /* sum of (div H)^2                              */
    FDTD_INV_COUNT = 7
};

/* Evaluate the invariants of the current state (E^n, H^{n+1/2}) in FP64 from
 * the stored values (binary16 storage decoded exactly).  sums: FDTD_INV_COUNT
 * doubles (required).  div_e, div_h: nx*ny*nz doubles each, or NULL: the
 * per-node divergence of eps E (0 on the PEC-wall nodes) and the per-cell
 * divergence of H.  `where` applies to all three outputs.  The reduction is
 * deterministic (fixed partition and summation order), so equal states give
 * equal sums.  A host `where` synchronises the stream (and then reports a
 * pending device error as the other synchronising calls do); a device
 * `where` is stream-ordered.  A scratch area for the partial sums is
 * allocated on the first call and kept until fdtd_destroy; host per-cell
 * outputs are staged through a temporary device array.
 * Errors: FDTD_EINVAL for a NULL sums pointer or a bad `where`. */
int fdtd_invariants(fdtd_ctx* ctx, double* sums, double* div_e, double* div_h, int where);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * reduction as fdtd_invariants with every output on the device: sums
 * (FDTD_INV_COUNT doubles, required), div_e and div_h (nx*ny*nz doubles each,
 * or NULL), all device pointers on the context's device, written in order on
 * the context's stream (nothing is synchronised or copied to the host).  The
 * call allocates nothing: the partial sums live in a static device array of
 * the library (1024 records of 8 doubles plus 8, 64 KiB in total, held on
 * every GPU the library runs on until the process ends; its address is looked
 * up once per device when a context is created).  Its size does not depend on
 * the grid, so every grid fits; a device ordinal >= 64 is refused
 * (FDTD_EUNSUPPORTED).  Every call on one GPU shares that array: calls that
 * overlap on one GPU (on different streams, or from different threads) race
 * and may return wrong sums; calls in order on one stream are safe.  Results
 * are bit-identical to fdtd_invariants on the same state.
 * Errors: FDTD_EINVAL for a NULL sums pointer. */
int fdtd_invariants_noalloc(fdtd_ctx* ctx, double* sums, double* div_e, double* div_h);

/* ---- gradient with respect to permittivity (reverse-time adjoint) -------
 *
 * The paper motivates fast FDTD by inverse design (Section 1), where a
 * solver is called for the gradient of a design objective.  The objective
 * here is a frequency-domain monitor:
 *
 *     F(r) = sum_{n=1..nsteps} E_c^n(r) exp(-i omega n dt),   r in the monitor box,
 *     J    = sum_r |F(r)|^2,
 *
 * E^n being the E field after step n of the run (E half-step and sources
 * done).  The gradient is the exact derivative of the discrete update
 * (Eq. 1 and its permutations, with cE = dt / (eps dx)): the reverse sweep
 * runs the transposed half-steps backwards in time and accumulates
 * dJ/dcE = sum_n lambda_E^n (.) CH(H^{n-1/2}) over the design box, and
 * dJ/deps = -dJ/dcE * cE / eps (0 on the tangential entries of PEC walls,
 * whose cE is pinned at 0).  With conductivity (fdtd_set_lossy_materials)
 * the update differentiated is the conductive one, sigma held fixed: the
 * reverse sweep also decays the adjoint E by ca each step and accumulates
 * dJ/dca = sum_n lambda_E^n (.) E^{n-1}, and
 * dJ/deps = (dx / dt) cb ((1 - ca) dJ/dca - cb dJ/dcb)
 * from the FP32 coefficients (0 where cb is pinned at 0).
 *
 * The run is cut into segments of checkpoint_every steps.  The forward run
 * records the design-box history of the last segment as it goes and stores
 * the state at the start of every earlier segment, which the sweep
 * recomputes.  checkpoint_every = 0 picks one segment (no checkpoint, no
 * recompute) when the whole history fits in half the device memory free at
 * the call, else 200.  The result does not depend on the segmenting. */
typedef struct {
    uint32_t struct_size;   /* = sizeof(fdtd_adjoint_spec)                      */
    int32_t mon_comp;       /* monitored component: FDTD_EX, FDTD_EY or FDTD_EZ */
    int32_t mon_lo[3];      /* monitor box [mon_lo, mon_hi) per axis            */
    int32_t mon_hi[3];
    int32_t des_lo[3];      /* design box [des_lo, des_hi) per axis             */
    int32_t des_hi[3];
    int32_t checkpoint_every;  /* steps per segment; 0 = automatic             */
    double omega;           /* angular frequency (radians per unit time)        */
    int64_t nsteps;         /* steps of the forward run, >= 1                   */
    double objective;       /* out: J (FP64)                                    */
    int64_t recomputed_steps;  /* out: forward steps run again by the sweep    */
    int32_t isotropic;      /* 0: three gradient blocks (dJ/deps_x, _y, _z);
                               1: one block, dJ/deps for a permittivity that
                               drives all three components of a cell (the
                               sum of the three, added in FP64)            */
} fdtd_adjoint_spec;

/* Run spec->nsteps steps forward from the current state (plain scheme, the
 * sources included) while accumulating F in FP64, then the reverse sweep.
 * Writes J to spec->objective and dJ/deps_c for c = x, y, z to grad_eps:
 * three FP32 blocks of the design box, each C-ordered [dx][dy][dz], laid out
 * component after component (with spec->isotropic = 1, one such block
 * holding their sum); `where` says whether grad_eps is host or device
 * memory.  On return the context holds the state after the forward run
 * (current step advanced by nsteps).  Device memory for the checkpoints
 * (one copy of the six fields per segment when there are several segments,
 * none with one), the adjoint fields and one segment's design-box history
 * (3 arrays per step, 6 with conductivity) is allocated for the call and
 * freed before it returns.
 * Errors: FDTD_EINVAL for a bad spec (component, empty or out-of-grid
 * boxes, nsteps < 1, checkpoint_every < 0, isotropic not 0 or 1,
 * struct_size), FDTD_ENOMEM when
 * the working memory does not fit; the context is unchanged in both cases.
 * Synchronises the context's stream. */
int fdtd_adjoint(fdtd_ctx* ctx, fdtd_adjoint_spec* spec, float* grad_eps, int where);

/* ---- tuning and measurement ------------------------------------------- */

enum {
    FDTD_OPT_SCHEME = 0,      /* switch scheme on a live context (state kept) */
    FDTD_OPT_BAND_STEPS = 1,  /* systolic: steps each tile stays resident:
                                 1..64, larger values act as 64; 0 = auto
                                 (a cost model per grid, shortened when the
                                 face rings of a longer band would pass the
                                 4 GB of 32-bit offsets; an explicit value
                                 that does not fit is FDTD_EUNSUPPORTED)    */
    FDTD_OPT_WORKGROUPS = 2,  /* systolic: persistent grid size, 0 = auto       */
    FDTD_OPT_SPIN_LIMIT = 3,  /* systolic: polls before a wait times out        */
    FDTD_OPT_PROFILE = 4,     /* 1 = time every kernel launch with HIP events    */
    FDTD_OPT_MATERIAL_IDS = 5,/* systolic: 1 (default) = stream per-cell material
                                 indices instead of the coefficient arrays where
                                 the context has them (FDTD_INFO_MATERIALS > 0);
                                 0 = always the arrays.  Same results.        */
    FDTD_OPT_GRAPHS = 6,      /* plain schemes: 1 (default) = calls of 16 steps
                                 or more replay a HIP graph of 16 steps
                                 (captured on first use, re-captured when the
                                 arrays, sources or scales change); 0 = one
                                 launch per kernel.  Same results; per-kernel
                                 timing (FDTD_OPT_PROFILE) launches directly. */
    FDTD_OPT_TILE_X = 7,      /* systolic: updated cells per tile along x on a
                                 lossless grid, 15, 11 or 19.  19 holds
                                 the material indices in registers: it needs
                                 them (FDTD_INFO_MATERIALS > 0), device-scope
                                 synchronisation and, on a periodic x axis,
                                 at least 20 cells, else the step returns
                                 FDTD_EUNSUPPORTED.  0 = default: 19 when
                                 every member of the launch allows it, else
                                 15.  Conductive grids always take 11; FP16
                                 storage takes 15 or 19.  A batch needs one
                                 width for all.                                */
    FDTD_OPT_AUTOTUNE_PLAIN = 8 /* 1 = fdtd_autotune also times the plain
                                 two-launch scheme (FP32 storage only, where
                                 every scheme gives the same bits) and switches
                                 the context to it when it is faster; 0
                                 (default) = systolic configurations only     */
};

/* Set a tuning option (see FDTD_OPT_*).  FDTD_EINVAL for unknown options or
 * out-of-range values. */
int fdtd_set_option(fdtd_ctx* ctx, int option, int64_t value);

/* Systolic scheme: choose the tile width along x and the band length (the
 * subdomain size and steps per exchange that Section 4 fixes by hand for one
 * GPU) by timing the candidates on this context's grid, for calls of nsteps
 * steps (runs of min(nsteps, 64) steps): widths 15 and 11 on lossless FP32
 * grids, and 19 when the grid has material indices (11 when conductive, 15
 * and 19 with FP16 storage), bands of 8, 12, 16, 24,
 * 32, 48, 64 steps and the run length itself, each run twice from the
 * current state.  The fields and step count are restored after every run
 * (a device copy of the six field arrays is held meanwhile), and the
 * fastest pair becomes the context's FDTD_OPT_TILE_X and
 * FDTD_OPT_BAND_STEPS.  The choice is kept for the process, keyed by grid
 * shape, boundaries, storage, conductivity, material indices and run length:
 * a later call with the same key takes it without timing anything.  With
 * FDTD_OPT_AUTOTUNE_PLAIN the plain two-launch scheme is timed as well (FP32
 * storage); when it is faster the context switches to it
 * (FDTD_INFO_SCHEME) and tile_x and band_steps read 0.
 * tile_x, band_steps: the chosen values, or NULL.  Synchronises.
 * Errors: FDTD_EUNSUPPORTED for another scheme or when no candidate runs,
 * FDTD_ENOMEM without room for the copy; the errors of fdtd_step. */
int fdtd_autotune(fdtd_ctx* ctx, int64_t nsteps, int64_t* tile_x, int64_t* band_steps);

enum {
    FDTD_KERNEL_PLAIN_E = 0,   /* plain E half-step                        */
    FDTD_KERNEL_PLAIN_H = 1,   /* plain H half-step                        */
    FDTD_KERNEL_SOURCES = 2,   /* plain-scheme point-source injection      */
    FDTD_KERNEL_SYSTOLIC = 3,  /* persistent systolic kernel               */
    FDTD_KERNEL_PLAIN_FUSED = 4, /* fused plain step (one launch per step) */
    FDTD_KERNEL_COUNT = 5
};

/* With FDTD_OPT_PROFILE on, the number of launches of a kernel and their
 * total device time in milliseconds (HIP events on the context's stream).
 * Synchronises the stream.  FDTD_OPT_PROFILE = 1 also resets the counters. */
int fdtd_kernel_stats(fdtd_ctx* ctx, int kernel, int64_t* launches, double* total_ms);

enum {
    FDTD_INFO_SYSTOLIC_GRID = 0,   /* persistent workgroups of the last systolic launch */
    FDTD_INFO_SYSTOLIC_BAND = 1,   /* steps per band of the last systolic launch         */
    FDTD_INFO_SYSTOLIC_TICKETS = 2,/* (band, tile) tickets of the last systolic launch    */
    FDTD_INFO_RING_SLOTS = 3,      /* face-ring slots of the last systolic launch        */
    FDTD_INFO_TILE_X = 4,          /* updated cells per systolic tile along x, y, z (x:  */
                                   /* 15, 11 or 19: FDTD_OPT_TILE_X; y and z: 15)         */
    FDTD_INFO_TILE_Y = 5,
    FDTD_INFO_TILE_Z = 6,
    FDTD_INFO_MATERIALS = 7,       /* entries of the context's material table, entry 0 */
                                   /* (+0, +0, +0) included; 0 = none (conductive, or  */
                                   /* more than 256 distinct triples)                   */
    FDTD_INFO_SCHEME = 8           /* the context's scheme (FDTD_SCHEME_*)              */
};

/* Read a piece of launch information (FDTD_INFO_*) into *value; 0 before the
 * first systolic launch.  FDTD_EINVAL for unknown keys or NULL arguments. */
int fdtd_get_info(const fdtd_ctx* ctx, int key, int64_t* value);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_H */
