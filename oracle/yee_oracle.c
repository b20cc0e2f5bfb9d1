/*
 * CPU oracle for the 3D Yee FDTD leapfrog update -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct definition that the GPU
 * path is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product library never does,
 * and the two share no code.
 *
 * What it computes (paper: Section 2, Eq. (1), and the E-then-H ordering of
 * the horizontal-bar scheme in the caption of Fig. 7):
 *
 *   State: Ex,Ey,Ez,Hx,Hy,Hz, each an nx*ny*nz array in C order (z fastest).
 *   Yee positions in units of the cell size: Ex at (i+1/2,j,k), Ey at
 *   (i,j+1/2,k), Ez at (i,j,k+1/2), Hx at (i,j+1/2,k+1/2), Hy at
 *   (i+1/2,j,k+1/2), Hz at (i+1/2,j+1/2,k).  This is the placement under
 *   which Eq. (1) reads H_z at j-1 and H_y at k-1.
 *
 *   One step (E first, then H; all index arithmetic modulo n on every axis):
 *     Ex = (Ex + cEx*(Hz - Hz[j-1])) - cEx*(Hy - Hy[k-1])          -- Eq. (1)
 *     Ey = (Ey + cEy*(Hx - Hx[k-1])) - cEy*(Hz - Hz[i-1])          -- cyclic
 *     Ez = (Ez + cEz*(Hy - Hy[i-1])) - cEz*(Hx - Hx[j-1])          -- cyclic
 *     sources: E_c[p] += w[m]  (soft additive source)
 *     Hx = (Hx - cH*(Ez[j+1] - Ez)) + cH*(Ey[k+1] - Ey)            -- Faraday
 *     Hy = (Hy - cH*(Ex[k+1] - Ex)) + cH*(Ez[i+1] - Ez)
 *     Hz = (Hz - cH*(Ey[i+1] - Ey)) + cH*(Ex[j+1] - Ex)
 *
 *   Each of the six operations per component (difference, product, sum,
 *   difference, product, difference) rounds once, left to right: Eq. (1)
 *   keeps its two separate products with dt/dy and dt/dz (Section 2 counts
 *   six flops per component), so neither side factors them.  This file must
 *   be compiled with -ffp-contract=off and without fast-math.
 *
 *   Materials: the paper's implementation multiplies the curl by per-cell
 *   "structural fields" (Section 4).  Here cE_c = dt/(eps_c*dx) per component
 *   per cell, computed in double; the FP32 oracle stores it rounded to float.
 *   cH = dt/dx (mu = 1, normalised units as in Eq. (1)).
 *
 *   Boundaries: the domain is periodic on every axis.  A PEC axis a
 *   additionally has cE = 0 for the two E components tangential to the
 *   planes normal to a on the index-0 plane; with those entries held at +0
 *   this closes a perfectly conducting box with its walls at 0 == n.
 *
 * Two element types are provided, double and float, with identical
 * operation order.  OpenMP parallelises over i-planes only: every cell's
 * arithmetic is independent of the thread count.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef struct {
    int32_t comp;           /* 0 = Ex, 1 = Ey, 2 = Ez                          */
    int32_t i, j, k;        /* cell                                            */
    const float* w;         /* waveform samples (FP32, computed by the caller) */
    int64_t len;            /* number of samples                               */
    int64_t first_step;     /* sample m is added in the step that starts at
                               step count first_step + m                     */
} oracle_source;

#define IDX(i, j, k) (((size_t)(i) * (size_t)ny + (size_t)(j)) * (size_t)nz + (size_t)(k))

/* cE for one component: dt / (eps * dx) in double; zero on the index-0 plane
 * of every PEC axis to which the component is tangential.  bc[a] = 0 means
 * PEC on axis a, 1 means periodic. */
void oracle_coeff_E(int nx, int ny, int nz, const int32_t bc[3], double dt, double dx,
                    int comp, const float* eps, double* out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                size_t p = IDX(i, j, k);
                double c = dt / ((double)eps[p] * dx);
                int coord[3] = {i, j, k};
                for (int a = 0; a < 3; ++a)
                    if (a != comp && bc[a] == 0 && coord[a] == 0) c = 0.0;
                out[p] = c;
            }
}

/* H half-step (shared by the lossless and lossy steps): reads the new E at
 * the forward neighbours. */
#define H_HALF_STEP(T)                                                                    \
        _Pragma("omp parallel for schedule(static)")                                      \
        for (int i = 0; i < nx; ++i) {                                                    \
            int ip = (i == nx - 1) ? 0 : i + 1;                                           \
            for (int j = 0; j < ny; ++j) {                                                \
                int jp = (j == ny - 1) ? 0 : j + 1;                                       \
                for (int k = 0; k < nz; ++k) {                                            \
                    int kp = (k == nz - 1) ? 0 : k + 1;                                   \
                    size_t p = IDX(i, j, k);                                              \
                    T a, b;                                                               \
                    a = Hx[p] - cH * (Ez[IDX(i, jp, k)] - Ez[p]);                         \
                    b = cH * (Ey[IDX(i, j, kp)] - Ey[p]);                                 \
                    Hx[p] = a + b;                                                        \
                    a = Hy[p] - cH * (Ex[IDX(i, j, kp)] - Ex[p]);                         \
                    b = cH * (Ez[IDX(ip, j, k)] - Ez[p]);                                 \
                    Hy[p] = a + b;                                                        \
                    a = Hz[p] - cH * (Ey[IDX(ip, j, k)] - Ey[p]);                         \
                    b = cH * (Ex[IDX(i, jp, k)] - Ex[p]);                                 \
                    Hz[p] = a + b;                                                        \
                }                                                                         \
            }                                                                             \
        }

/* E half-step: reads H at the backward neighbours. */
#define E_HALF_STEP(T)                                                                    \
        _Pragma("omp parallel for schedule(static)")                                      \
        for (int i = 0; i < nx; ++i) {                                                    \
            int im = (i == 0) ? nx - 1 : i - 1;                                           \
            for (int j = 0; j < ny; ++j) {                                                \
                int jm = (j == 0) ? ny - 1 : j - 1;                                       \
                for (int k = 0; k < nz; ++k) {                                            \
                    int km = (k == 0) ? nz - 1 : k - 1;                                   \
                    size_t p = IDX(i, j, k);                                              \
                    T a, b;                                                               \
                    a = Ex[p] + cEx[p] * (Hz[p] - Hz[IDX(i, jm, k)]);                     \
                    b = cEx[p] * (Hy[p] - Hy[IDX(i, j, km)]);                             \
                    Ex[p] = a - b;                                                        \
                    a = Ey[p] + cEy[p] * (Hx[p] - Hx[IDX(i, j, km)]);                     \
                    b = cEy[p] * (Hz[p] - Hz[IDX(im, j, k)]);                             \
                    Ey[p] = a - b;                                                        \
                    a = Ez[p] + cEz[p] * (Hy[p] - Hy[IDX(im, j, k)]);                     \
                    b = cEz[p] * (Hx[p] - Hx[IDX(i, jm, k)]);                             \
                    Ez[p] = a - b;                                                        \
                }                                                                         \
            }                                                                             \
        }

#define DEFINE_STEP(T, NAME)                                                              \
void NAME(int nx, int ny, int nz, const T* cEx, const T* cEy, const T* cEz, T cH,         \
          T* Ex, T* Ey, T* Ez, T* Hx, T* Hy, T* Hz, int64_t nsteps, int64_t step0,         \
          const oracle_source* src, int nsrc)                                             \
{                                                                                         \
    for (int64_t s = step0; s < step0 + nsteps; ++s) {                                    \
        E_HALF_STEP(T)                                                                    \
        /* soft sources, after the E half-step */                                         \
        for (int q = 0; q < nsrc; ++q) {                                                  \
            int64_t m = s - src[q].first_step;                                            \
            if (m < 0 || m >= src[q].len) continue;                                       \
            T* f = src[q].comp == 0 ? Ex : (src[q].comp == 1 ? Ey : Ez);                  \
            size_t p = IDX(src[q].i, src[q].j, src[q].k);                                 \
            f[p] = f[p] + (T)src[q].w[m];                                                 \
        }                                                                                 \
        H_HALF_STEP(T)                                                                    \
    }                                                                                     \
}

DEFINE_STEP(double, oracle_step_f64)
DEFINE_STEP(float, oracle_step_f32)

/* The two half-steps on their own (no sources), for callers that act on the
 * state between them (the FP16-storage rounding of the plain scheme). */
void oracle_half_E_f32(int nx, int ny, int nz, const float* cEx, const float* cEy,
                       const float* cEz, float* Ex, float* Ey, float* Ez, const float* Hx,
                       const float* Hy, const float* Hz)
{
    E_HALF_STEP(float)
}

void oracle_half_H_f32(int nx, int ny, int nz, float cH, const float* Ex, const float* Ey,
                       const float* Ez, float* Hx, float* Hy, float* Hz)
{
    H_HALF_STEP(float)
}

/*
 * Lossy materials (the conductivity "structural fields" of Section 4).
 * With conductivity sigma, Ampere's law eps dE/dt + sigma E = curl H is
 * discretised semi-implicitly (sigma E at the half-step mean of the old and
 * new E), which gives, per component c,
 *
 *   E = (ca*E + cb*(d1)) - cb*(d2),
 *   ca = (1 - h) / (1 + h),  cb = (dt / (eps dx)) / (1 + h),  h = sigma dt / (2 eps),
 *
 * with d1, d2 the same differences as in the lossless step.  With sigma = 0,
 * ca = 1 and cb = dt/(eps dx) exactly, and 1*E = E, so this step equals the
 * lossless one bit for bit.  On PEC-tangential index-0 entries ca = 1 and
 * cb = 0 (the entry stays +0).  The H half-step is unchanged.
 */
void oracle_coeff_lossy(int nx, int ny, int nz, const int32_t bc[3], double dt, double dx,
                        int comp, const float* eps, const float* sigma, double* ca, double* cb)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                size_t p = IDX(i, j, k);
                double e = (double)eps[p];
                double h = (double)sigma[p] * dt / (2.0 * e);
                double a = (1.0 - h) / (1.0 + h);
                double b = (dt / (e * dx)) / (1.0 + h);
                int coord[3] = {i, j, k};
                for (int d = 0; d < 3; ++d)
                    if (d != comp && bc[d] == 0 && coord[d] == 0) {
                        a = 1.0;
                        b = 0.0;
                    }
                ca[p] = a;
                cb[p] = b;
            }
}

#define DEFINE_STEP_LOSSY(T, NAME)                                                        \
void NAME(int nx, int ny, int nz, const T* cax, const T* cay, const T* caz, const T* cbx, \
          const T* cby, const T* cbz, T cH, T* Ex, T* Ey, T* Ez, T* Hx, T* Hy, T* Hz,     \
          int64_t nsteps, int64_t step0, const oracle_source* src, int nsrc)             \
{                                                                                         \
    for (int64_t s = step0; s < step0 + nsteps; ++s) {                                    \
        _Pragma("omp parallel for schedule(static)")                                      \
        for (int i = 0; i < nx; ++i) {                                                    \
            int im = (i == 0) ? nx - 1 : i - 1;                                           \
            for (int j = 0; j < ny; ++j) {                                                \
                int jm = (j == 0) ? ny - 1 : j - 1;                                       \
                for (int k = 0; k < nz; ++k) {                                            \
                    int km = (k == 0) ? nz - 1 : k - 1;                                   \
                    size_t p = IDX(i, j, k);                                              \
                    T a, b;                                                               \
                    a = cax[p] * Ex[p] + cbx[p] * (Hz[p] - Hz[IDX(i, jm, k)]);            \
                    b = cbx[p] * (Hy[p] - Hy[IDX(i, j, km)]);                             \
                    Ex[p] = a - b;                                                        \
                    a = cay[p] * Ey[p] + cby[p] * (Hx[p] - Hx[IDX(i, j, km)]);            \
                    b = cby[p] * (Hz[p] - Hz[IDX(im, j, k)]);                             \
                    Ey[p] = a - b;                                                        \
                    a = caz[p] * Ez[p] + cbz[p] * (Hy[p] - Hy[IDX(im, j, k)]);            \
                    b = cbz[p] * (Hx[p] - Hx[IDX(i, jm, k)]);                             \
                    Ez[p] = a - b;                                                        \
                }                                                                         \
            }                                                                             \
        }                                                                                 \
        for (int q = 0; q < nsrc; ++q) {                                                  \
            int64_t m = s - src[q].first_step;                                            \
            if (m < 0 || m >= src[q].len) continue;                                       \
            T* f = src[q].comp == 0 ? Ex : (src[q].comp == 1 ? Ey : Ez);                  \
            size_t p = IDX(src[q].i, src[q].j, src[q].k);                                 \
            f[p] = f[p] + (T)src[q].w[m];                                                 \
        }                                                                                 \
        H_HALF_STEP(T)                                                                    \
    }                                                                                     \
}

/* Round an FP64 coefficient array to FP32 (the FP32 oracle's structural field). */
void oracle_round_f32(const double* in, float* out, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) out[p] = (float)in[p];
}

/* Number of OpenMP threads a parallel region would use (for reporting). */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_threads(int n) { (void)n; }
#endif

DEFINE_STEP_LOSSY(double, oracle_step_lossy_f64)
DEFINE_STEP_LOSSY(float, oracle_step_lossy_f32)
