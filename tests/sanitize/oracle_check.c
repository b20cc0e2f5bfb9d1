/* Exercise of the C oracle (oracle/yee_oracle.c) built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_sanitizers_cpu.py: every entry
 * point on thin and odd grids, all eight boundary mixes, sources on the first
 * and last cells, FP64 and FP32 and the conductive step.  Exits non-zero if a
 * result is not finite, a PEC-frozen entry leaves +0, or FP32 strays from
 * FP64 by more than 1e-5 (relative L2) after a few steps. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t comp, i, j, k;
    const float* w;
    int64_t len, first_step;
} oracle_source;

void oracle_coeff_E(int, int, int, const int32_t*, double, double, int, const float*, double*);
void oracle_coeff_lossy(int, int, int, const int32_t*, double, double, int, const float*, const float*, double*,
                        double*);
void oracle_step_f64(int, int, int, const double*, const double*, const double*, double, double*, double*, double*,
                     double*, double*, double*, int64_t, int64_t, const oracle_source*, int);
void oracle_step_f32(int, int, int, const float*, const float*, const float*, float, float*, float*, float*,
                     float*, float*, float*, int64_t, int64_t, const oracle_source*, int);
void oracle_step_lossy_f64(int, int, int, const double*, const double*, const double*, const double*,
                           const double*, const double*, double, double*, double*, double*, double*, double*,
                           double*, int64_t, int64_t, const oracle_source*, int);
void oracle_step_lossy_f32(int, int, int, const float*, const float*, const float*, const float*, const float*,
                           const float*, float, float*, float*, float*, float*, float*, float*, int64_t, int64_t,
                           const oracle_source*, int);
void oracle_half_E_f32(int, int, int, const float*, const float*, const float*, float*, float*, float*,
                       const float*, const float*, const float*);
void oracle_half_H_f32(int, int, int, float, const float*, const float*, const float*, float*, float*, float*);
void oracle_round_f32(const double*, float*, int64_t);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static int frozen(int c, int i, int j, int k, const int32_t bc[3])
{
    const int co[3] = {i, j, k};
    for (int a = 0; a < 3; ++a)
        if (a != c && bc[a] == 0 && co[a] == 0) return 1;
    return 0;
}

static int run_case(int nx, int ny, int nz, const int32_t bc[3], int lossy)
{
    const size_t n = (size_t)nx * ny * nz;
    float* eps = malloc(n * sizeof(float));
    float* sig = malloc(n * sizeof(float));
    double *c64[3], *a64[3];
    float *c32[3], *a32[3];
    double* f64[6];
    float* f32[6];
    for (size_t p = 0; p < n; ++p) {
        eps[p] = (float)(1.0 + 11.0 * urand());
        sig[p] = (float)(0.3 * urand());
    }
    for (int c = 0; c < 3; ++c) {
        c64[c] = malloc(n * sizeof(double));
        a64[c] = malloc(n * sizeof(double));
        c32[c] = malloc(n * sizeof(float));
        a32[c] = malloc(n * sizeof(float));
        if (lossy)
            oracle_coeff_lossy(nx, ny, nz, bc, 0.5, 1.0, c, eps, sig, a64[c], c64[c]);
        else
            oracle_coeff_E(nx, ny, nz, bc, 0.5, 1.0, c, eps, c64[c]);
        oracle_round_f32(c64[c], c32[c], (int64_t)n);
        oracle_round_f32(a64[c], a32[c], lossy ? (int64_t)n : 0);
    }
    for (int q = 0; q < 6; ++q) {
        f64[q] = malloc(n * sizeof(double));
        f32[q] = malloc(n * sizeof(float));
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j)
                for (int k = 0; k < nz; ++k) {
                    const size_t p = ((size_t)i * ny + j) * nz + k;
                    float v = (float)(0.2 * urand() - 0.1);
                    if (q < 3 && frozen(q, i, j, k, bc)) v = 0.0f;
                    f32[q][p] = v;
                    f64[q][p] = v;
                }
    }
    float wave[8] = {0.5f, -0.25f, 0.125f, 1.0f, -1.0f, 0.75f, 0.3f, -0.6f};
    oracle_source src[2] = {{2, nx - 1, ny - 1, nz - 1, wave, 8, 0}, {0, nx / 2, ny / 2, nz / 2, wave, 5, 1}};
    int nsrc = 0;
    if (!frozen(2, nx - 1, ny - 1, nz - 1, bc)) src[nsrc++] = src[0];
    if (!frozen(0, nx / 2, ny / 2, nz / 2, bc)) src[nsrc++] = (oracle_source){0, nx / 2, ny / 2, nz / 2, wave, 5, 1};
    const int steps = 6;
    if (lossy) {
        oracle_step_lossy_f64(nx, ny, nz, a64[0], a64[1], a64[2], c64[0], c64[1], c64[2], 0.5, f64[0], f64[1], f64[2],
                              f64[3], f64[4], f64[5], steps, 0, src, nsrc);
        oracle_step_lossy_f32(nx, ny, nz, a32[0], a32[1], a32[2], c32[0], c32[1], c32[2], 0.5f, f32[0], f32[1],
                              f32[2], f32[3], f32[4], f32[5], steps, 0, src, nsrc);
    } else {
        oracle_step_f64(nx, ny, nz, c64[0], c64[1], c64[2], 0.5, f64[0], f64[1], f64[2], f64[3], f64[4], f64[5],
                        steps, 0, src, nsrc);
        oracle_step_f32(nx, ny, nz, c32[0], c32[1], c32[2], 0.5f, f32[0], f32[1], f32[2], f32[3], f32[4], f32[5],
                        steps, 0, src, nsrc);
        oracle_half_E_f32(nx, ny, nz, c32[0], c32[1], c32[2], f32[0], f32[1], f32[2], f32[3], f32[4], f32[5]);
        oracle_half_H_f32(nx, ny, nz, 0.5f, f32[0], f32[1], f32[2], f32[3], f32[4], f32[5]);
        oracle_half_E_f32(nx, ny, nz, c32[0], c32[1], c32[2], f32[0], f32[1], f32[2], f32[3], f32[4], f32[5]);
        oracle_half_H_f32(nx, ny, nz, 0.5f, f32[0], f32[1], f32[2], f32[3], f32[4], f32[5]);
        oracle_step_f64(nx, ny, nz, c64[0], c64[1], c64[2], 0.5, f64[0], f64[1], f64[2], f64[3], f64[4], f64[5], 2,
                        steps, src, 0);
    }
    double num = 0.0, den = 0.0;
    int bad = 0;
    for (int q = 0; q < 6; ++q)
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j)
                for (int k = 0; k < nz; ++k) {
                    const size_t p = ((size_t)i * ny + j) * nz + k;
                    if (!isfinite(f32[q][p]) || !isfinite(f64[q][p])) bad = 1;
                    if (q < 3 && frozen(q, i, j, k, bc) && (f32[q][p] != 0.0f || signbit(f32[q][p]))) bad = 1;
                    const double d = (double)f32[q][p] - f64[q][p];
                    num += d * d;
                    den += f64[q][p] * f64[q][p];
                }
    const double rel = sqrt(num / (den > 0 ? den : 1.0));
    if (rel > 1e-5) bad = 1;
    if (bad)
        fprintf(stderr, "case %dx%dx%d bc %d%d%d lossy %d: rel %g\n", nx, ny, nz, bc[0], bc[1], bc[2], lossy, rel);
    for (int c = 0; c < 3; ++c) {
        free(c64[c]);
        free(a64[c]);
        free(c32[c]);
        free(a32[c]);
    }
    for (int q = 0; q < 6; ++q) {
        free(f64[q]);
        free(f32[q]);
    }
    free(eps);
    free(sig);
    return bad;
}

int main(void)
{
    const int shapes[][3] = {{8, 8, 8}, {1, 6, 11}, {5, 1, 3}, {2, 3, 1}, {9, 7, 16}, {1, 1, 1}};
    int bad = 0, ncase = 0;
    for (unsigned s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (int m = 0; m < 8; ++m)
            for (int lossy = 0; lossy < 2; ++lossy) {
                const int32_t bc[3] = {m & 1, (m >> 1) & 1, (m >> 2) & 1};
                bad |= run_case(shapes[s][0], shapes[s][1], shapes[s][2], bc, lossy);
                ++ncase;
            }
    printf("oracle exercise: %d cases, %s\n", ncase, bad ? "FAILED" : "passed");
    return bad;
}
