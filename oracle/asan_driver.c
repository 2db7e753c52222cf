/*
 * Sanitizer driver for the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Compiled together with h2d_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py, it runs the
 * oracle's entry points (build, matvec, GMRES, export, free) on small
 * deterministic inputs that reach its edge cases: one point, a ragged tree,
 * points on cell boundaries, a clustered set with empty boxes, zero
 * tolerance (every block dense), duplicates (EDUP) and bad arguments.
 * Any out-of-bounds access, leak or undefined operation ends the run with
 * a sanitizer report and a nonzero status.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct { int32_t kind, diag_mode; double c, diag_value; } kern_t;
typedef struct orc_h orc_h;
int orc_build(const double* xy, int64_t n, const kern_t* k, int32_t leaf_max, double tol, int32_t fac, orc_h** out);
int orc_matvec(const orc_h* h, const double* psi, double* b);
int orc_gmres(const orc_h* h, const double* b, double* x, double tol, int32_t restart, int32_t max_iter,
              int32_t* iters, double* relres);
int orc_export(const orc_h* h, const char* path);
void orc_free(orc_h* h);

/* splitmix64 (Steele, Lea and Flood 2014): a fixed, seedable source of
 * test coordinates */
static uint64_t sm_state = 1;
static double unif(void)
{
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int run(const char* what, const double* xy, int64_t n, kern_t k, int leaf, double tol, const char* path)
{
    orc_h* h = NULL;
    int st = orc_build(xy, n, &k, leaf, tol, 1, &h);
    if (st) { printf("%s: build status %d\n", what, st); return st; }
    double* x = malloc(sizeof(double) * (size_t)n);
    double* y = malloc(sizeof(double) * (size_t)n);
    double* z = malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) x[i] = unif();
    orc_matvec(h, x, y);
    int32_t it = 0;
    double rr = 0.0;
    int gs = orc_gmres(h, y, z, 1e-10, 20, 60, &it, &rr);
    if (path) orc_export(h, path);
    printf("%s: n=%lld gmres status %d its %d relres %.2e\n", what, (long long)n, gs, it, rr);
    free(x); free(y); free(z);
    orc_free(h);
    return 0;
}

int main(int argc, char** argv)
{
    const char* path = argc > 1 ? argv[1] : NULL;
    kern_t logk = {0, 0, 0.0, 0.0}, mq = {2, 1, 0.3, 1e-3}, gauss = {3, 1, 0.05, 1e-2}, invr = {1, 0, 0.0, 0.0};
    double one[2] = {0.25, -0.5};
    logk.diag_value = 1.0;
    if (run("one point", one, 1, logk, 4, 1e-10, NULL)) return 1;
    enum { N = 700 };
    static double xy[2 * N];
    for (int i = 0; i < 2 * N; ++i) xy[i] = unif();
    logk.diag_value = N;
    if (run("uniform log", xy, N, logk, 16, 1e-10, path)) return 1;
    if (run("uniform mq, ragged leaves", xy, 333, mq, 7, 1e-8, NULL)) return 1;
    if (run("zero tolerance", xy, 200, mq, 8, 0.0, NULL)) return 1;
    /* points on dyadic cell boundaries, including the closed top/right edge */
    static double grid[2 * 289];
    for (int a = 0; a < 17; ++a)
        for (int b = 0; b < 17; ++b) { grid[2 * (a * 17 + b)] = -1.0 + a / 8.0; grid[2 * (a * 17 + b) + 1] = -1.0 + b / 8.0; }
    if (run("boundary grid 1/r", grid, 289, invr, 9, 1e-10, NULL)) return 1;
    /* two tight clusters: deep tree, most boxes empty */
    static double cl[2 * 400];
    for (int i = 0; i < 400; ++i) {
        double c = (i & 1) ? 0.5 : -0.5;
        cl[2 * i] = c + 0.01 * unif();
        cl[2 * i + 1] = c + 0.01 * unif();
    }
    if (run("clusters gauss", cl, 400, gauss, 10, 1e-10, NULL)) return 1;
    /* errors: duplicates with a kernel singular at r = 0, bad sizes */
    double dup[6] = {0.1, 0.2, 0.5, 0.5, 0.1, 0.2};
    orc_h* h = NULL;
    kern_t l3 = {0, 0, 0.0, 3.0};
    if (orc_build(dup, 3, &l3, 8, 1e-10, 1, &h) != 4 || h) { printf("duplicates not refused\n"); return 1; }
    if (orc_build(dup, 0, &l3, 8, 1e-10, 1, &h) == 0) { printf("n = 0 not refused\n"); return 1; }
    printf("sanitizer driver done\n");
    return 0;
}
