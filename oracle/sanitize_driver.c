/*
 * sanitize_driver.c -- runs every entry point of the oracle's C core on
 * ghosted patches whose arrays are allocated at exactly the documented sizes,
 * for an AddressSanitizer / UndefinedBehaviorSanitizer build (test
 * infrastructure, like the oracle itself):
 *
 *   gcc -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all \
 *       -fno-omit-frame-pointer -ffp-contract=off oracle/oracle.c \
 *       oracle/sanitize_driver.c -lm -o <exe>
 *
 * Patches: spherical and cartesian, 8 and 9 variables (the CME density
 * tracer), every limiter, odd interior sizes; states smooth with rho, p > 0.
 * Any out-of-bounds access, use of freed memory, signed overflow, misaligned
 * load or similar aborts the run with the sanitizer's report; the program also
 * checks that every output is finite.  Prints "ok" and exits 0 otherwise.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ni, nj, nk;
    int cartesian;
    const double *f0, *f1, *f2;
    double gamma, omega, gm;
    int limiter;
    int nv;
} ora_patch;

void ora_prim(const double *u, double *w, double gamma);
void ora_cons(const double *w, double *u, double gamma);
double ora_fast_speed(const double *w, int d, double gamma);
void ora_flux(const double *w, int d, double gamma, double *f);
void ora_rusanov(const double *wl, const double *wr, int d, double gamma, double *f);
double ora_slope(int limiter, double wm, double w0, double wp, double xm, double x0, double xp);
int ora_rhs(const ora_patch *p, const double *U, double *L, double *F0, double *F1, double *F2);
int ora_rhs_hancock(const ora_patch *p, const double *U, double *L);
double ora_max_rate(const ora_patch *p, const double *U);
void ora_indicator(const ora_patch *p, const double *U, double eps, double *E_rho, double *E_v, double *divv,
                   double *divscale);
void ora_divb(const ora_patch *p, const double *U, double *D);

static int failures = 0;

static void check_finite(const char *what, const double *a, size_t n)
{
    for (size_t q = 0; q < n; ++q)
        if (!isfinite(a[q])) {
            fprintf(stderr, "%s: non-finite value at %zu\n", what, q);
            ++failures;
            return;
        }
}

/* exact-size heap copy, so that the sanitizer sees the array's true end */
static double *alloc(size_t n)
{
    double *a = (double *)malloc(n * sizeof(double));
    if (!a) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    for (size_t q = 0; q < n; ++q) a[q] = NAN;
    return a;
}

static void run_patch(int cartesian, int nv, int limiter, int ni, int nj, int nk)
{
    const double gamma = 1.5;
    double *f[3];
    const int n[3] = {ni, nj, nk};
    for (int d = 0; d < 3; ++d) {
        f[d] = alloc((size_t)n[d] + 5);
        for (int m = 0; m < n[d] + 5; ++m) {
            const double x = (m - 2) / (double)n[d];
            if (cartesian) f[d][m] = x * (1.0 + 0.1 * d);
            else if (d == 0) f[d][m] = 0.2 * exp(0.9 * x);                 /* stretched r, AU */
            else if (d == 1) f[d][m] = 1.0 + 1.1 * x;                      /* colatitude, rad */
            else f[d][m] = 0.3 + 1.5 * x;                                   /* longitude, rad */
        }
    }
    ora_patch p = {ni, nj, nk, cartesian, f[0], f[1], f[2], gamma, cartesian ? 0.0 : 0.06, cartesian ? 0.0 : 0.3,
                   limiter, nv};
    const size_t G = (size_t)(ni + 4) * (nj + 4) * (nk + 4), C = (size_t)ni * nj * nk;
    double *U = alloc((size_t)nv * G);
    for (int k = 0; k < nk + 4; ++k)
        for (int j = 0; j < nj + 4; ++j)
            for (int i = 0; i < ni + 4; ++i) {
                const double x = i / (double)(ni + 4), y = j / (double)(nj + 4), z = k / (double)(nk + 4);
                double w[9] = {1.0 + 0.3 * sin(6.0 * x + 2.0 * z), 0.4 + 0.1 * cos(5.0 * y), 0.05 * sin(3.0 * z),
                               -0.1 + 0.05 * x, 0.8 + 0.2 * cos(4.0 * x + y), 0.3 + 0.1 * y, 0.1 * sin(2.0 * x),
                               -0.2 + 0.1 * z, 0.5 + 0.4 * sin(7.0 * x * y)};
                double u[9];
                ora_cons(w, u, gamma);
                u[8] = w[0] * w[8];
                const size_t cell = ((size_t)k * (nj + 4) + j) * (ni + 4) + i;
                for (int v = 0; v < nv; ++v) U[(size_t)v * G + cell] = u[v];
            }
    double *L = alloc((size_t)nv * C);
    double *F0 = alloc((size_t)nv * nk * nj * (ni + 1));
    double *F1 = alloc((size_t)nv * nk * (nj + 1) * ni);
    double *F2 = alloc((size_t)nv * (nk + 1) * nj * ni);
    int bad = ora_rhs(&p, U, L, F0, F1, F2);
    if (bad) {
        fprintf(stderr, "ora_rhs: %d non-physical cells\n", bad);
        ++failures;
    }
    check_finite("L", L, (size_t)nv * C);
    check_finite("F0", F0, (size_t)nv * nk * nj * (ni + 1));
    check_finite("F1", F1, (size_t)nv * nk * (nj + 1) * ni);
    check_finite("F2", F2, (size_t)nv * (nk + 1) * nj * ni);
    bad = ora_rhs(&p, U, L, NULL, NULL, NULL);
    bad += ora_rhs_hancock(&p, U, L);
    if (bad) ++failures;
    check_finite("L_H", L, (size_t)nv * C);
    const double rate = ora_max_rate(&p, U);
    if (!(rate > 0.0 && isfinite(rate))) {
        fprintf(stderr, "rate %g\n", rate);
        ++failures;
    }
    double *Er = alloc(C), *Ev = alloc(C), *dv = alloc(C), *ds = alloc(C), *D = alloc(C);
    ora_indicator(&p, U, 0.01, Er, Ev, dv, ds);
    ora_divb(&p, U, D);
    check_finite("E_rho", Er, C);
    check_finite("E_v", Ev, C);
    check_finite("divv", dv, C);
    check_finite("divscale", ds, C);
    check_finite("divb", D, C);
    free(Er), free(Ev), free(dv), free(ds), free(D);
    free(L), free(F0), free(F1), free(F2), free(U);
    for (int d = 0; d < 3; ++d) free(f[d]);
}

int main(void)
{
    /* pointwise entry points */
    const double w[8] = {1.2, 0.3, -0.1, 0.2, 0.7, 0.4, -0.3, 0.1};
    double u[8], w2[8], fl[8], fr[8];
    ora_cons(w, u, 1.5);
    ora_prim(u, w2, 1.5);
    for (int d = 0; d < 3; ++d) {
        ora_flux(w, d, 1.5, fl);
        ora_rusanov(w, w2, d, 1.5, fr);
        check_finite("flux", fl, 8);
        check_finite("rusanov", fr, 8);
        const double c = ora_fast_speed(w, d, 1.5);
        if (!(c > 0.0)) ++failures;
    }
    for (int lim = 0; lim < 3; ++lim) {
        const double s = ora_slope(lim, 1.0, 1.5, 1.7, 0.0, 1.0, 2.5);
        if (!isfinite(s)) ++failures;
    }
    /* patches */
    for (int cart = 0; cart < 2; ++cart)
        for (int nv = 8; nv <= 9; ++nv)
            for (int lim = 0; lim < 3; ++lim) {
                run_patch(cart, nv, lim, 5, 3, 4);
                run_patch(cart, nv, lim, 1, 1, 1);
            }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
