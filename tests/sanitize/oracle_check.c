/* The oracle's C functions on small inputs, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitize_cpu.py (one thread).  Alongside the memory
 * and undefined-behaviour checks of the sanitizers it checks a few closed forms: d^l_{00}(0) = 1,
 * d^l_{ll}(beta) = cos^{2l}(beta/2), and that a column's u from oracle_totalconv_u equals the
 * sum over rings of d^l times the cotangent taken from oracle_wigner_d.  Prints "ok" and exits
 * with status 0, or the first failed check and status 1. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef long double ld;

int oracle_wigner_d(int lmax, int npair, const int* mb, const int* ms, int nring, const double* xring,
                    double* d, double* mant, long long* ex, int nthreads);
int oracle_totalconv_fwd(int lmax, int mbmax, int nring, const double* xring, const double* alm,
                         const double* blm, int ncol, const int* cmb, const int* cms, int nsel,
                         const int* ring_sel, double eps, double* C, int nthreads);
int oracle_totalconv_u(int lmax, int mbmax, int nring, const double* xring, const double* G, int ncol,
                       const int* cmb, const int* cms, ld* u, int nthreads);
int oracle_ring_grid_x(int nring, const double* beta, double* x);
int oracle_datacube(int lmax, int mbmax, int nring, const double* C, int nalpha, int ngamma, int npts,
                    const int* ring, const int* ia, const int* ig, double* out, int nthreads);

static int failed = 0;

static void check(int ok, const char* what)
{
    printf("%s %s\n", ok ? "pass" : "FAIL", what);
    if (!ok) failed = 1;
}

static double urand(unsigned* s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0 - 0.5;
}

int main(void)
{
    enum { L = 16, NR = 9, M = 3 };
    const ld pi = 3.14159265358979323846264338327950288L;
    double beta[NR], x[NR];
    for (int j = 0; j < NR; ++j) beta[j] = (double)(j * pi / (NR - 1));   /* poles included */
    check(oracle_ring_grid_x(NR, beta, x) == 0 && x[0] == 1.0 && x[NR - 1] == -1.0, "ring_grid_x with the poles");

    const int pmb[4] = {0, 3, -2, 5}, pms[4] = {0, -2, 7, 5};
    double* d = malloc(sizeof(double) * 4 * (L + 1) * NR);
    double* mant = malloc(sizeof(double) * 4 * (L + 1) * NR);
    long long* ex = malloc(sizeof(long long) * 4 * (L + 1) * NR);
    check(oracle_wigner_d(L, 4, pmb, pms, NR, x, d, mant, ex, 1) == 0, "wigner_d runs");
    int one = 1, diag = 1;
    for (int l = 0; l <= L; ++l) one = one && fabs(d[(size_t)l * NR + 0] - 1.0) < 1e-15;
    for (int j = 0; j < NR; ++j) {   /* pair 3: d^5_{55} = cos^10(beta/2) */
        const double c = (double)cosl((ld)beta[j] / 2);
        diag = diag && fabs(d[(size_t)3 * (L + 1) * NR + 5 * NR + j] - pow(c, 10)) < 1e-15;
    }
    check(one, "d^l_{00}(0) = 1");
    check(diag, "d^l_{ll} = cos^{2l}(beta/2)");
    const int far_mb[1] = {0}, far_ms[1] = {L + 1};
    check(oracle_wigner_d(L, 1, far_mb, far_ms, NR, x, d, NULL, NULL, 1) != 0, "a pair beyond lmax is refused");

    unsigned seed = 1002u;
    const int nalm = (L + 1) * (L + 2) / 2;
    double* alm = malloc(sizeof(double) * 2 * nalm);
    double* blm = malloc(sizeof(double) * 2 * (2 * M + 1) * (L + 1));
    for (int i = 0; i < 2 * nalm; ++i) alm[i] = urand(&seed);
    for (int i = 0; i < 2 * (2 * M + 1) * (L + 1); ++i) blm[i] = urand(&seed);
    const int ncol = (2 * M + 1) * (L + 1);
    int* cmb = malloc(sizeof(int) * ncol);
    int* cms = malloc(sizeof(int) * ncol);
    for (int mb = -M, i = 0; mb <= M; ++mb)
        for (int ms = 0; ms <= L; ++ms, ++i) { cmb[i] = mb; cms[i] = ms; }
    int sel[NR];
    for (int j = 0; j < NR; ++j) sel[j] = j;
    double* C = malloc(sizeof(double) * 2 * ncol * NR);
    check(oracle_totalconv_fwd(L, M, NR, x, alm, blm, ncol, cmb, cms, NR, sel, 0.0, C, 1) == 0, "totalconv_fwd runs");
    int finite = 1;
    for (int i = 0; i < 2 * ncol * NR; ++i) finite = finite && isfinite(C[i]);
    check(finite, "forward output finite");

    /* u of one column against the sum over rings of d^l G */
    const int col_mb[1] = {-2}, col_ms[1] = {7};
    double G[2 * NR];
    for (int j = 0; j < 2 * NR; ++j) G[j] = urand(&seed);
    ld u[2 * (L + 1)];
    check(oracle_totalconv_u(L, M, NR, x, G, 1, col_mb, col_ms, u, 1) == 0, "totalconv_u runs");
    check(oracle_wigner_d(L, 1, col_mb, col_ms, NR, x, d, NULL, NULL, 1) == 0, "wigner_d of the column");
    int agree = 1;
    for (int l = 0; l <= L; ++l) {
        ld re = 0, im = 0;
        for (int j = 0; j < NR; ++j) {
            re += (ld)d[(size_t)l * NR + j] * G[2 * j];
            im += (ld)d[(size_t)l * NR + j] * G[2 * j + 1];
        }
        agree = agree && fabsl(u[2 * l] - re) < 1e-14L && fabsl(u[2 * l + 1] - im) < 1e-14L;
    }
    check(agree, "u equals the ring sum of d^l G");

    const int pr[3] = {0, 4, 8}, pa[3] = {0, 1, 5}, pg[3] = {0, 7, 3};
    double cube[3];
    check(oracle_datacube(L, M, NR, C, 6, 2 * L + 1, 3, pr, pa, pg, cube, 1) == 0 && isfinite(cube[1]),
          "datacube runs");
    const int far_a[1] = {6};
    check(oracle_datacube(L, M, NR, C, 6, 2 * L + 1, 1, pr, far_a, pg, cube, 1) != 0, "alpha index beyond nalpha");

    free(d); free(mant); free(ex); free(alm); free(blm); free(cmb); free(cms); free(C);
    if (failed) return 1;
    printf("ok\n");
    return 0;
}
