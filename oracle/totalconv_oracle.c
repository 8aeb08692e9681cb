/*
 * CPU oracle for reduced Wigner elements and the total-convolution sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline timing of the benchmark load this file's library; the product
 * path never does, and it shares no code, header, table or helper with the
 * HIP library.  It is plain, slow and meant to be checked by eye against
 * Prezeau & Reinecke, "Algorithm for the evaluation of reduced Wigner
 * matrices" (arXiv:1002.1050):
 *
 *   d^l_{m m'}(beta)   reduced Wigner element, convention <l m|exp(-i beta J_y)|l m'>
 *                      (Sec. 2, eq. reducedwignerdef).
 *   l-recursion        Sec. 2 eq. lrec, written with the coefficients
 *                      F0, F1, F2 of Sec. 4.2.2 (from their closed forms).
 *   seeds              Sec. 3.2 eqs. ini1..ini2 at l0 = max(|m|,|m'|),
 *                      evaluated as a logarithm (eq. logstart) in long double.
 *   scaled values      Sec. 3.2: a value is kept as a significand times an
 *                      integer power of two, so that seeds far below the
 *                      long double range stay exact.
 *   convolution        Sec. 4.1 eq. convdef:
 *                      C_{mb,msky}(beta) = sum_l conj(b_{l,mb}) d^l_{mb,msky}(beta) s_{l,msky}.
 *   data cube          Sec. 4.1 eq. conviqt: the double sum over mb and msky of
 *                      e^{-i mb alpha} e^{-i msky gamma} C_{mb,msky}(beta), term by term.
 *
 * Readings of the paper taken here (the paper is silent or garbled there):
 *   - Seed rows (printed rows 2-4 all read d^l_{-l,m}):
 *       d^l_{l,m}  = A c^{l+m} (-s)^{l-m}      d^l_{-l,m} = A c^{l-m} s^{l+m}
 *       d^l_{m,l}  = A c^{l+m} s^{l-m}         d^l_{m,-l} = A c^{l-m} (-s)^{l+m}
 *     with c = cos(beta/2), s = sin(beta/2), A = sqrt((2l)!/((l+m)!(l-m)!)).
 *   - F1 and F2 at l = 0 are set to 0 (the printed forms divide by zero; only
 *     the (0,0) chain reaches l = 0 and there d^{-1} = 0).
 *   - A ring is given by x = cos(beta) as a double (the per-ring cos(beta) the
 *     paper precomputes, Sec. 4.2.2); c = cos(beta/2) and s = sin(beta/2) are
 *     derived from that x in long double.
 *   - A power that is zero contributes a factor 1 even when its base is zero;
 *     a zero base with a positive power makes the whole chain zero (Sec. 3.2,
 *     the -infinity case).
 *   - Sky coefficients are stored for m >= 0; s_{l,-m} = (-1)^m conj(s_{l,m})
 *     (Sec. 4.2.3, eq. blmslmsym).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double ld;

/* ------------------------------------------------------------------ rings */

typedef struct {
    ld x;        /* cos(beta) rounded to double, then widened */
    ld lc, ls;   /* ln cos(beta/2), ln sin(beta/2) (may be -inf) */
    int c_zero, s_zero;
} ring_t;

static void ring_setup(double xd, ring_t* r)
{
    ld x = (ld)xd;
    ld c = sqrtl((1.0L + x) / 2.0L);
    ld s = sqrtl((1.0L - x) / 2.0L);
    r->x = x;
    r->c_zero = (c == 0.0L);
    r->s_zero = (s == 0.0L);
    r->lc = r->c_zero ? -INFINITY : logl(c);
    r->ls = r->s_zero ? -INFINITY : logl(s);
}

/* ------------------------------------------------------------------ seeds */

/* Seed d^{l0}_{mb,ms}(beta), l0 = max(|mb|,|ms|), as mant * 2^ex.
 * Returns 0 if the chain is identically zero. */
static int seed_value(int mb, int ms, const ring_t* r, ld* mant, long long* ex)
{
    int amb = abs(mb), ams = abs(ms);
    int l0 = amb > ams ? amb : ams;
    int m, p, q, neg;   /* d = A c^p (sign s)^q */
    if (ams >= amb) {
        m = mb;
        if (ms >= 0) { p = l0 + mb; q = l0 - mb; neg = 0; }        /* d^l_{m,l}  */
        else         { p = l0 - mb; q = l0 + mb; neg = q & 1; }    /* d^l_{m,-l} */
    } else {
        m = ms;
        if (mb > 0)  { p = l0 + ms; q = l0 - ms; neg = q & 1; }    /* d^l_{l,m}  */
        else         { p = l0 - ms; q = l0 + ms; neg = 0; }        /* d^l_{-l,m} */
    }
    if ((p > 0 && r->c_zero) || (q > 0 && r->s_zero)) {
        *mant = 0.0L; *ex = 0;
        return 0;
    }
    /* ln|d| = (ln (2l0)! - ln (l0+m)! - ln (l0-m)!)/2 + p ln c + q ln s   (eq. logstart) */
    ld lnd = 0.5L * (lgammal((ld)(2 * l0 + 1)) - lgammal((ld)(l0 + m + 1)) - lgammal((ld)(l0 - m + 1)));
    if (p > 0) lnd += (ld)p * r->lc;
    if (q > 0) lnd += (ld)q * r->ls;
    ld k = floorl(lnd / logl(2.0L));
    ld frac = lnd - k * logl(2.0L);
    *mant = expl(frac);
    if (neg) *mant = -*mant;
    *ex = (long long)k;
    return 1;
}

/* ----------------------------------------------------- recursion tables */

/* F0, F1, F2 of Sec. 4.2.2 from their closed forms, for l in [l0, lmax-1]:
 *   d^{l+1} = F0_l (x - F1_l) d^l - F2_l d^{l-1}.                       */
static void coef_tables(int mb, int ms, int lmax, ld* F0, ld* F1, ld* F2)
{
    int amb = abs(mb), ams = abs(ms);
    int l0 = amb > ams ? amb : ams;
    ld b2 = (ld)mb * mb, s2 = (ld)ms * ms;
    for (int l = l0; l < lmax; ++l) {
        ld L = (ld)l, L1 = (ld)(l + 1);
        ld up = (L1 * L1 - b2) * (L1 * L1 - s2);
        F0[l] = L1 * (2.0L * L + 1.0L) / sqrtl(up);
        if (l == 0) {
            F1[l] = 0.0L;
            F2[l] = 0.0L;
        } else {
            F1[l] = (ld)mb * (ld)ms / (L * L1);
            F2[l] = (L1 / L) * sqrtl((L * L - b2) * (L * L - s2) / up);
        }
    }
}

static long long clampll(long long v, long long lo, long long hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Value of mant * 2^ex as a long double (underflows to zero far below range). */
static ld scaled_to_ld(ld mant, long long ex)
{
    return ldexpl(mant, (int)clampll(ex, -40000, 40000));
}

/* Walk one chain from l0 to lmax.  visit(l, mant, ex, ctx) sees d^l = mant * 2^ex.
 * Renormalises by an exact power of two whenever |mant| leaves [2^-64, 2^64]. */
typedef void (*visit_fn)(int l, ld mant, long long ex, void* ctx);

static void walk_chain(int mb, int ms, int lmax, const ring_t* r,
                       const ld* F0, const ld* F1, const ld* F2,
                       visit_fn visit, void* ctx)
{
    int amb = abs(mb), ams = abs(ms);
    int l0 = amb > ams ? amb : ams;
    ld b, a = 0.0L;          /* b = d^l, a = d^{l-1}, both in units of 2^ex */
    long long ex;
    if (!seed_value(mb, ms, r, &b, &ex)) return;   /* identically zero chain */
    const ld big = 18446744073709551616.0L;        /* 2^64 */
    const ld small = 1.0L / big;
    for (int l = l0;; ++l) {
        visit(l, b, ex, ctx);
        if (l == lmax) break;
        ld nb = F0[l] * (r->x - F1[l]) * b - F2[l] * a;
        a = b;
        b = nb;
        ld ab = fabsl(b);
        if (ab != 0.0L && (ab > big || ab < small)) {
            int k;
            frexpl(b, &k);
            b = ldexpl(b, -k);
            a = ldexpl(a, -k);
            ex += k;
        }
    }
}

/* ------------------------------------------------------ d^l outputs */

typedef struct {
    double* out;       /* base of [lmax+1] strided by nring */
    long long stride;
    double* mant;
    long long* exo;
} dvisit_t;

static void visit_store(int l, ld mant, long long ex, void* ctx)
{
    dvisit_t* v = (dvisit_t*)ctx;
    if (v->out) v->out[(long long)l * v->stride] = (double)scaled_to_ld(mant, ex);
    if (v->mant) {
        int k = 0;
        ld f = (mant == 0.0L) ? 0.0L : frexpl(mant, &k);
        v->mant[(long long)l * v->stride] = (double)f;
        v->exo[(long long)l * v->stride] = (mant == 0.0L) ? 0 : ex + k;
    }
}

static int check_pairs(int lmax, int npair, const int* mb, const int* ms)
{
    if (lmax < 0 || npair < 0) return -1;
    for (int i = 0; i < npair; ++i)
        if (abs(mb[i]) > lmax || abs(ms[i]) > lmax) return -1;
    return 0;
}

static void set_threads(int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* d[i][l][j] = d^l_{mb[i],ms[i]}(beta_j), ring j given by xring[j] = cos(beta_j) for l in [0,lmax] (zero for l < l0).
 * If mant/ex are non-null they receive d = mant * 2^ex with mant in [0.5,1). */
int oracle_wigner_d(int lmax, int npair, const int* mb, const int* ms,
                    int nring, const double* xring,
                    double* d, double* mant, long long* ex, int nthreads)
{
    if (check_pairs(lmax, npair, mb, ms) || nring < 0) return -1;
    set_threads(nthreads);
    long long plane = (long long)(lmax + 1) * nring;
    if (d) memset(d, 0, sizeof(double) * plane * npair);
    if (mant) {
        memset(mant, 0, sizeof(double) * plane * npair);
        memset(ex, 0, sizeof(long long) * plane * npair);
    }
    ring_t* rings = (ring_t*)malloc(sizeof(ring_t) * (nring > 0 ? nring : 1));
    for (int j = 0; j < nring; ++j) {
        if (!(xring[j] >= -1.0 && xring[j] <= 1.0)) { free(rings); return -1; }
        ring_setup(xring[j], &rings[j]);
    }
    int err = 0;
#pragma omp parallel
    {
        ld* F = (ld*)malloc(sizeof(ld) * 3 * (lmax + 1));
        if (!F) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < npair; ++i) {
            if (!F) continue;
            ld *F0 = F, *F1 = F + (lmax + 1), *F2 = F + 2 * (lmax + 1);
            coef_tables(mb[i], ms[i], lmax, F0, F1, F2);
            for (int j = 0; j < nring; ++j) {
                dvisit_t v;
                long long base = (long long)i * plane + j;
                v.out = d ? d + base : NULL;
                v.mant = mant ? mant + base : NULL;
                v.exo = ex ? ex + base : NULL;
                v.stride = nring;
                walk_chain(mb[i], ms[i], lmax, &rings[j], F0, F1, F2, visit_store, &v);
            }
        }
        free(F);
    }
    free(rings);
    return err;
}

/* ------------------------------------------------------ convolution */

static void sky_coef(int lmax, const double* alm, int l, int m, ld* re, ld* im)
{
    int am = abs(m);
    long long idx = (long long)am * (2 * lmax + 1 - am) / 2 + l;
    ld r = alm[2 * idx], i = alm[2 * idx + 1];
    if (m < 0) {            /* s_{l,-m} = (-1)^m conj(s_{l,m}) */
        ld sg = (am & 1) ? -1.0L : 1.0L;
        r = sg * r;
        i = -sg * i;
    }
    *re = r;
    *im = i;
}

typedef struct {
    const ld* wre;      /* weight conj(b_{l,mb}) s_{l,msky} per l */
    const ld* wim;
    ld acc_re, acc_im;
    ld eps;             /* accumulate from the first |d| > eps (0: every term) */
    int started;
} cvisit_t;

static void visit_acc(int l, ld mant, long long ex, void* ctx)
{
    cvisit_t* v = (cvisit_t*)ctx;
    ld d = scaled_to_ld(mant, ex);
    if (!v->started) {
        if (fabsl(d) > v->eps || v->eps == 0.0L) v->started = 1;
        else return;
    }
    v->acc_re += v->wre[l] * d;
    v->acc_im += v->wim[l] * d;
}

static int check_conv(int lmax, int mbmax, int nring, int ncol, const int* cmb, const int* cms)
{
    if (lmax < 0 || mbmax < 0 || mbmax > lmax || nring < 1 || ncol < 0) return -1;
    for (int i = 0; i < ncol; ++i)
        if (abs(cmb[i]) > mbmax || abs(cms[i]) > lmax) return -1;
    return 0;
}

/* C[i][k] = C_{cmb[i],cms[i]}(beta_{ring_sel[k]})  (complex, interleaved); rings by x = cos(beta).
 * alm: packed m-major sky (m >= 0); blm: [2*mbmax+1][lmax+1] beam, row mb+mbmax.
 * cms[i] may be negative (the sky's reality relation supplies s_{l,-m}). */
int oracle_totalconv_fwd(int lmax, int mbmax, int nring, const double* xring,
                         const double* alm, const double* blm,
                         int ncol, const int* cmb, const int* cms,
                         int nsel, const int* ring_sel,
                         double eps, double* C, int nthreads)
{
    if (check_conv(lmax, mbmax, nring, ncol, cmb, cms) || nsel < 0) return -1;
    for (int k = 0; k < nsel; ++k)
        if (ring_sel[k] < 0 || ring_sel[k] >= nring) return -1;
    set_threads(nthreads);
    ring_t* rings = (ring_t*)malloc(sizeof(ring_t) * nring);
    for (int j = 0; j < nring; ++j) {
        if (!(xring[j] >= -1.0 && xring[j] <= 1.0)) { free(rings); return -1; }
        ring_setup(xring[j], &rings[j]);
    }
    const int chunk = 64;
    int nchunk = (nsel + chunk - 1) / chunk;
    long long nitem = (long long)ncol * nchunk;
    int err = 0;
#pragma omp parallel
    {
        ld* F = (ld*)malloc(sizeof(ld) * 5 * (lmax + 1));
        if (!F) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (long long it = 0; it < nitem; ++it) {
            if (!F) continue;
            int i = (int)(it / nchunk), c = (int)(it % nchunk);
            int mb = cmb[i], ms = cms[i];
            ld *F0 = F, *F1 = F + (lmax + 1), *F2 = F + 2 * (lmax + 1);
            ld *wre = F + 3 * (lmax + 1), *wim = F + 4 * (lmax + 1);
            coef_tables(mb, ms, lmax, F0, F1, F2);
            const double* brow = blm + 2LL * (mb + mbmax) * (lmax + 1);
            for (int l = 0; l <= lmax; ++l) {
                ld sr, si;
                sky_coef(lmax, alm, l, ms, &sr, &si);
                if (l < abs(ms)) { sr = 0.0L; si = 0.0L; }
                ld br = brow[2 * l], bi = -(ld)brow[2 * l + 1];   /* conj(b) */
                wre[l] = br * sr - bi * si;
                wim[l] = br * si + bi * sr;
            }
            int k1 = c * chunk + chunk;
            if (k1 > nsel) k1 = nsel;
            for (int k = c * chunk; k < k1; ++k) {
                cvisit_t v = { wre, wim, 0.0L, 0.0L, (ld)eps, 0 };
                walk_chain(mb, ms, lmax, &rings[ring_sel[k]], F0, F1, F2, visit_acc, &v);
                C[2 * ((long long)i * nsel + k)] = (double)v.acc_re;
                C[2 * ((long long)i * nsel + k) + 1] = (double)v.acc_im;
            }
        }
        free(F);
    }
    free(rings);
    return err;
}

/* ------------------------------------------------------------- adjoint */

typedef struct {
    ld* ure;    /* [lmax+1] */
    ld* uim;
    ld gre, gim;
} uvisit_t;

static void visit_u(int l, ld mant, long long ex, void* ctx)
{
    uvisit_t* v = (uvisit_t*)ctx;
    ld d = scaled_to_ld(mant, ex);
    v->ure[l] += d * v->gre;
    v->uim[l] += d * v->gim;
}

/* u[i][l] = sum_j d^l_{cmb[i],cms[i]}(beta[j]) * G[i][j]   (all rings j).
 * G: [ncol][nring] complex (the cotangent of C for the listed columns).
 * u: [ncol][lmax+1] complex as pairs of long double.
 * The gradients then follow from u:  sky_bar_{l,msky} = sum_mb b_{l,mb} u_l(mb,msky),
 * beam_bar_{l,mb} = sum_msky s_{l,msky} conj(u_l(mb,msky)). */
int oracle_totalconv_u(int lmax, int mbmax, int nring, const double* xring,
                       const double* G, int ncol, const int* cmb, const int* cms,
                       ld* u, int nthreads)
{
    if (check_conv(lmax, mbmax, nring, ncol, cmb, cms)) return -1;
    set_threads(nthreads);
    ring_t* rings = (ring_t*)malloc(sizeof(ring_t) * nring);
    for (int j = 0; j < nring; ++j) {
        if (!(xring[j] >= -1.0 && xring[j] <= 1.0)) { free(rings); return -1; }
        ring_setup(xring[j], &rings[j]);
    }
    memset(u, 0, sizeof(ld) * 2 * (long long)ncol * (lmax + 1));
    int err = 0;
#pragma omp parallel
    {
        ld* F = (ld*)malloc(sizeof(ld) * 5 * (lmax + 1));
        if (!F) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < ncol; ++i) {
            if (!F) continue;
            ld *F0 = F, *F1 = F + (lmax + 1), *F2 = F + 2 * (lmax + 1);
            ld *ure = F + 3 * (lmax + 1), *uim = F + 4 * (lmax + 1);
            coef_tables(cmb[i], cms[i], lmax, F0, F1, F2);
            for (int l = 0; l <= lmax; ++l) { ure[l] = 0.0L; uim[l] = 0.0L; }
            for (int j = 0; j < nring; ++j) {
                uvisit_t v = { ure, uim, G[2 * ((long long)i * nring + j)], G[2 * ((long long)i * nring + j) + 1] };
                walk_chain(cmb[i], cms[i], lmax, &rings[j], F0, F1, F2, visit_u, &v);
            }
            for (int l = 0; l <= lmax; ++l) {
                u[2 * ((long long)i * (lmax + 1) + l)] = ure[l];
                u[2 * ((long long)i * (lmax + 1) + l) + 1] = uim[l];
            }
        }
        free(F);
    }
    free(rings);
    return err;
}

/* cos(beta) evaluated in long double and rounded once: turns a colatitude into a ring. */
int oracle_ring_x(int nring, const double* beta, double* x)
{
    for (int j = 0; j < nring; ++j) x[j] = (double)cosl((ld)beta[j]);
    return 0;
}

/* The rings of a colatitude grid: oracle_ring_x for each ring, then, for every pair of
 * rings j < k = nring-1-j whose colatitudes add up to pi to within 2^-48 (a grid symmetric
 * about the equator whose colatitudes were rounded to doubles), the ring with the larger
 * colatitude takes exactly minus the other ring's x, so that the pair is an exact mirror
 * pair (beta, pi - beta) of Sec. 4.2.3. */
int oracle_ring_grid_x(int nring, const double* beta, double* x)
{
    const ld pi = 3.14159265358979323846264338327950288L;
    const ld tol = 0x1p-48L;
    oracle_ring_x(nring, beta, x);
    for (int j = 0, k = nring - 1; j < k; ++j, --k) {
        const ld gap = (ld)beta[j] + (ld)beta[k] - pi;
        if (gap >= -tol && gap <= tol) {
            if (beta[k] >= beta[j]) x[k] = -x[j];
            else x[j] = -x[k];
        }
    }
    return 0;
}

int oracle_max_threads(void)
{
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------ data cube
 * Sec. 4.1 eq. conviqt at sampled points, by the definition:
 *   c(alpha_a, beta_j, gamma_g) = sum_{mb=-M}^{M} sum_{msky=-L}^{L}
 *                                 e^{-i mb alpha_a} e^{-i msky gamma_g} C_{mb,msky}(beta_j),
 *   alpha_a = 2 pi a / nalpha, gamma_g = 2 pi g / ngamma,
 * where the columns with msky < 0 are C_{mb,msky} = conj(C_{-mb,-msky}) (real sky
 * and beam, Sec. 4.2.3).  C: [2M+1][L+1][nring] complex (msky >= 0, as the forward
 * writes it).  out[p] = Re c at point (ring[p], ia[p], ig[p]).
 */
static const ld PI_L = 3.14159265358979323846264338327950288L;

int oracle_datacube(int lmax, int mbmax, int nring, const double* C, int nalpha, int ngamma,
                    int npts, const int* ring, const int* ia, const int* ig, double* out, int nthreads)
{
    if (lmax < 0 || mbmax < 0 || mbmax > lmax || nring < 1 || nalpha < 1 || ngamma < 1 || npts < 0)
        return 1;
    for (int p = 0; p < npts; ++p)
        if (ring[p] < 0 || ring[p] >= nring || ia[p] < 0 || ia[p] >= nalpha || ig[p] < 0 || ig[p] >= ngamma)
            return 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < npts; ++p) {
        const int j = ring[p], a = ia[p], g = ig[p];
        ld re = 0.0L;
        for (int mb = -mbmax; mb <= mbmax; ++mb) {
            for (int ms = -lmax; ms <= lmax; ++ms) {
                /* C_{mb,ms}: stored for ms >= 0, else the conjugate of C_{-mb,-ms} */
                const int smb = ms >= 0 ? mb : -mb, sms = ms >= 0 ? ms : -ms;
                const double* z = C + 2 * (((size_t)(smb + mbmax) * (lmax + 1) + sms) * nring + j);
                const ld cr = z[0], ci = ms >= 0 ? z[1] : -z[1];
                /* phase e^{-i theta}, theta = 2 pi (mb a / nalpha + ms g / ngamma), reduced exactly */
                const long long na = (((long long)mb * a) % nalpha + nalpha) % nalpha;
                const long long ng = (((long long)ms * g) % ngamma + ngamma) % ngamma;
                const ld th = 2.0L * PI_L * ((ld)na / (ld)nalpha + (ld)ng / (ld)ngamma);
                /* Re(e^{-i th} (cr + i ci)) = cos(th) cr + sin(th) ci */
                re += cosl(th) * cr + sinl(th) * ci;
            }
        }
        out[p] = (double)re;
    }
    return 0;
}
