/*
 * totalconv.h -- C ABI of libtotalconv, the MI355X (gfx950) implementation of
 * the reduced-Wigner l-recursion and the total-convolution coefficients of
 * Prezeau & Reinecke, "Algorithm for the evaluation of reduced Wigner
 * matrices" (arXiv:1002.1050).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - d^l_{m m'}(beta) = <l m| exp(-i beta J_y) |l m'>  (Sec. 2, eq. reducedwignerdef).
 * - Rings.  The problem is stated on colatitudes beta_j in [0, pi] (Sec. 4.1, the
 *   beta grid of eqs. conviqt and convdef).  The library turns them into the ring
 *   cosines it computes on, once per call (tc_rings_from_beta): x_j = cos(beta_j)
 *   evaluated in long double and rounded once to double (the per-ring cos(beta) that
 *   Sec. 4.2.2 precomputes; the poles are allowed), and for each j < k = nring-1-j
 *   whose colatitudes add up to pi within 2^-48 (a grid symmetric about the equator,
 *   rounded to doubles) the ring with the larger colatitude gets exactly -x of the
 *   other.  Rings j and nring-1-j with x[nring-1-j] == -x[j] form a mirror pair
 *   (beta, pi - beta) and share one recursion (Sec. 4.2.3, appendix eq.
 *   pithetasym); any other ring is computed on its own.  Every entry point that
 *   takes rings has a twin with the suffix _x that takes the cosines x directly
 *   (doubles in [-1, 1]; same pairing rule on x).
 * - Complex arrays are interleaved FP64 pairs (re, im), 16-byte aligned.
 * - Sky ("alm"): s_{l,m} for 0 <= m <= l <= lmax, packed m-major,
 *   index(l, m) = m*(2*lmax+1-m)/2 + l; s_{l,-m} = (-1)^m conj(s_{l,m}) is implied
 *   (real sky, Sec. 4.2.3 eq. blmslmsym).
 * - Beam ("blm"): [2*mbmax+1][lmax+1], row mb+mbmax holds b_{l,mb}; entries with
 *   l < |mb| are ignored.
 * - Coefficients ("C"): [2*mbmax+1][lmax+1][nring], element (mb, msky, j) holds
 *   C_{mb,msky}(beta_j) for mb in [-mbmax, mbmax] and msky in [0, lmax]; the
 *   columns with msky < 0 follow from C_{-mb,-msky} = conj(C_{mb,msky})
 *   (Sec. 4.2.3) and are not stored.
 *
 * Memory, streams, errors
 * -----------------------
 * - Pointers marked (host) are host memory; every other pointer is device memory
 *   of the current HIP device.  The caller owns all memory; the library never
 *   frees a caller buffer.
 * - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL for the
 *   default stream) and the call returns without waiting for it.  The small
 *   host-computed tables (rings, column list, seed normalisations) are copied into
 *   the workspace on that stream; the library keeps their host images for the
 *   calls of recent shapes and ring sets (at most 64, 1 GiB in all) in pinned
 *   memory it allocates and frees itself, so that a repeated call only enqueues
 *   that copy.  Buffers must stay valid until the stream has passed the call.
 * - Return value 0 on success, otherwise one of the negative TC_E* codes;
 *   tc_last_error() returns a message for the calling thread's last failure.
 *   Invalid arguments are rejected before any GPU work is enqueued.
 * - Results are deterministic: no floating-point atomics; the order of every
 *   sum is fixed by the tile configuration.
 */
#ifndef TOTALCONV_H
#define TOTALCONV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC_OK 0
#define TC_EINVAL (-1)        /* invalid argument                         */
#define TC_EHIP (-2)          /* a HIP runtime call failed                */
#define TC_ENOMEM (-3)        /* workspace too small or allocation failed */
#define TC_EUNSUPPORTED (-4)  /* valid request the library cannot serve   */

#define TC_OP_WIGNER 0
#define TC_OP_FWD 1
#define TC_OP_ADJ 2
#define TC_OP_FWD_POL 3       /* tiles / workspace of totalconv_fwd_pol */
#define TC_OP_CUBE 4          /* timing of totalconv_datacube */
#define TC_OP_MATRIX 5        /* tiles / timing of wigner_d_matrix */

#define TC_POL_SEPARATE 0     /* polarised: one output per (sky, beam) pair */
#define TC_POL_SUM 1          /* polarised: one output, the sum over the pairs */

#define TC_LMAX_LIMIT 16384

/* Message for the calling thread's most recent failure ("" if none). */
const char* tc_last_error(void);

/* ABI revision of this header. */
int tc_abi_version(void);

/*
 * Device workspace, in bytes, that an entry point needs.
 *   op = TC_OP_WIGNER: `mbmax` is the number of (mb, msky) pairs;
 *   op = TC_OP_FWD / TC_OP_ADJ / TC_OP_FWD_POL: the arguments of totalconv_fwd /
 *   totalconv_adj (and totalconv_adj_pol) / totalconv_fwd_pol.
 * Returns 0 for invalid arguments.
 */
size_t totalconv_workspace_bytes(int op, int lmax, int mbmax, int nring);

/*
 * As totalconv_workspace_bytes, for the given ring set (host, nring colatitudes;
 * _x: nring cosines): exact when the rings form mirror pairs, which need fewer
 * ring slots than the worst case assumed above.  Returns 0 for invalid arguments.
 */
size_t totalconv_workspace_bytes_rings(int op, int lmax, int mbmax, int nring, const double* beta);
size_t totalconv_workspace_bytes_rings_x(int op, int lmax, int mbmax, int nring, const double* cosbeta);

/*
 * The ring cosines the library computes on for the colatitudes beta (host, nring
 * doubles in [0, pi]): cosbeta[j] = cos(beta_j) in long double rounded once, with
 * the mirror rule of the conventions above.  cosbeta: host output, nring doubles.
 * TC_EINVAL for nring < 1, a NULL pointer or a colatitude outside [0, pi] (NaN
 * included); nothing is written then.  Host only: touches no device.
 */
int tc_rings_from_beta(int nring, const double* beta, double* cosbeta);

/*
 * Reduced Wigner elements by the l-recursion of Sec. 3.2 (seeds eqs. ini1..ini2
 * at l0 = max(|mb|,|msky|) evaluated as logarithms, eq. logstart; the recursion
 * eq. lrec in the F0/F1/F2 form of Sec. 4.2.2; exact power-of-two scaling while
 * values are below 2^-900).
 *   lmax         0 <= lmax <= TC_LMAX_LIMIT
 *   npair        number of (mb, msky) pairs, >= 1
 *   mb, msky     (host) npair integers each, |mb|, |msky| <= lmax
 *   nring        number of rings, >= 1
 *   beta         (host) nring colatitudes in [0, pi] (_x: cosbeta, nring cosines in [-1, 1])
 *   d            out: [npair][lmax+1][nring] doubles, d[i][l][j] = d^l_{mb[i],msky[i]}(beta_j),
 *                0 for l < l0; values below the double range come out as 0 or subnormal
 *   workspace    at least totalconv_workspace_bytes(TC_OP_WIGNER, lmax, npair, nring) bytes
 */
int wigner_d_rings(int lmax, int npair, const int* mb, const int* msky,
                   int nring, const double* beta, double* d,
                   void* workspace, size_t ws_bytes, void* stream);
int wigner_d_rings_x(int lmax, int npair, const int* mb, const int* msky,
                     int nring, const double* cosbeta, double* d,
                     void* workspace, size_t ws_bytes, void* stream);

/*
 * The full reduced Wigner matrix at one l (Sec. 3.1): d^l_{m m'}(beta_j) for
 * -l <= m, m' <= l, without the elements of any other l.  Each row of fixed m is
 * walked in m' with the three-term relation of Sec. 2 (eq. mrec), downwards from
 * its closed-form end point d^l_{m,l} (Sec. 3.2 seed, as a logarithm, with exact
 * power-of-two scaling), over 0 <= m <= m' <= l at beta and at pi - beta; the
 * other elements follow from the symmetries of the appendix.  This is the
 * recursion that the ratio form of Sec. 3.1 writes as ratios of neighbours.
 *   l            0 <= l <= TC_LMAX_LIMIT
 *   nring >= 1;  beta (host) nring colatitudes in [0, pi] (the poles included; _x: cosines)
 *   d            out: [nring][2l+1][2l+1] doubles, d[j][m+l][m'+l] = d^l_{m m'}(beta_j);
 *                values below the double range come out as 0 or subnormal
 *   workspace    at least wigner_d_matrix_workspace_bytes(l, nring) bytes
 * tc_set_tile(TC_OP_MATRIX, R) picks R in {1, 2} rows per lane (0: built-in).
 */
size_t wigner_d_matrix_workspace_bytes(int l, int nring);
int wigner_d_matrix(int l, int nring, const double* beta, double* d,
                    void* workspace, size_t ws_bytes, void* stream);
int wigner_d_matrix_x(int l, int nring, const double* cosbeta, double* d,
                      void* workspace, size_t ws_bytes, void* stream);

/*
 * Total-convolution coefficients (Sec. 4.1, eq. convdef):
 *   C_{mb,msky}(beta_j) = sum_{l=l0}^{lmax} conj(b_{l,mb}) d^l_{mb,msky}(beta_j) s_{l,msky}.
 * Terms whose |d| stays below 2^-100 (about the paper's 1e-30) before the first
 * crossing of that threshold within a group of rings (the 64*R consecutive ring
 * slots, mirror pairs or single rings, that one wavefront walks; R is the tile's
 * chains per lane) may be left out of the sum (Sec. 4.2.1); the recursion itself
 * always runs over every l.  The same holds for totalconv_adj.  A ring and
 * its mirror ring pi - beta share one recursion (Sec. 4.2.3); on columns whose beam rows
 * mb and -mb are equal up to a sign for every l >= |mb| (read on the device each call),
 * the two rings' sums are formed from the sums over even and over odd l, which changes
 * only the rounding.
 *   lmax, mbmax  0 <= mbmax <= lmax <= TC_LMAX_LIMIT
 *   nring        >= 1;  beta (host) nring colatitudes in [0, pi] (_x: cosbeta, cosines in [-1, 1])
 *   alm          sky, (lmax+1)(lmax+2)/2 complex
 *   blm          beam, (2*mbmax+1)*(lmax+1) complex
 *   C            out: (2*mbmax+1)*(lmax+1)*nring complex
 *   workspace    at least totalconv_workspace_bytes(TC_OP_FWD, lmax, mbmax, nring) bytes
 */
int totalconv_fwd(int lmax, int mbmax, int nring, const double* beta,
                  const double* alm, const double* blm, double* C,
                  void* workspace, size_t ws_bytes, void* stream);
int totalconv_fwd_x(int lmax, int mbmax, int nring, const double* cosbeta,
                    const double* alm, const double* blm, double* C,
                    void* workspace, size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): totalconv_fwd without a
 * workspace argument.  Its tables (ring tables, column list, seed normalisations,
 * beam-row signs) live in a static device array of the library, one per GPU,
 * TC_NOALLOC_SCRATCH_BYTES (8 MiB) long and held until the process ends: enough for
 * lmax 4096 with mbmax 14 on 8192 rings, or lmax 8192 with mbmax 16 on 16384 rings.
 * Allocates no device or pinned memory (no hipMalloc, hipFree or hipHostMalloc): the
 * tables are built on the host and copied on `stream` from pageable memory.  All
 * calls on one GPU share its array and the last call's contents stay in it; calls
 * that overlap on one GPU (several streams or threads) race and must be serialised.
 * TC_ENOMEM when the tables would exceed the array; otherwise the arguments, checks
 * and results of totalconv_fwd, whose kernels it runs (equal bit for bit).
 */
#define TC_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
int totalconv_fwd_noalloc(int lmax, int mbmax, int nring, const double* beta,
                          const double* alm, const double* blm, double* C, void* stream);

/*
 * Adjoint of totalconv_fwd (not in the paper; the exact transpose of eq. convdef).
 * With Cbar = dL/dconj(C) (the layout of C; PyTorch's gradient convention),
 *   alm_bar_{l,msky} = sum_{mb,j} b_{l,mb} d^l_{mb,msky}(beta_j) Cbar_{mb,msky,j}
 *   blm_bar_{l,mb}   = sum_{msky,j} s_{l,msky} d^l_{mb,msky}(beta_j) conj(Cbar_{mb,msky,j})
 * d is recomputed on the fly.  alm_bar (layout of alm) and blm_bar (layout of blm)
 * may each be NULL; blm_bar entries with l < |mb| are written as 0.
 *   workspace    at least totalconv_workspace_bytes(TC_OP_ADJ, lmax, mbmax, nring) bytes
 */
int totalconv_adj(int lmax, int mbmax, int nring, const double* beta,
                  const double* alm, const double* blm, const double* Cbar,
                  double* alm_bar, double* blm_bar,
                  void* workspace, size_t ws_bytes, void* stream);
int totalconv_adj_x(int lmax, int mbmax, int nring, const double* cosbeta,
                    const double* alm, const double* blm, const double* Cbar,
                    double* alm_bar, double* blm_bar,
                    void* workspace, size_t ws_bytes, void* stream);

/*
 * Polarised total convolution (footnote of Sec. 4.1: eq. convdef evaluated for
 * the additional gradient and curl pairs (b^G, s^G), (b^C, s^C) beside the
 * temperature pair).  The npair (1..3) pairs share one recursion.
 *   alm, blm     (host) arrays of npair device pointers, each laid out as in
 *                totalconv_fwd (pair p: s^p and b^p)
 *   mode         TC_POL_SEPARATE: C[p] = C^p, the convolution of pair p
 *                (npair outputs);
 *                TC_POL_SUM: C[0] = sum_p C^p, the polarised detector's
 *                coefficients (one output)
 *   C            (host) array of device pointers to the outputs, each laid out
 *                as C of totalconv_fwd
 *   workspace    at least totalconv_workspace_bytes(TC_OP_FWD_POL, lmax, mbmax, nring) bytes
 * Each output equals, up to rounding order, the sum of totalconv_fwd over the
 * pairs it covers.  TC_EINVAL for npair outside [1, 3], an unknown mode or a
 * NULL pointer among the used entries.
 */
int totalconv_fwd_pol(int lmax, int mbmax, int nring, const double* beta, int npair,
                      const double* const* alm, const double* const* blm, int mode,
                      double* const* C, void* workspace, size_t ws_bytes, void* stream);
int totalconv_fwd_pol_x(int lmax, int mbmax, int nring, const double* cosbeta, int npair,
                        const double* const* alm, const double* const* blm, int mode,
                        double* const* C, void* workspace, size_t ws_bytes, void* stream);

/*
 * Adjoint of totalconv_fwd_pol.  Cbar: (host) array of device pointers to the
 * cotangents of the outputs (npair for TC_POL_SEPARATE, 1 for TC_POL_SUM).
 * alm_bar, blm_bar: (host) arrays of npair device pointers (entries may be
 * NULL; either array may be NULL) receiving the gradients of pair p, as
 * totalconv_adj gives them for that pair's sky, beam and cotangent.  In
 * TC_POL_SUM mode the pairs share one reduction over the rings and one launch
 * forms every pair's sky gradient from it (each equal, bit for bit, to what
 * totalconv_adj returns for that pair and the one cotangent); in
 * TC_POL_SEPARATE mode the cotangents are reduced one after the other.
 *   workspace    at least totalconv_workspace_bytes(TC_OP_ADJ, lmax, mbmax, nring) bytes
 */
int totalconv_adj_pol(int lmax, int mbmax, int nring, const double* beta, int npair,
                      const double* const* alm, const double* const* blm, int mode,
                      const double* const* Cbar, double* const* alm_bar, double* const* blm_bar,
                      void* workspace, size_t ws_bytes, void* stream);
int totalconv_adj_pol_x(int lmax, int mbmax, int nring, const double* cosbeta, int npair,
                        const double* const* alm, const double* const* blm, int mode,
                        const double* const* Cbar, double* const* alm_bar, double* const* blm_bar,
                        void* workspace, size_t ws_bytes, void* stream);

/*
 * Data cube (Sec. 4.1, eq. conviqt): from the coefficients C of totalconv_fwd,
 *   cube[j][a][g] = c(alpha_a, beta_j, gamma_g)
 *                 = sum_{mb=-mbmax}^{mbmax} sum_{msky=-lmax}^{lmax}
 *                   e^{-i mb alpha_a} e^{-i msky gamma_g} C_{mb,msky}(beta_j),
 *   alpha_a = 2 pi a / nalpha (a < nalpha), gamma_g = 2 pi g / ngamma (g < ngamma),
 * with the msky < 0 columns taken from C_{-mb,-msky} = conj(C_{mb,msky}) (real
 * sky and beam, Sec. 4.2.3).  c is then real; the imaginary part that rounding
 * (or a beam that is not real) leaves in the msky = 0 term is dropped.  The sum
 * over mb is done directly, the one over msky by an FFT of length ngamma.
 *   lmax, mbmax  0 <= mbmax <= lmax <= 8192
 *   nring        >= 1; C as written by totalconv_fwd (device)
 *   nalpha       >= 1, nalpha * (2*mbmax+1) <= 4096
 *   ngamma       a power of two in [max(2, 2*lmax), 16384] (at 2*lmax the two
 *                terms msky = +-lmax meet in one frequency, as the definition
 *                evaluated on that grid requires)
 *   cube         out: [nring][nalpha][ngamma] doubles, 16-byte aligned
 *   workspace    at least totalconv_datacube_workspace_bytes(...) bytes: the
 *                phase and twiddle tables and the alpha sums of two ring chunks
 *                (rings are processed in chunks of about 768 MB of alpha sums, the
 *                sums over mb of one chunk formed while the FFTs of the chunk
 *                before run on a second stream of the library)
 * TC_EUNSUPPORTED if the device allows less LDS per workgroup than the FFT of
 * length ngamma needs (8.5 * ngamma + 16 bytes).
 * totalconv_datacube_ring_chunk returns the rings per chunk (0 for bad sizes).
 */
size_t totalconv_datacube_workspace_bytes(int lmax, int mbmax, int nring, int nalpha, int ngamma);
int totalconv_datacube_ring_chunk(int lmax, int mbmax, int nring, int nalpha, int ngamma);
int totalconv_datacube(int lmax, int mbmax, int nring, const double* C, int nalpha, int ngamma,
                       double* cube, void* workspace, size_t ws_bytes, void* stream);

/*
 * Tile selection for later calls in this process (not in the paper; a tuning
 * knob of this implementation).  Each lane walks R chains; a workgroup covers
 * 256*R ring slots of one column.  op = TC_OP_FWD or TC_OP_ADJ (R in {2, 4, 8}),
 * TC_OP_FWD_POL (R in {2, 4}), TC_OP_WIGNER (R in {1, 4}) or TC_OP_MATRIX (R in
 * {1, 2}: one-wave workgroups with R rows per lane in place of the built-in two-wave
 * workgroups with one row per lane); for TC_OP_CUBE, R > 0 sets the rings the data cube processes per chunk
 * (and so its workspace).  R = 0 restores the built-in choice.  Affects
 * the workspace sizes reported afterwards.  Returns TC_EINVAL for other values.
 * Not synchronised: set it from the thread that issues the calls.
 */
int tc_set_tile(int op, int R);

/*
 * Full tile selection: R chains per lane, TB values of l per LDS coefficient
 * block (32 or 64) and TR (4, the only built value; kept so that tiles stay
 * (R, TB, TR) triples).  0 keeps the built-in value of a parameter.  Same
 * scope and rules as tc_set_tile; TC_EINVAL for combinations that are not built.
 */
int tc_set_tile_ex(int op, int R, int TB, int TR);

/* The R that the next call of `op` at this lmax would use. */
int tc_get_tile(int op, int lmax);

/* The full tile (R, TB, TR) that the next call of `op` at this lmax would use. */
int tc_get_tile_ex(int op, int lmax, int* R, int* TB, int* TR);

/*
 * Batched plan: many detectors -- each with its own beam, mbmax, lmax and ring
 * set -- convolved with one shared sky, all captured in one HIP graph (the
 * batching is not in the paper).  Detectors with the same lmax and the same ring
 * cosines share walks of the recursion (largest mbmax first, as the polarised
 * pairs of Sec. 4.1's footnote share theirs): in the forward up to four per walk
 * (two at R 8), one even / odd walk feeding every member's output; in the
 * adjoint two per walk at TB 32 and R <= 4 (at R 8 the second detector's
 * cotangents do not fit the registers), one walk adding into both detectors'
 * sums.  One workgroup per work item (walk, column, ring tile), the items
 * longest first.  Forward: one launch per chains-per-lane R, the launches of
 * different R on parallel graph branches.  Adjoint: one launch per (R, lmax)
 * group, the groups one after the other; after each, a second stream runs its
 * detectors' beam gradients and adds their sky gradients to alm_bar (always in
 * the same order) beside the next group's walks.  Every beam gradient and forward
 * output equals what totalconv_fwd / totalconv_adj computes for that detector at
 * the tile the plan walks it with, bit for bit.
 */
typedef struct tc_detector {
    int lmax;                /* 0 <= mbmax <= lmax <= lmax_sky                     */
    int mbmax;
    int nring;
    const double* beta;      /* (host) nring colatitudes in [0, pi], or NULL:      */
    const double* cosbeta;   /* (host) nring ring cosines, used when beta is NULL;  */
                             /* either is read at plan creation only                */
    const double* blm;       /* beam [2*mbmax+1][lmax+1] complex                    */
    double* C;               /* forward: out [2*mbmax+1][lmax+1][nring] complex     */
    const double* Cbar;      /* adjoint: in, layout of C                            */
    double* blm_bar;         /* adjoint: out, layout of blm, may be NULL            */
} tc_detector;

/*
 * Build a plan for op = TC_OP_FWD or TC_OP_ADJ over ndet >= 1 detectors and the
 * sky alm (packed at lmax_sky).  For the adjoint, alm_bar (layout of alm, may
 * be NULL) receives the sky gradient summed over all detectors.  The plan keeps
 * the device pointers it is given (they must stay valid while it is used) and
 * owns its tables and partial-sum buffers (device memory allocated here and
 * released by tc_plan_destroy).  Creation is synchronous on `stream`.  The
 * pointed-to data may change between executions: each execution reads the
 * beams, sky and cotangents afresh (including, for the forward, which beam rows
 * are equal up to a sign, as totalconv_fwd does).  A detector is walked with the
 * largest R not above the plan's (tc_plan_tile) whose 256 R ring slots its rings
 * still fill more than half of (R halved while 128 R >= its slots).
 */
int tc_plan_create(void** plan, int op, int ndet, const tc_detector* dets, int lmax_sky,
                   const double* alm, double* alm_bar, void* stream);

/* Enqueue the plan's graph on `stream` (asynchronous). */
int tc_plan_execute(void* plan, void* stream);

/* Device bytes the plan owns, and its largest R (the R of op's current tile). */
size_t tc_plan_device_bytes(void* plan);
int tc_plan_tile(void* plan);

/* Release the plan (synchronises with its last launch first).  NULL is ignored. */
int tc_plan_destroy(void* plan);

/*
 * Kernel timing (diagnostics, not in the paper).  tc_timing_enable(n), n >= 1,
 * creates n pairs of HIP timing events per operation on the current device;
 * from then on every wigner_d_rings / totalconv_fwd / totalconv_adj /
 * totalconv_fwd_pol call records one pair (under op TC_OP_WIGNER, TC_OP_FWD,
 * TC_OP_ADJ, TC_OP_FWD_POL) on its own stream, directly before and after its
 * recursion kernel; totalconv_datacube records one TC_OP_CUBE pair around all
 * of its kernels (both streams), wigner_d_matrix one TC_OP_MATRIX pair (for the adjoint: without the two short epilogue kernels
 * that finish the gradients; totalconv_adj_pol records one TC_OP_ADJ pair per
 * cotangent), reusing the pairs cyclically.  n = 0 releases the events and
 * stops the recording.  Calls must then run on streams of that device.
 * Returns TC_OK, TC_EINVAL for n < 0 or n > 65536, TC_EHIP if event creation
 * fails.  Not thread-safe: enable, read and the timed calls belong to one thread.
 */
int tc_timing_enable(int n);

/*
 * Waits for the pairs of the last k = min(n, recorded, capacity) calls of `op`
 * and writes their kernel durations in milliseconds to ms[0..k-1] (host),
 * oldest first.  Returns k (0 if timing is off or nothing was recorded), or a
 * negative TC_E* code.
 */
int tc_timing_read(int op, float* ms, int n);

#ifdef __cplusplus
}
#endif

#endif /* TOTALCONV_H */
