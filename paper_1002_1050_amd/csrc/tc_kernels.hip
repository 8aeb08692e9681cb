// gfx950 kernels of libtotalconv: reduced Wigner elements by the l-recursion
// and the total-convolution sum with its adjoint (Prezeau & Reinecke,
// arXiv:1002.1050, Secs. 3.2 and 4).
//
// Mapping.  A workgroup owns one (mb, msky) column and NT*R ring slots of it;
// each lane walks R chains (one per ring slot) up in l, in lock-step, so the
// per-l recursion coefficients and weights are uniform across the workgroup.
// A lane takes R consecutive slots and a wave 64 R (slots run from the pole to
// the equator), so that the chains of a wave share their regime: all still below
// the skip threshold, or not, over the same stretch of l.
// They are built per block of TB values of l in LDS (double-buffered: the next
// block is prepared while the current one is consumed) and read back as
// broadcasts.  A ring slot is either a mirror pair (beta, pi - beta) -- one
// recursion serves both rings through d^l_{-mb,msky}(pi-beta) =
// (-1)^(l-msky) d^l_{mb,msky}(beta) (appendix eq. pithetasym) -- or a single ring.
//
// Numbers.  Everything is FP64.  The seed at l0 = max(|mb|,|msky|) is formed
// as a logarithm in double-double (Sec. 3.2 eq. logstart) and split into a
// significand and a power of two.  While a chain's value is below 2^-900 it is
// carried as d * 2^E with E < 0 and renormalised by exact powers of two every
// RS_STEPS steps; once it reaches 2^-900 it is folded into a plain double (E = 0),
// as Sec. 3.2 prescribes.  The checks are wave-uniform branches, so the inner
// loop has no per-step branches.

#include <hip/hip_runtime.h>

#include "tc_internal.h"

namespace tc {
namespace {

// Tile parameters (template arguments): R chains per lane, NT lanes per workgroup,
// TB values of l per coefficient block; TR is kept in the tile triple (value 4) and no
// longer shapes any kernel: the adjoint's row sums move every step.
constexpr int TS = 8;         // steps between skip checks
constexpr int FOLD_EXP = -900;  // fold scaled values into plain doubles at 2^-900
// A step of the normalised walk (below) multiplies max(|e^l|, |e^{l-1}|) by at most
// alpha F0 |x - F1| + 1 <= 2 (l+1) 2 + 1 < 2^17 for l <= 16384 (F0 <= l+1, |x - F1| <= 2,
// alpha <= 2), which bounds growth inside a TS block.
constexpr int GROWTH_BITS_PER_STEP = 17;
// Scaled chains are rescaled (and folded) only every RS_STEPS steps: a rescaled chain
// keeps max(|e|, |e_prev|) < 1, so its significand stays below 2^(17 RS_STEPS) = 2^544
// until the next rescale, and a chain still scaled after one (true exponent below -900)
// stays below 2^-356 until the next, where the skip test of a chain at 2^-100
// (GROWTH_BITS_PER_STEP * TS bits of headroom) cannot fire.  Between rescales the skip
// test looks at the plain chains only.
constexpr int RS_STEPS = 32;
template <int TB>
constexpr int rs_block() { static_assert(TB % TS == 0 && (TB % RS_STEPS == 0 || RS_STEPS % TB == 0), "tile"); return TB < RS_STEPS ? TB : RS_STEPS; }
constexpr int SKIP_EXP_MAX = -(FOLD_EXP + GROWTH_BITS_PER_STEP * RS_STEPS) - GROWTH_BITS_PER_STEP * TS;  // 220
static_assert(RS_STEPS % TS == 0 && GROWTH_BITS_PER_STEP * RS_STEPS < 1023 && SKIP_EXP_MAX >= 100,
              "rescale period: no overflow of a scaled significand, no missed hot chain at skip 2^-100");

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Loads and stores through a pointer taken from a struct in memory (the batched
// kernels read their arguments from a device array) are marked as global memory, so that
// they compile to global rather than flat instructions, with a scalar base where the
// address is uniform.
template <class T>
__device__ __forceinline__ T ldg(const T* p) { return *(const __attribute__((address_space(1))) T*)p; }
template <class T>
__device__ __forceinline__ void stg(T* p, T v) { *(__attribute__((address_space(1))) T*)p = v; }
// double2 is a class (its copy takes a generic reference): move it as a native vector
typedef double native_double2 __attribute__((ext_vector_type(2)));
template <>
__device__ __forceinline__ double2 ldg(const double2* p)
{
    const native_double2 v = *(const __attribute__((address_space(1))) native_double2*)p;
    return make_double2(v.x, v.y);
}
template <>
__device__ __forceinline__ void stg(double2* p, double2 v)
{
    native_double2 w;
    w.x = v.x;
    w.y = v.y;
    *(__attribute__((address_space(1))) native_double2*)p = w;
}

// Minimum resident waves per SIMD asked of the compiler for R chains per lane
// (bounds the VGPR budget: 512 / waves).
template <int R>
constexpr int min_waves() { return R >= 8 ? 2 : (R >= 4 ? 3 : 4); }

// Polarised forward: NC > 1 outputs carry 4 NC sums per chain, so their budget is one
// step lower than the scalar kernel's; the summed output (NC = 1) keeps the scalar one.
template <int R, int NC, int NP>
constexpr int fwd_min_waves() { return NC == 1 ? min_waves<R>() : (R >= 4 ? 2 : 3); }

// The forward's even / odd form holds 2 complex sums per chain in the same registers but
// needs fewer temporaries: R = 4 fits 4 waves per SIMD (its few spills sit outside the
// step loop), which hides more of each step's broadcast LDS reads.
template <int R>
constexpr int rows_min_waves() { return R >= 8 ? 2 : 4; }

// The adjoint's LDS (about 37 KB per workgroup with TB = 32, 74 KB with TB = 64; mostly
// the emitted row sums of two blocks) caps residency at 4 or 2 workgroups (waves per
// SIMD) per CU.
template <int R, int TB>
constexpr int adj_min_waves() { return min_waves<R>() < (TB >= 64 ? 2 : 4) ? min_waves<R>() : (TB >= 64 ? 2 : 4); }

// ------------------------------------------------------------- double-double
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    e = b - (s - a);
}

// (sh, sl) += n * (ah + al), n an integer held exactly in a double
__device__ __forceinline__ void dd_add_times(double& sh, double& sl, double n, double ah, double al)
{
    const double ph = n * ah;
    const double pl = fma(n, ah, -ph) + n * al;
    double s, e;
    two_sum(sh, ph, s, e);
    e += sl + pl;
    fast_two_sum(s, e, sh, sl);
}

__device__ __forceinline__ void dd_mul(double ah, double al, double bh, double bl, double& yh, double& yl)
{
    const double p = ah * bh;
    const double e = fma(ah, bh, -p) + (ah * bl + al * bh);
    fast_two_sum(p, e, yh, yl);
}

// --------------------------------------------------------------------- seeds
// Seed d^{l0}_{mb,ms} = A c^p (+-s)^q at l0 = max(|mb|,|ms|), c = cos(beta/2),
// s = sin(beta/2) (Sec. 3.2 eqs. ini1..ini2; the printed row labels are read as
// d_{l,m}, d_{-l,m}, d_{m,l}, d_{m,-l}).
struct SeedShape {
    int p, q;
    bool neg;
};

__device__ __forceinline__ SeedShape seed_shape(int mb, int ms)
{
    const int amb = abs(mb), ams = abs(ms);
    const int l0 = max(amb, ams);
    SeedShape s;
    if (ams >= amb) {
        if (ms >= 0) { s.p = l0 + mb; s.q = l0 - mb; s.neg = false; }   // d_{m,l}
        else         { s.p = l0 - mb; s.q = l0 + mb; s.neg = (s.q & 1); }  // d_{m,-l}
    } else {
        if (mb > 0)  { s.p = l0 + ms; s.q = l0 - ms; s.neg = (s.q & 1); }  // d_{l,m}
        else         { s.p = l0 - ms; s.q = l0 + ms; s.neg = false; }   // d_{-l,m}
    }
    return s;
}

// ln|d| = lnA + p ln c + q ln s in double-double, then d = 2^f * 2^k.
// Returns the value in (d, E) form: E = 0 and d plain when |d| >= 2^-900,
// otherwise d in [1, 2) and E = k < 0.  A zero base with a positive power gives
// the zero chain (Sec. 3.2, the -infinity case).
__device__ __forceinline__ void seed_value(double lnAh, double lnAl, SeedShape sh,
                                           double lch, double lcl, double lsh, double lsl,
                                           double& d, int& E)
{
    if ((sh.p > 0 && __builtin_isinf(lch)) || (sh.q > 0 && __builtin_isinf(lsh))) {
        d = 0.0;
        E = 0;
        return;
    }
    double h = lnAh, lo = lnAl;
    if (sh.p > 0) dd_add_times(h, lo, (double)sh.p, lch, lcl);
    if (sh.q > 0) dd_add_times(h, lo, (double)sh.q, lsh, lsl);
    double yh, yl;
    dd_mul(h, lo, 0x1.71547652b82fep+0, 0x1.777d0ffda0d24p-56, yh, yl);   // ln -> log2
    const double k = floor(yh);
    const double f = (yh - k) + yl;
    const double m = exp2(f);
    const int ik = (int)k;
    if (ik >= FOLD_EXP) {
        d = ldexp(m, ik);
        E = 0;
    } else {
        d = m;
        E = ik;
    }
    if (sh.neg) d = -d;
}

// ------------------------------------------------------ recursion coefficients
// d^{l+1} = F0_l (x - F1_l) d^l - F2_l d^{l-1}  (Sec. 4.2.2), evaluated as
// fma(x, A, nB) * d^l - F2 d^{l-1} with A = F0, nB = -F0 F1.  F0 and F2 come from
// their closed forms; at l = lmax (and beyond) the step is switched off.
__device__ __forceinline__ void recursion_coefs(int l, int mb, int ms, int lmax,
                                                double& A, double& nB, double& F2)
{
    if (l >= lmax) {
        A = 0.0; nB = 0.0; F2 = 0.0;
        return;
    }
    const double l1 = (double)(l + 1);
    const double b2 = (double)mb * (double)mb, s2 = (double)ms * (double)ms;
    const double den = sqrt(l1 * l1 - b2) * sqrt(l1 * l1 - s2);
    A = l1 * (2.0 * (double)l + 1.0) / den;
    if (l == 0) {           // F1_0 = F2_0 = 0 (only the (0,0) chain reaches l = 0)
        nB = 0.0;
        F2 = 0.0;
        return;
    }
    const double ll = (double)l;
    const double F1 = ((double)mb * (double)ms) / (ll * l1);
    nB = -(A * F1);
    F2 = (l1 * (sqrt(ll * ll - b2) * sqrt(ll * ll - s2))) / (ll * den);
}

// ------------------------------------------------------------ normalised walk
// The walks carry e^l = c_l d^l with c_{l0} = c_{l0+1} = 1 and c_{l+1} = c_{l-1} / F2_l.
// The step then reads e^{l+1} = alpha_l F0 (x - F1) e^l - e^{l-1} with alpha_l = c_{l+1} / c_l:
// two FP64 instructions, u = fma(x, A', nB') and e' = fma(u, e, -e_prev) with A' = alpha F0 and
// nB' = -alpha F0 F1, where the plain step takes three.  A value d^l is e^l / c_l: the forward
// folds 1/c_l into its weights, the adjoint into its per-l sums, the Wigner walk into its stores.
// Each factor (l+1)^2 - a^2 of F2's denominator exceeds l^2 - a^2 by at least 2l + 1, so
// F2_l <= (l+1)/l (l/(l+1))^2 = l/(l+1) < 1: c_l >= 1 grows along each parity of l, |d| <= |e|,
// and every skip test taken on e is conservative.  alpha is largest at its start,
// q(l0+2)/q(l0+1) <= 2 with q(l)^2 = (l^2 - mb^2)(l^2 - msky^2) / l^2 (the bound the growth
// constant above assumes; the host tests check it over the extreme columns up to l = 16384).
struct NormCoef {
    double A, nB;   // alpha_l F0_l, -alpha_l F0_l F1_l (0 from l = lmax on: the step is off)
    double ic;      // 1 / c_l
};

// Coefficients of l = lb + lane for one block of TB values of l, computed by all 64 lanes of
// one wave (the lanes past TB only take part in the scans).  carry holds c_{lb-2}, c_{lb-1}
// (ignored for the first block, whose carry is 1, 1) and is replaced by c_{lb+TB-2}, c_{lb+TB-1}.
// c_l is a product over segments of NORM_SEG values of l, each taking the last two c of the one
// before, so it rounds the same way for every TB (plans and plain calls agree bit for bit).
constexpr int NORM_SEG = 32;

template <int TB>
__device__ __forceinline__ NormCoef norm_coefs(int lb, int l0, int mb, int ms, int lmax, bool first, double* carry)
{
    static_assert(TB <= 64 && TB % NORM_SEG == 0, "one wave, whole segments");
    const int i = threadIdx.x & 63;
    const int l = lb + i;
    double A, nB, F2;
    recursion_coefs(l, mb, ms, lmax, A, nB, F2);
    double m = 1.0;   // c_l / c_{l-2}
    if (l >= l0 + 2 && l <= lmax) {
        double A1, nB1, F2m;
        recursion_coefs(l - 1, mb, ms, lmax, A1, nB1, F2m);
        m = 1.0 / F2m;
    }
    double c = m;     // products over the lanes of one parity within the segment: offsets 2 .. 16
    const int j = i & (NORM_SEG - 1);
#pragma unroll
    for (int off = 2; off < NORM_SEG; off *= 2) {
        const double v = __shfl_up(c, off, 64);
        if (j >= off) c *= v;
    }
    if (i < NORM_SEG) c *= (i & 1) ? (first ? 1.0 : carry[1]) : (first ? 1.0 : carry[0]);
    const double s_even = __shfl(c, NORM_SEG - 2, 64), s_odd = __shfl(c, NORM_SEG - 1, 64);
    if (i >= NORM_SEG) c *= (i & 1) ? s_odd : s_even;
    const double c_up = __shfl_up(c, 1, 64);
    double c_next = __shfl_down(c, 1, 64);                      // c_{l+1}
    if (i == 63) c_next = (l < lmax) ? (1.0 / F2) * c_up : c_up;  // as the next block's first lane
    const double alpha = c_next / c;
    if (i == TB - 2) carry[0] = c;
    if (i == TB - 1) carry[1] = c;
    return NormCoef{alpha * A, alpha * nB, 1.0 / c};
}

// Binary exponent e of max(|d|, |d_prev|) (|v| in [2^(e-1), 2^e)); a zero value does
// not count (the caller treats d = d_prev = 0 as the zero chain).
__device__ __forceinline__ int chain_exponent(double d, double dp)
{
    int e1, e2;
    frexp(d, &e1);
    frexp(dp, &e2);
    constexpr int NONE = -(1 << 20);
    return max(d != 0.0 ? e1 : NONE, dp != 0.0 ? e2 : NONE);
}

// For plain chains (E = 0) the skip test of check_chain reduces to a threshold:
// max(|d|, |d_prev|) >= 2^(-skip_exp - GROWTH_BITS_PER_STEP * TS).
template <int R>
__device__ __forceinline__ bool lane_may_be_hot(const double (&d)[R], const double (&dp)[R], double thr)
{
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) m = fmax(m, fmax(fabs(d[r]), fabs(dp[r])));
    return m >= thr;
}

// The same test between two rescales, while some chains are still scaled: those
// cannot be hot yet (see RS_STEPS), and their d is in scaled units, so they are left out.
template <int R>
__device__ __forceinline__ bool lane_may_be_hot_plain(const double (&d)[R], const double (&dp)[R],
                                                      const int (&E)[R], double thr)
{
    double m = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) m = fmax(m, E[r] == 0 ? fmax(fabs(d[r]), fabs(dp[r])) : 0.0);
    return m >= thr;
}

__device__ __forceinline__ double hot_threshold(int skip_exp)
{
    return ldexp(1.0, -skip_exp - GROWTH_BITS_PER_STEP * TS);
}

// One scale check of a chain (every RS_STEPS steps in the convolution walks, every
// TS steps where each d is written out).  From the exponent e of max(|d|, |d_prev|)
// it takes the true exponent te = E + e of the chain.
//  - rescale: a scaled chain (E < 0) is folded into plain doubles once te reaches
//    -900 (k = E), otherwise brought back to a significand near 1 (k = -e); the
//    power of two k applied to (d, d_prev) is returned for the caller's sums.
//  - returns whether |d| may reach 2^-skip_exp within the next TS steps (the walks
//    take that test from the plain chains' magnitudes instead, every TS steps).
// Branch-free per chain; the callers' conditions are wave-uniform.
__device__ __forceinline__ bool check_chain(double& d, double& dp, int& E, int skip_exp, bool rescale, int& k)
{
    const bool nz = (d != 0.0) | (dp != 0.0);
    const int e = chain_exponent(d, dp);
    const int te = E + e;
    k = 0;
    if (rescale) {
        const bool sc = nz & (E < 0);
        const bool fold = te >= FOLD_EXP;
        k = sc ? (fold ? E : -e) : 0;
        E = sc ? (fold ? 0 : te) : E;
        d = ldexp(d, k);
        dp = ldexp(dp, k);
    }
    return nz & (te + GROWTH_BITS_PER_STEP * TS > -skip_exp);
}

// One wave stages a whole block, so that its square roots and divisions keep all lanes busy,
// and the duty rotates over the workgroup's waves from block to block.
// Whether this lane's wave stages block `blk` (all of its lanes take part in norm_coefs).
template <int NT>
__device__ __forceinline__ bool stage_wave(int tid, int blk)
{
    return (tid >> 6) == blk % (NT / 64);
}

__device__ __forceinline__ size_t packed_index(int lmax, int l, int m)
{
    return (size_t)m * (size_t)(2 * lmax + 1 - m) / 2 + (size_t)l;
}

// ================================================================ wigner_d_rings
template <int R, int NT, int TB>
__global__ void __launch_bounds__(NT) k_wigner(const WignerArgs a)
{
    __shared__ double4 cf[2][TB];   // {A', nB', 1/c, -} per l
    __shared__ double carry[2];
    const int tid = threadIdx.x;
    const int pair = blockIdx.x / a.ntile;
    const int tile = blockIdx.x - pair * a.ntile;
    const int mb = a.col.mb[pair], ms = a.col.ms[pair];
    const int L = a.lmax;
    const int l0 = max(abs(mb), abs(ms));
    const SeedShape sh = seed_shape(mb, ms);
    const double lnAh = a.col.lnA[2 * pair], lnAl = a.col.lnA[2 * pair + 1];
    double* const out = a.d + (size_t)pair * (size_t)(L + 1) * (size_t)a.nring;

    double x[R], d[R], dp[R];
    int E[R], jj[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = tile * (NT * R) + r * NT + tid;
        jj[r] = j < a.nring ? j : -1;
        x[r] = 0.0; d[r] = 0.0; dp[r] = 0.0; E[r] = 0;
        if (jj[r] >= 0) {
            x[r] = a.ring.x[j];
            seed_value(lnAh, lnAl, sh, a.ring.lch[j], a.ring.lcl[j], a.ring.lsh[j], a.ring.lsl[j], d[r], E[r]);
            for (int l = 0; l < l0; ++l) out[(size_t)l * a.nring + j] = 0.0;
        }
    }
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) scaled |= (E[r] < 0);
    scaled = wave_any(scaled);

    const int lane = tid & 63;
    if (stage_wave<NT>(tid, 0)) {
        const NormCoef k = norm_coefs<TB>(l0, l0, mb, ms, L, true, carry);
        if (lane < TB) cf[0][lane] = make_double4(k.A, k.nB, k.ic, 0.0);
    }
    __syncthreads();
    const int nblk = (L - l0) / TB + 1;
    for (int kb = 0; kb < nblk; ++kb) {
        const int buf = kb & 1;
        const int lb = l0 + kb * TB;
        for (int s0 = 0; s0 < TB; s0 += TS) {
            if (scaled) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    int k;
                    check_chain(d[r], dp[r], E[r], 0, true, k);
                    any |= (E[r] < 0);
                }
                scaled = wave_any(any);
            }
#pragma unroll
            for (int t = 0; t < TS; ++t) {
                const int l = lb + s0 + t;
                const double4 k = cf[buf][s0 + t];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (jj[r] >= 0 && l <= L)
                        out[(size_t)l * a.nring + jj[r]] = ((E[r] == 0) ? d[r] : ldexp(d[r], E[r])) * k.z;
                    const double u = fma(x[r], k.x, k.y);
                    const double dn = fma(u, d[r], -dp[r]);
                    dp[r] = d[r];
                    d[r] = dn;
                }
            }
        }
        if (stage_wave<NT>(tid, kb + 1) && kb + 1 < nblk) {
            const NormCoef k = norm_coefs<TB>(lb + TB, l0, mb, ms, L, false, carry);
            if (lane < TB) cf[buf ^ 1][lane] = make_double4(k.A, k.nB, k.ic, 0.0);
        }
        __syncthreads();
    }
}

// ================================================================== forward
// Weights of step l for the (sky, beam) pair p: w1 = conj(b^p_{l,mb}) s^p_{l,msky} for
// the direct ring and w2 = (-1)^(l-msky) conj(b^p_{l,-mb}) s^p_{l,msky} for the mirror
// ring.  Scalar convolution: one pair.  Polarised convolution (footnote of Sec. 4.1):
// the temperature, gradient and curl pairs share the recursion, each with its own
// weights (NC = NP outputs) or with their weights summed (one output, NC = 1).  Detectors
// that share lmax and rings share it the same way, one output each (batched plans).
// Pair p's beam and output rows run over mb = -pmbmax[p] .. pmbmax[p].
struct RawW {
    double br, bi, b2r, b2i, sr, si;
};

__device__ __forceinline__ RawW load_weights_raw(const FwdArgs& a, int p, int l, int mb, int ms)
{
    RawW w{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (l <= a.lmax) {
        const double2* blm = reinterpret_cast<const double2*>(a.blm[p]);
        const double2* alm = reinterpret_cast<const double2*>(a.alm[p]);
        const double2 b1 = ldg(blm + (size_t)(mb + a.pmbmax[p]) * (a.lmax + 1) + l);
        const double2 b2 = ldg(blm + (size_t)(-mb + a.pmbmax[p]) * (a.lmax + 1) + l);
        const double2 s = ldg(alm + packed_index(a.sky_lmax, l, ms));
        w = RawW{b1.x, b1.y, b2.x, b2.y, s.x, s.y};
    }
    return w;
}

__device__ __forceinline__ double4 pair_weights(const RawW& w, int l, int ms)
{
    // conj(b) * s
    const double w1r = w.br * w.sr + w.bi * w.si;
    const double w1i = w.br * w.si - w.bi * w.sr;
    const double sg = ((l - ms) & 1) ? -1.0 : 1.0;
    const double w2r = sg * (w.b2r * w.sr + w.b2i * w.si);
    const double w2i = sg * (w.b2r * w.si - w.b2i * w.sr);
    return make_double4(w1r, w1i, w2r, w2i);
}

// Output c's weights from the raw loads of the NP pairs: pair c itself, or (NC = 1)
// the sum over all pairs in pair order.
template <int NC, int NP>
__device__ __forceinline__ double4 output_weights(const RawW (&raw)[NP], int c, int l, int ms)
{
    if (NC == NP) return pair_weights(raw[c], l, ms);
    double4 w = pair_weights(raw[0], l, ms);
#pragma unroll
    for (int p = 1; p < NP; ++p) {
        const double4 v = pair_weights(raw[p], l, ms);
        w.x += v.x; w.y += v.y; w.z += v.z; w.w += v.w;
    }
    return w;
}

// LDS slots of one l: {A, nB, F2, -}, then the general form's {w1r, w1i, w2r, w2i} per output
// or the even / odd form's {w1r, w1i} of two outputs per slot.
template <int NC, bool ROWS>
constexpr int coef_slots() { return ROWS ? 1 + (NC + 1) / 2 : 1 + NC; }

// The weights take the factor 1/c_l of the normalised walk.
template <int NC, int NP>
__device__ __forceinline__ void stage_block(const NormCoef& k, const RawW (&raw)[NP], int l, int ms, double4* slot)
{
    slot[0] = make_double4(k.A, k.nB, 0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double4 w = output_weights<NC, NP>(raw, c, l, ms);
        slot[1 + c] = make_double4(w.x * k.ic, w.y * k.ic, w.z * k.ic, w.w * k.ic);
    }
}

// The even / odd form needs w1 only: b^c_{l,mb} of each output and the sky, which the
// outputs of one walk share (the pairs' skies are one array).
template <int NC>
struct RawRows {
    double br[NC], bi[NC];
    double sr, si;
};

template <int NC, int P0>
__device__ __forceinline__ RawRows<NC> load_rows_raw(const FwdArgs& a, int l, int mb, int ms)
{
    RawRows<NC> w;
    w.sr = 0.0; w.si = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) { w.br[c] = 0.0; w.bi[c] = 0.0; }
    if (l <= a.lmax) {
        const double2 s = ldg(reinterpret_cast<const double2*>(a.alm[P0]) + packed_index(a.sky_lmax, l, ms));
        w.sr = s.x; w.si = s.y;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double2* blm = reinterpret_cast<const double2*>(a.blm[P0 + c]);
            const double2 b = ldg(blm + (size_t)(mb + a.pmbmax[P0 + c]) * (a.lmax + 1) + l);
            w.br[c] = b.x; w.bi[c] = b.y;
        }
    }
    return w;
}

template <int NC>
__device__ __forceinline__ void stage_block_rows(const NormCoef& k, const RawRows<NC>& w, double4* slot)
{
    slot[0] = make_double4(k.A, k.nB, 0.0, 0.0);
    double wr[NC + 1], wi[NC + 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) {   // conj(b) * s, as in pair_weights, times 1/c_l
        wr[c] = (w.br[c] * w.sr + w.bi[c] * w.si) * k.ic;
        wi[c] = (w.br[c] * w.si - w.bi[c] * w.sr) * k.ic;
    }
    wr[NC] = 0.0; wi[NC] = 0.0;
#pragma unroll
    for (int c = 0; c < NC; c += 2) slot[1 + c / 2] = make_double4(wr[c], wi[c], wr[c + 1], wi[c + 1]);
}

template <int R, int NC, bool ACC, int NS>
__device__ __forceinline__ void fwd_steps(const double4 (*cf)[NS], int s0,
                                          const double (&x)[R], double (&d)[R], double (&dp)[R],
                                          double (&c1r)[NC][R], double (&c1i)[NC][R],
                                          double (&c2r)[NC][R], double (&c2i)[NC][R])
{
#pragma unroll
    for (int t = 0; t < TS; ++t) {
        const double4 k = cf[s0 + t][0];
        double4 w[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (ACC) w[c] = cf[s0 + t][1 + c];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ACC) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    c1r[c][r] = fma(w[c].x, d[r], c1r[c][r]);
                    c1i[c][r] = fma(w[c].y, d[r], c1i[c][r]);
                    c2r[c][r] = fma(w[c].z, d[r], c2r[c][r]);
                    c2i[c][r] = fma(w[c].w, d[r], c2i[c][r]);
                }
            }
            const double u = fma(x[r], k.x, k.y);
            const double dn = fma(u, d[r], -dp[r]);
            dp[r] = d[r];
            d[r] = dn;
        }
    }
}

// Beam rows mb and -mb related by a sign s (b_{l,-mb} = s b_{l,mb}, as for a beam with
// real coefficients): then w2 = s (-1)^(l-msky) w1, and the direct and mirror sums both
// follow from the sums of w1 d over the even and over the odd steps of the walk, so a
// step adds w1 d into one of two sums (2 instead of 4 fused multiply-adds per chain and
// output).  The step parity is that of t (blocks and groups have even lengths): P0 += at
// even t, P1 at odd t, in the c1 and c2 registers of the general form.
template <int R, int NC, bool ACC, int NS>
__device__ __forceinline__ void fwd_steps_rows(const double4 (*cf)[NS], int s0,
                                               const double (&x)[R], double (&d)[R], double (&dp)[R],
                                               double (&p0r)[NC][R], double (&p0i)[NC][R],
                                               double (&p1r)[NC][R], double (&p1i)[NC][R])
{
    // With one output, each step's coefficients and weights are read during the step before (more
    // outputs leave no registers for it: their walks read them at the step).
    constexpr bool AHEAD = NC == 1;
    constexpr int NV = ACC ? (NC + 1) / 2 : 0;
    double4 kn;
    double4 vn[NV > 0 ? NV : 1];
    if constexpr (AHEAD) {
        kn = cf[s0][0];
#pragma unroll
        for (int c = 0; c < NV; ++c) vn[c] = cf[s0][1 + c];
    }
#pragma unroll
    for (int t = 0; t < TS; ++t) {
        if constexpr (!AHEAD) {
            kn = cf[s0 + t][0];
#pragma unroll
            for (int c = 0; c < NV; ++c) vn[c] = cf[s0 + t][1 + c];
        }
        const double4 k = kn;
        double wr[NC], wi[NC];
        if (ACC) {
#pragma unroll
            for (int c = 0; c < NC; c += 2) {
                const double4 v = vn[c / 2];
                wr[c] = v.x; wi[c] = v.y;
                if (c + 1 < NC) { wr[c + 1] = v.z; wi[c + 1] = v.w; }
            }
        }
        if (AHEAD && t + 1 < TS) {
            kn = cf[s0 + t + 1][0];
#pragma unroll
            for (int c = 0; c < NV; ++c) vn[c] = cf[s0 + t + 1][1 + c];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ACC) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if ((t & 1) == 0) {
                        p0r[c][r] = fma(wr[c], d[r], p0r[c][r]);
                        p0i[c][r] = fma(wi[c], d[r], p0i[c][r]);
                    } else {
                        p1r[c][r] = fma(wr[c], d[r], p1r[c][r]);
                        p1i[c][r] = fma(wi[c], d[r], p1i[c][r]);
                    }
                }
            }
            const double u = fma(x[r], k.x, k.y);
            const double dn = fma(u, d[r], -dp[r]);
            dp[r] = d[r];
            d[r] = dn;
        }
    }
}

template <int TB, int NS>
struct FwdShared {
    double4 cf[2][TB][NS];   // coefficient slots of the current and the next block
    double carry[2];         // c of the last two l of the latest staged block
};

// One (column, ring tile) work item of the forward over pairs P0 .. P0 + NP - 1 into outputs
// P0 .. P0 + NC - 1.  ROWS: the even / odd form, output c with beam row sign rows_sign[c].
template <int R, int NT, int TB, int NC, int NP, bool ROWS, int P0, int NS>
__device__ __forceinline__ void fwd_column_walk(const FwdArgs& a, int ci, int tile, const int* rows_sign,
                                                FwdShared<TB, NS>& sh_)
{
    static_assert(NC == 1 || NC == NP, "one output per pair, or one summed output");
    static_assert(!ROWS || NC == NP, "the even / odd form: one output per pair");
    static_assert(NS >= coef_slots<NC, ROWS>() && P0 + NP <= kMaxPairs, "coefficient slots, pairs");
    const int tid = threadIdx.x;
    const int mb = ldg(a.col.mb + ci), ms = ldg(a.col.ms + ci);
    const int L = a.lmax;
    const int l0 = max(abs(mb), ms);
    const SeedShape sh = seed_shape(mb, ms);
    const double lnAh = ldg(a.col.lnA + 2 * ci), lnAl = ldg(a.col.lnA + 2 * ci + 1);

    // the ring indices of the slots are read again for the stores (not held through the walk)
    const int s_base = tile * (NT * R) + tid * R;   // a wave: 64 R consecutive ring pairs
    double x[R], d[R], dp[R], c1r[NC][R], c1i[NC][R], c2r[NC][R], c2i[NC][R];
    int E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = s_base + r;
        x[r] = 0.0; d[r] = 0.0; dp[r] = 0.0; E[r] = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            c1r[c][r] = 0.0; c1i[c][r] = 0.0; c2r[c][r] = 0.0; c2i[c][r] = 0.0;
        }
        if (s < a.nslot) {
            const int j = ldg(a.slots + 2 * s);
            x[r] = ldg(a.ring.x + j);
            seed_value(lnAh, lnAl, sh, ldg(a.ring.lch + j), ldg(a.ring.lcl + j), ldg(a.ring.lsh + j),
                       ldg(a.ring.lsl + j), d[r], E[r]);
        }
    }
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) scaled |= (E[r] < 0);
    scaled = wave_any(scaled);
    bool acc_on = (a.skip_exp <= 0);
    const double thr = hot_threshold(a.skip_exp);

    RawW raw[NP];         // general form: the loads of the next block, in flight during a block
    RawRows<NC> rraw;     // even / odd form
    auto load_raw = [&](int l) {
        if constexpr (ROWS) {
            rraw = load_rows_raw<NC, P0>(a, l, mb, ms);
        } else {
#pragma unroll
            for (int p = 0; p < NP; ++p) raw[p] = load_weights_raw(a, P0 + p, l, mb, ms);
        }
    };
    // the staging wave's lanes: l = lb + lane; the coefficients need all 64 lanes
    const int lane = tid & 63;
    auto stage_raw = [&](int lb, bool first, double4 (*slots)[NS]) {
        const NormCoef k = norm_coefs<TB>(lb, l0, mb, ms, L, first, sh_.carry);
        if (lane < TB) {
            if constexpr (ROWS)
                stage_block_rows<NC>(k, rraw, slots[lane]);
            else
                stage_block<NC, NP>(k, raw, lb + lane, ms, slots[lane]);
        }
    };
    if (stage_wave<NT>(tid, 0)) {
        if (lane < TB) load_raw(l0 + lane);
        stage_raw(l0, true, sh_.cf[0]);
    }
    __syncthreads();
    constexpr int RS_BLK = rs_block<TB>();   // steps between rescales of scaled chains
    const int nblk = (L - l0) / TB + 1;
    for (int kb = 0; kb < nblk; ++kb) {
        const int buf = kb & 1;
        const int lb = l0 + kb * TB;
        const bool stage = stage_wave<NT>(tid, kb + 1) && (kb + 1 < nblk);
        if (stage && lane < TB) load_raw(lb + TB + lane);   // in flight during the block
        for (int s1 = 0; s1 < TB; s1 += RS_BLK) {
            if (scaled) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    int k;
                    (void)check_chain(d[r], dp[r], E[r], a.skip_exp, true, k);
                    if (acc_on) {   // sums in the chain's scaled units follow it
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            c1r[c][r] = ldexp(c1r[c][r], k); c1i[c][r] = ldexp(c1i[c][r], k);
                            c2r[c][r] = ldexp(c2r[c][r], k); c2i[c][r] = ldexp(c2i[c][r], k);
                        }
                    }
                    any |= (E[r] < 0);
                }
                scaled = wave_any(any);
            }
            // kept rolled: unrolled, the 4-wave forward spills twice as many registers
#pragma unroll 1
            for (int s0 = s1; s0 < s1 + RS_BLK; s0 += TS) {
                if (!acc_on)
                    acc_on = wave_any(scaled ? lane_may_be_hot_plain<R>(d, dp, E, thr) : lane_may_be_hot<R>(d, dp, thr));
                if (!acc_on)
                    fwd_steps<R, NC, false>(sh_.cf[buf], s0, x, d, dp, c1r, c1i, c2r, c2i);
                else if constexpr (ROWS)
                    fwd_steps_rows<R, NC, true>(sh_.cf[buf], s0, x, d, dp, c1r, c1i, c2r, c2i);
                else
                    fwd_steps<R, NC, true>(sh_.cf[buf], s0, x, d, dp, c1r, c1i, c2r, c2i);
            }
        }
        if (stage) stage_raw(lb + TB, false, sh_.cf[buf ^ 1]);
        __syncthreads();
    }

    if constexpr (ROWS) {
        // direct sum P0 + P1; mirror sum s (-1)^(msky + l0) (P0 - P1)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double sg = ((ms + l0) & 1) ? -(double)rows_sign[c] : (double)rows_sign[c];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double er = c1r[c][r] + c2r[c][r], ei = c1i[c][r] + c2i[c][r];
                const double mr = sg * (c1r[c][r] - c2r[c][r]), mi = sg * (c1i[c][r] - c2i[c][r]);
                c1r[c][r] = er; c1i[c][r] = ei; c2r[c][r] = mr; c2i[c][r] = mi;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int M = a.pmbmax[P0 + c];
        const size_t row_d = ((size_t)(mb + M) * (L + 1) + ms) * (size_t)a.nring;
        const size_t row_m = ((size_t)(-mb + M) * (L + 1) + ms) * (size_t)a.nring;
        double2* C = reinterpret_cast<double2*>(a.C[P0 + c]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int s = s_base + r;
            if (s < a.nslot) {
                const int jd = ldg(a.slots + 2 * s), jm = ldg(a.slots + 2 * s + 1);
                stg(C + row_d + jd, make_double2(ldexp(c1r[c][r], E[r]), ldexp(c1i[c][r], E[r])));
                if (jm >= 0)
                    stg(C + row_m + jm, make_double2(ldexp(c2r[c][r], E[r]), ldexp(c2i[c][r], E[r])));
            }
        }
    }
}

// Beam row sign of pair p for row mb (0: the rows are not related by a sign).
__device__ __forceinline__ int row_sign(const FwdArgs& a, int p, int mb)
{
    return ldg(a.beam_sym[p] + mb + a.pmbmax[p]);
}

// The scalar forward runs as two launches over every (column, tile): k_fwd_rows takes the
// columns whose beam rows are equal up to a sign, k_fwd the others (and every polarised
// column); a workgroup whose column belongs to the other launch returns at once.
template <int R, int NT, int TB, int NC, int NP>
__global__ void __launch_bounds__(NT, (fwd_min_waves<R, NC, NP>())) k_fwd(const FwdArgs a)
{
    __shared__ FwdShared<TB, 1 + NC> sh;
    const int ci = blockIdx.x / a.ntile;
    if constexpr (NC == 1 && NP == 1) {
        if (a.beam_sym[0] && row_sign(a, 0, ldg(a.col.mb + ci)) != 0) return;
    }
    const int none[NC] = {};
    fwd_column_walk<R, NT, TB, NC, NP, false, 0>(a, ci, blockIdx.x - ci * a.ntile, none, sh);
}

template <int R, int NT, int TB>
__global__ void __launch_bounds__(NT, (rows_min_waves<R>())) k_fwd_rows(const FwdArgs a)
{
    __shared__ FwdShared<TB, 2> sh;
    const int ci = blockIdx.x / a.ntile;
    const int s[1] = {row_sign(a, 0, ldg(a.col.mb + ci))};
    if (s[0] == 0) return;
    fwd_column_walk<R, NT, TB, 1, 1, true, 0>(a, ci, blockIdx.x - ci * a.ntile, s, sh);
}

// Batched form: one workgroup per (walk, column, ring tile) item, the items in order of cost,
// longest first (workgroups start in index order).  A walk serves the npair <= walk_pairs<R>()
// detectors that share its lmax and rings, ordered by mbmax, largest first: the first k of them
// have the column's beam row mb.  When all k have that row pair equal up to a sign, one even /
// odd walk feeds the k outputs; otherwise each detector takes a walk of its own, in the form a
// plain call would take, so every output is the one a plain call with this tile writes.
//
// Detectors per walk: the even / odd sums take 8 VGPRs per chain and output, so R = 8 chains
// per lane hold two outputs within the 2-wave budget and R <= 4 hold four.
template <int R>
constexpr int walk_pairs() { return R >= 8 ? 2 : 4; }

template <int R>
constexpr int items_min_waves() { return R >= 4 ? 2 : 3; }

template <int R, int NT, int TB, int NS, int P>
__device__ __forceinline__ void fwd_item_alone(const FwdArgs& a, int ci, int tile, int k, const int (&s)[kMaxPairs],
                                               FwdShared<TB, NS>& cf)
{
    if (P < k) {
        if (s[P] != 0)
            fwd_column_walk<R, NT, TB, 1, 1, true, P>(a, ci, tile, s + P, cf);
        else
            fwd_column_walk<R, NT, TB, 1, 1, false, P>(a, ci, tile, s + P, cf);
    }
}

template <int R, int NT, int TB>
__global__ void __launch_bounds__(NT, (items_min_waves<R>())) k_fwd_items(const FwdArgs* __restrict__ walks,
                                                                          const int* __restrict__ items)
{
    constexpr int K = walk_pairs<R>();
    static_assert(K == 2 || K == 4, "walk sizes");
    constexpr int NS = coef_slots<K, true>() > 2 ? coef_slots<K, true>() : 2;
    __shared__ FwdShared<TB, NS> cf;
    const int* item = items + 3 * (size_t)blockIdx.x;
    const FwdArgs a = walks[item[0]];
    const int ci = item[1], tile = item[2];
    const int mb = ldg(a.col.mb + ci);
    int k = 0, s[kMaxPairs];
    bool rows = true;
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
        s[p] = 0;
        if (p < K && p < a.npair && a.pmbmax[p] >= abs(mb)) {
            k = p + 1;
            s[p] = row_sign(a, p, mb);
            rows = rows && s[p] != 0;
        }
    }
    if (rows) {
        if (k == 1) { fwd_column_walk<R, NT, TB, 1, 1, true, 0>(a, ci, tile, s, cf); return; }
        if (k == 2) { fwd_column_walk<R, NT, TB, 2, 2, true, 0>(a, ci, tile, s, cf); return; }
        if constexpr (K == 4) {
            if (k == 3) { fwd_column_walk<R, NT, TB, 3, 3, true, 0>(a, ci, tile, s, cf); return; }
            fwd_column_walk<R, NT, TB, 4, 4, true, 0>(a, ci, tile, s, cf);
            return;
        }
    }
    fwd_item_alone<R, NT, TB, NS, 0>(a, ci, tile, k, s, cf);
    fwd_item_alone<R, NT, TB, NS, 1>(a, ci, tile, k, s, cf);
    if constexpr (K == 4) {
        fwd_item_alone<R, NT, TB, NS, 2>(a, ci, tile, k, s, cf);
        fwd_item_alone<R, NT, TB, NS, 3>(a, ci, tile, k, s, cf);
    }
}

// ================================================================== adjoint
// Per column and l: u_l = sum_j d^l(beta_j) Cbar_j over the direct rings (U)
// and sum_j d^l(beta_j) Cbar_{-mb,msky}(pi - beta_j) over the mirror rings (V).
//
// Systolic row sums.  The 16 lanes of a row walk skewed: lane k (k = lane mod 16) is k
// steps behind lane 0 of its row, so at the row's time t it is at l = l0 + t - k.  Each
// lane carries four running sums (U re/im, V re/im).  Every step the sums move one lane
// up the row (DPP row_shr:1; lane 0 of the row starts a fresh sum at 0) and the lane adds
// d * Cbar of its R chains for its own l: a sum visits the 16 lanes of the row at the
// same l and leaves lane 15 complete, 15 steps after it began, where it is written to
// LDS.  After the TB block's barrier the four rows' and the waves' sums of each l are
// added in a fixed order and written out.  No LDS round trip sits in the step loop and
// nothing is reduced across lanes but the one shift per sum and step; the order of
// every sum is fixed, so the result is deterministic.

constexpr int ROW = 16;             // lanes per systolic row
constexpr int SKEW = ROW - 1;       // steps lane 15 trails lane 0 of its row

// The value of the lane one below in the same row of 16; lane 0 of a row gets 0.
__device__ __forceinline__ double row_shift_up(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x111, 0xF, 0xF, true);   // row_shr:1
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x111, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Emitted row sums: slot (t - 16) mod 2 TB for the sum that leaves lane 15 at time t
// (l offset t - 15), then (wave, row, component); slots are out_stride doubles apart: two more
// than the NW 4 4 NC they hold, an even count, so that every slot is 16-byte aligned and a step
// group's emissions are 128-bit stores at constant offsets from one address (the reads of the
// block sum, one slot per lane, then meet at most two to a bank).  NC cotangents share the walk:
// 4 NC components.
template <int NT, int NC>
constexpr int out_stride() { return (NT / 64) * 4 * 4 * NC + 2; }

// The coefficient ring holds four blocks of TB l offsets plus a copy of its first TS
// slots behind its end, so that the TS consecutive offsets of a step group never wrap.
// NCMAX: the most cotangents a walk in this workgroup serves.
template <int NT, int TB, int NCMAX>
struct AdjShared {
    double2 cfa[4 * TB + TS];                     // {A', nB'} per l offset, slot = offset mod 4 TB
    double cic[4 * TB + TS];                      // 1 / c_l per l offset (the copy is not read)
    double out[2 * TB * out_stride<NT, NCMAX>()]; // emitted row sums
    double carry[2];                              // normalisation carry between blocks
};

template <int NT, int TB, int NCMAX>
constexpr size_t adj_lds_bytes() { return sizeof(AdjShared<NT, TB, NCMAX>); }

// One ring tile of column ci for the cotangents 0 .. NC - 1 of the walk (a.Cbar[c], sums into
// a.U[c], a.V[c], rows of cotangent c offset by a.pmbmax[c]).
template <int R, int NT, int TB, int NC, int NCMAX>
__device__ __forceinline__ void adj_column(const AdjArgs& a, int ci, int tile, AdjShared<NT, TB, NCMAX>& sh_)
{
    static_assert(TB % TS == 0 && TS % 2 == 0 && TB >= ROW, "step groups: pairs of steps, TS per check");
    static_assert(NC <= NCMAX && NC <= kMaxPairs, "cotangents per walk");
    constexpr int NW = NT / 64;
    constexpr int NS = 4 * NC;              // running sums per lane: (U re, U im, V re, V im) per cotangent
    constexpr int CF_N = 4 * TB;            // coefficient ring: offset blocks kb-1, kb (read), kb+1 (staged)
    constexpr int CF_MASK = CF_N - 1;
    constexpr int OUT_MASK = 2 * TB - 1;    // emitted sums: windows kb (written) and kb-1 (summed)
    constexpr int OS = out_stride<NT, NC>();
    static_assert((CF_N & CF_MASK) == 0 && (2 * TB & OUT_MASK) == 0 && (SKEW + 1) % TS == 0, "ring sizes");
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int kr = lane & (ROW - 1), row = lane >> 4;
    const int mb = ldg(a.col.mb + ci), ms = ldg(a.col.ms + ci);
    const int L = a.lmax;
    const int l0 = max(abs(mb), ms);
    const int n = L - l0 + 1;              // l values of a chain
    const SeedShape sh = seed_shape(mb, ms);
    const double lnAh = ldg(a.col.lnA + 2 * ci), lnAl = ldg(a.col.lnA + 2 * ci + 1);
    const int s_base = tile * (NT * R) + tid * R;   // a wave: 64 R consecutive ring slots

    double x[R], d[R], dp[R], g1r[NC][R], g1i[NC][R], g2r[NC][R], g2i[NC][R];
    int E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = s_base + r;
        x[r] = 0.0; d[r] = 0.0; dp[r] = 0.0; E[r] = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) { g1r[c][r] = 0.0; g1i[c][r] = 0.0; g2r[c][r] = 0.0; g2i[c][r] = 0.0; }
        if (s < a.nslot) {
            const int j = ldg(a.slots + 2 * s);
            x[r] = ldg(a.ring.x + j);
            seed_value(lnAh, lnAl, sh, ldg(a.ring.lch + j), ldg(a.ring.lcl + j), ldg(a.ring.lsh + j),
                       ldg(a.ring.lsl + j), d[r], E[r]);
        }
    }
    // A scaled chain (E < 0, |d| < 2^-900) contributes nothing; its cotangents are
    // loaded when it folds into plain doubles.
    auto load_g = [&](int r) {
        const int s = s_base + r;
        if (s < a.nslot && E[r] == 0) {
            const int jd = ldg(a.slots + 2 * s), jm = ldg(a.slots + 2 * s + 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double2* Cbar = reinterpret_cast<const double2*>(a.Cbar[c]);
                const int M = a.pmbmax[c];
                const size_t row_d = ((size_t)(mb + M) * (L + 1) + ms) * (size_t)a.nring;
                const size_t row_m = ((size_t)(-mb + M) * (L + 1) + ms) * (size_t)a.nring;
                const double2 v1 = ldg(Cbar + row_d + jd);
                g1r[c][r] = v1.x; g1i[c][r] = v1.y;
                if (jm >= 0) {
                    const double2 v2 = ldg(Cbar + row_m + jm);
                    g2r[c][r] = v2.x; g2i[c][r] = v2.y;
                }
            }
        }
    };
#pragma unroll
    for (int r = 0; r < R; ++r) load_g(r);
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) scaled |= (E[r] < 0);
    scaled = wave_any(scaled);
    bool acc_on = (a.skip_exp <= 0);    // wave-uniform
    const double thr = hot_threshold(a.skip_exp);

    // one U and one V row per column and cotangent: ring tile 0 writes them, each later tile
    // (walked after it by the same workgroup) adds to them
    const size_t urow = packed_index(L, 0, ms);   // + l

    auto stage = [&](int blk) {
        if (stage_wave<NT>(tid, blk)) {
            const NormCoef k = norm_coefs<TB>(l0 + blk * TB, l0, mb, ms, L, blk == 0, sh_.carry);
            if (lane < TB) {
                const int slot = (blk * TB + lane) & CF_MASK;
                sh_.cfa[slot] = make_double2(k.A, k.nB);
                sh_.cic[slot] = k.ic;
                if (slot < TS) sh_.cfa[CF_N + slot] = make_double2(k.A, k.nB);   // the copy behind the ring's end
            }
        }
    };
    // Lane 15 of each row stores the sums that leave it.  The sums alternate between two
    // register sets step by step, so that the two sums a pair of steps completes are both
    // still held after it and one store (a branch: only these lanes take it) serves two steps.
    const bool exit_lane = kr == SKEW;
    double* const outw = sh_.out + (wave * 4 + row) * NS;
    double sa[NS], sb[NS];   // set a: the sums after an odd step; set b: after an even step
#pragma unroll
    for (int q = 0; q < NS; ++q) { sa[q] = 0.0; sb[q] = 0.0; }
    auto emit2 = [&](int t) {   // step t completed set b, step t + 1 set a; slots t - 16, t - 15
        if (exit_lane) {
            double* o = outw + ((t - SKEW - 1) & OUT_MASK) * OS;
#pragma unroll
            for (int q = 0; q < NS; ++q) o[q] = sb[q];
            o = outw + ((t - SKEW) & OUT_MASK) * OS;
#pragma unroll
            for (int q = 0; q < NS; ++q) o[q] = sa[q];
        }
    };
    // The same for step t0 + h of a step group that starts at t0, a multiple of TS: the group's
    // slots t0 - 16 .. t0 - 16 + TS - 1 do not wrap the ring (t0 - 16 is a multiple of TS too), so
    // they are og (the group's first slot, one address per group) plus constant offsets.
    static_assert((SKEW + 1) % TS == 0 && (2 * TB) % TS == 0, "a step group's slots do not wrap");
    auto emit2_in = [&](double* og, int h) {
        if (exit_lane) {
            double* o = og + h * OS;
#pragma unroll
            for (int q = 0; q < NS; ++q) o[q] = sb[q];
            o = og + (h + 1) * OS;
#pragma unroll
            for (int q = 0; q < NS; ++q) o[q] = sa[q];
        }
    };
    auto shift_a_to_b = [&]() {
#pragma unroll
        for (int q = 0; q < NS; ++q) sb[q] = row_shift_up(sa[q]);
    };
    auto shift_b_to_a = [&]() {
#pragma unroll
        for (int q = 0; q < NS; ++q) sa[q] = row_shift_up(sb[q]);
    };
    // one step of the R chains of this lane: coefficients k; the sums s take e * Cbar
    auto step = [&](const double2 k, double (&s)[NS]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                s[4 * c + 0] = fma(d[r], g1r[c][r], s[4 * c + 0]);
                s[4 * c + 1] = fma(d[r], g1i[c][r], s[4 * c + 1]);
                s[4 * c + 2] = fma(d[r], g2r[c][r], s[4 * c + 2]);
                s[4 * c + 3] = fma(d[r], g2i[c][r], s[4 * c + 3]);
            }
            const double u = fma(x[r], k.x, k.y);
            const double dn = fma(u, d[r], -dp[r]);
            dp[r] = d[r];
            d[r] = dn;
        }
    };

    stage(0);
    __syncthreads();
    constexpr int RS_BLK = rs_block<TB>();   // steps between rescales of scaled chains
    // lane 15 of a row finishes l = L at time n - 1 + SKEW
    const int nblk = (n + SKEW + TB - 1) / TB;
    for (int kb = 0; kb < nblk; ++kb) {
        const int buf_t = kb * TB;
        for (int s1 = 0; s1 < TB; s1 += RS_BLK) {
            if (scaled) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool was = E[r] < 0;
                    int k;
                    (void)check_chain(d[r], dp[r], E[r], a.skip_exp, true, k);
                    if (was && E[r] == 0) load_g(r);
                    any |= (E[r] < 0);
                }
                scaled = wave_any(any);
            }
            for (int s0 = s1; s0 < s1 + RS_BLK; s0 += TS) {
                const int t0 = buf_t + s0;   // row time of the group's first step
                // a lane that has not started yet holds its seed, so the test covers it
                if (!acc_on)
                    acc_on = wave_any(scaled ? lane_may_be_hot_plain<R>(d, dp, E, thr) : lane_may_be_hot<R>(d, dp, thr));
                if (t0 < SKEW) {
                    // start of the walk: lane k holds its chain (seed, 0) until time k and adds nothing
#pragma unroll
                    for (int t = 0; t < TS; ++t) {
                        const int tt = t0 + t;
                        const bool live = tt >= kr;
                        const int off = live ? tt - kr : 0;
                        const double2 k = sh_.cfa[off & CF_MASK];
                        if (t & 1) shift_b_to_a(); else shift_a_to_b();
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const double dd = (live && acc_on) ? d[r] : 0.0;
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                double* s = (t & 1) ? sa : sb;
                                s[4 * c + 0] = fma(dd, g1r[c][r], s[4 * c + 0]);
                                s[4 * c + 1] = fma(dd, g1i[c][r], s[4 * c + 1]);
                                s[4 * c + 2] = fma(dd, g2r[c][r], s[4 * c + 2]);
                                s[4 * c + 3] = fma(dd, g2i[c][r], s[4 * c + 3]);
                            }
                            const double u = fma(x[r], k.x, k.y);
                            const double dn = fma(u, d[r], -dp[r]);
                            dp[r] = live ? d[r] : dp[r];
                            d[r] = live ? dn : d[r];
                        }
                        if (t & 1) emit2(tt - 1);
                    }
                } else if (acc_on) {
                    // pairs of steps; each pair's coefficients are read during the pair before
                    const int cb = (t0 - kr) & CF_MASK;
                    double* const og = outw + ((t0 - SKEW - 1) & OUT_MASK) * OS;
                    double2 kn0 = sh_.cfa[cb], kn1 = sh_.cfa[cb + 1];
#pragma unroll
                    for (int h = 0; h < TS; h += 2) {
                        const double2 k0 = kn0, k1 = kn1;
                        if (h + 2 < TS) {
                            kn0 = sh_.cfa[cb + h + 2]; kn1 = sh_.cfa[cb + h + 3];
                        }
                        shift_a_to_b();
                        step(k0, sb);
                        shift_b_to_a();
                        step(k1, sa);
                        emit2_in(og, h);
                    }
                } else {
                    const int cb = (t0 - kr) & CF_MASK;
#pragma unroll
                    for (int t = 0; t < TS; ++t) {
                        const double2 k = sh_.cfa[cb + t];
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const double u = fma(x[r], k.x, k.y);
                            const double dn = fma(u, d[r], -dp[r]);
                            dp[r] = d[r];
                            d[r] = dn;
                        }
                    }
                    // nothing is added yet: every sum of these steps is zero
#pragma unroll
                    for (int q = 0; q < NS; ++q) { sa[q] = 0.0; sb[q] = 0.0; }
                    double* const og = outw + ((t0 - SKEW - 1) & OUT_MASK) * OS;
#pragma unroll
                    for (int t = 0; t < TS; t += 2) emit2_in(og, t);
                }
            }
        }
        if (kb + 1 < nblk) stage(kb + 1);
        __syncthreads();
        // window kb: the sums of l offsets kb TB - 15 .. (kb+1) TB - 16, all emitted in this
        // block; the waves and rows in a fixed order (the next block writes the other window)
        for (int q = tid; q < TB * NS; q += NT) {
            const int o = buf_t - SKEW + q / NS, comp = q % NS;
            if (o >= 0 && o < n) {
                const double* src = sh_.out + ((o - 1) & OUT_MASK) * OS + comp;
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < NW * 4; ++w) v += src[NS * w];
                v *= sh_.cic[o & CF_MASK];   // e^l back to d^l
                const int c = comp >> 2, part = comp & 3;
                // the cotangent's rows by selection: a runtime index into the argument
                // record would move the record to scratch memory
                double* uv = part < 2 ? a.U[0] : a.V[0];
                int M = a.pmbmax[0];
#pragma unroll
                for (int cc = 1; cc < NC; ++cc)
                    if (c == cc) { uv = part < 2 ? a.U[cc] : a.V[cc]; M = a.pmbmax[cc]; }
                double* dst = uv + 2 * ((size_t)(mb + M) * (size_t)a.P + urow + l0 + o) + (part & 1);
                stg(dst, (tile == 0) ? v : ldg(dst) + v);
            }
        }
    }
}

// All ring tiles of column ci, one after the other in one workgroup: tile 0 writes the
// column's U and V rows, each later tile adds to them (the same thread writes an element in
// every tile), so no launch has to wait for another.  The column's values the compiler keeps
// across tiles spill outside the step loops only.
template <int R, int NT, int TB, int NC, int NCMAX>
__device__ __forceinline__ void adj_tiles(const AdjArgs& a, int ci, AdjShared<NT, TB, NCMAX>& sh)
{
    for (int tile = 0; tile < a.ntile; ++tile) {
        if (tile > 0) __syncthreads();   // the tile before still reads the LDS ring in its last block sums
        adj_column<R, NT, TB, NC, NCMAX>(a, ci, tile, sh);
    }
}

template <int R, int NT, int TB, int TR>
__global__ void __launch_bounds__(NT, (adj_min_waves<R, TB>())) k_adj(const AdjArgs a)
{
    static_assert(adj_lds_bytes<NT, TB, 1>() * adj_min_waves<R, TB>() <= 160 * 1024, "LDS per CU");
    __shared__ AdjShared<NT, TB, 1> sh;
    adj_tiles<R, NT, TB, 1, 1>(a, blockIdx.x, sh);
}

// Batched form: one workgroup per (walk, column) item, the items longest first.  A walk serves
// the npair <= adj_walk_pairs<TB>() detectors that share its lmax and rings, ordered by mbmax,
// largest first: the first k of them have the column's beam row mb, and one walk adds into
// the sums of all k (2 + 4 k instructions and 4 k / R row shifts per chain step, where k walks
// of their own take 6 k and 4 k / R).  Two cotangents double the emitted-sum buffer, which
// with TB 64 would leave one workgroup per CU, and hold 8 cotangent doubles per chain, which
// at R 8 exceed the 256 registers of two waves per SIMD: paired walks are built with TB 32 and
// R <= 4 only (two workgroups per CU).
template <int R, int TB>
constexpr int adj_walk_pairs() { return (R <= 4 && TB <= 32) ? 2 : 1; }

// Paired walks hold two workgroups per CU (their LDS), which is the register budget they get.
template <int R, int TB>
constexpr int adj_items_min_waves() { return adj_walk_pairs<R, TB>() == 2 ? 2 : adj_min_waves<R, TB>(); }

template <int R, int NT, int TB, int TR>
__global__ void __launch_bounds__(NT, (adj_items_min_waves<R, TB>())) k_adj_items(const AdjArgs* __restrict__ dets,
                                                                            const int* __restrict__ items)
{
    constexpr int K = adj_walk_pairs<R, TB>();
    static_assert(adj_lds_bytes<NT, TB, K>() * 2 <= 160 * 1024, "two workgroups per CU");
    __shared__ AdjShared<NT, TB, K> sh;
    const int* item = items + 2 * (size_t)blockIdx.x;
    const int ci = item[1];
    if constexpr (K == 2) {
        // read in place: a copy of the record would sit in scratch memory in this form
        const AdjArgs& a = dets[item[0]];
        if (a.npair > 1 && a.pmbmax[1] >= abs(ldg(a.col.mb + ci)))
            adj_tiles<R, NT, TB, 2, K>(a, ci, sh);
        else
            adj_tiles<R, NT, TB, 1, K>(a, ci, sh);
    } else {
        const AdjArgs a = dets[item[0]];
        adj_tiles<R, NT, TB, 1, K>(a, ci, sh);
    }
}

// u(mb, ms, l) = U[mb] + (-1)^(l-ms) V[-mb], defined for l >= max(|mb|, ms)
__device__ __forceinline__ double2 u_value(const EpiArgs& e, int mb, int ms, int l, size_t k)
{
    const double2 a = ldg(reinterpret_cast<const double2*>(e.U) + (size_t)(mb + e.mbmax) * e.P + k);
    const double2 b = ldg(reinterpret_cast<const double2*>(e.V) + (size_t)(-mb + e.mbmax) * e.P + k);
    const double sg = ((l - ms) & 1) ? -1.0 : 1.0;
    return make_double2(a.x + sg * b.x, a.y + sg * b.y);
}

// Adds sum_mb b_{l,mb} u(mb, ms, l) of one detector to (ar, ai), mb ascending.  The rows are
// read SKY_ROWS at a time before any is used, so that a thread keeps that many row loads in
// flight instead of one.
constexpr int SKY_ROWS = 8;
__device__ __forceinline__ void sky_grad_terms(const EpiArgs& e, int ms, int l, double& ar, double& ai)
{
    const size_t k = packed_index(e.lmax, l, ms);
    const double2* U = reinterpret_cast<const double2*>(e.U) + k;
    const double2* V = reinterpret_cast<const double2*>(e.V) + k;
    const double2* blm = reinterpret_cast<const double2*>(e.blm) + l;
    const int M = e.mbmax, lo = max(-M, -l), hi = min(M, l);   // rows with l >= |mb|
    const double sg = ((l - ms) & 1) ? -1.0 : 1.0;
    for (int mb0 = lo; mb0 <= hi; mb0 += SKY_ROWS) {
        double2 ua[SKY_ROWS], va[SKY_ROWS], ba[SKY_ROWS];
#pragma unroll
        for (int q = 0; q < SKY_ROWS; ++q) {
            const int mb = min(mb0 + q, hi);   // past the last row: a repeat of it, not added
            ua[q] = ldg(U + (size_t)(mb + M) * e.P);
            va[q] = ldg(V + (size_t)(-mb + M) * e.P);
            ba[q] = ldg(blm + (size_t)(mb + M) * (e.lmax + 1));
        }
#pragma unroll
        for (int q = 0; q < SKY_ROWS; ++q) {
            if (mb0 + q <= hi) {
                const double2 u = make_double2(ua[q].x + sg * va[q].x, ua[q].y + sg * va[q].y);
                const double2 b = ba[q];
                ar += b.x * u.x - b.y * u.y;
                ai += b.x * u.y + b.y * u.x;
            }
        }
    }
}

// alm_bar_{l,ms} = sum_mb b_{l,mb} u(mb, ms, l)
__global__ void __launch_bounds__(256) k_adj_sky(const EpiArgs e)
{
    const int ms = blockIdx.y;
    const int l = ms + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > e.sky_lmax) return;
    double ar = 0.0, ai = 0.0;
    if (l <= e.lmax) sky_grad_terms(e, ms, l, ar, ai);
    stg(reinterpret_cast<double2*>(e.alm_bar) + packed_index(e.sky_lmax, l, ms), make_double2(ar, ai));
}

// Batched form: the sky gradient of ndet detectors, summed in their order; with accumulate the
// sum is added to what alm_bar holds (the detectors of earlier launches), else it replaces it.
__global__ void __launch_bounds__(256) k_adj_sky_multi(const EpiArgs* __restrict__ eps, int ndet, int sky_lmax,
                                                       int accumulate, double* __restrict__ alm_bar)
{
    const int ms = blockIdx.y;
    const int l = ms + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > sky_lmax) return;
    double2* out = reinterpret_cast<double2*>(alm_bar) + packed_index(sky_lmax, l, ms);
    double ar = 0.0, ai = 0.0;
    if (accumulate) {
        const double2 o = ldg(out);
        ar = o.x;
        ai = o.y;
    }
    for (int dt = 0; dt < ndet; ++dt) {
        const EpiArgs& e = eps[dt];
        if (l <= e.lmax) sky_grad_terms(e, ms, l, ar, ai);
    }
    stg(out, make_double2(ar, ai));
}

// blm_bar_{l,mb} = sum_{ms <= l} s_{l,ms} conj(u(mb, ms, l)), one thread per (l, mb)
__global__ void __launch_bounds__(256) k_adj_beam(const EpiArgs e)
{
    const int mb = (int)blockIdx.y - e.mbmax;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > e.lmax) return;
    double2* out = reinterpret_cast<double2*>(e.blm_bar) + (size_t)(mb + e.mbmax) * (e.lmax + 1) + l;
    if (l < abs(mb)) {
        stg(out, make_double2(0.0, 0.0));
        return;
    }
    const double2* alm = reinterpret_cast<const double2*>(e.alm);
    double br = 0.0, bi = 0.0;
#pragma unroll 4
    for (int ms = 0; ms <= l; ++ms) {
        const double2 u = u_value(e, mb, ms, l, packed_index(e.lmax, l, ms));
        const double2 s = ldg(alm + packed_index(e.sky_lmax, l, ms));
        br += s.x * u.x + s.y * u.y;
        bi += s.y * u.x - s.x * u.y;
    }
    stg(out, make_double2(br, bi));
}

template <typename Args>
int launch_grid(void (*kern)(Args), const Args& a, int blocks, int nt, void* stream)
{
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(nt), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// Beam rows related by a sign: sym[M + mb] = sym[M - mb] = s if b_{l,-mb} = s b_{l,mb} for
// every l >= |mb| (s = +1 when both signs hold, as for zero rows and mb = 0), else 0.
__global__ void __launch_bounds__(256) k_beam_symmetry(const double2* __restrict__ blm, int lmax, int mbmax,
                                                       int* __restrict__ sym)
{
    const int mb = blockIdx.x;   // 0 .. mbmax
    const double2* bp = blm + (size_t)(mbmax + mb) * (lmax + 1);
    const double2* bm = blm + (size_t)(mbmax - mb) * (lmax + 1);
    bool plus = true, minus = true;
    for (int l = mb + (int)threadIdx.x; l <= lmax; l += 256) {
        const double2 p = bp[l], m = bm[l];
        plus = plus && (m.x == p.x) && (m.y == p.y);
        minus = minus && (m.x == -p.x) && (m.y == -p.y);
    }
    plus = __syncthreads_and(plus);
    minus = __syncthreads_and(minus);
    if (threadIdx.x == 0) {
        const int s = plus ? 1 : (minus ? -1 : 0);
        sym[mbmax + mb] = s;
        sym[mbmax - mb] = s;
    }
}

}  // namespace

// Built tile variants.  Forward and adjoint: R in {2, 4, 8}, TB in {32, 64}, TR = 4.
// Polarised forward (op 3): R in {2, 4}, TB in {32, 64}.  Wigner: R in {1, 4}, TB = 32.
bool tile_supported(int op, Tile t)
{
    if (t.NT != 256) return false;
    if (op == 0) return (t.R == 1 || t.R == 4) && t.TB == 32;
    const bool r_ok = t.R == 2 || t.R == 4 || t.R == 8;
    const bool tb_ok = t.TB == 32 || t.TB == 64;
    if (op == 1) return r_ok && tb_ok;
    if (op == 2) return r_ok && tb_ok && t.TR == 4;
    if (op == 3) return (t.R == 2 || t.R == 4) && tb_ok;
    return false;
}

int launch_wigner(const WignerArgs& a, Tile t, void* stream)
{
    const int blocks = a.npair * a.ntile;
    switch (t.R) {
    case 1: return launch_grid(k_wigner<1, 256, 32>, a, blocks, 256, stream);
    case 4: return launch_grid(k_wigner<4, 256, 32>, a, blocks, 256, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

// Maps a runtime (R, TB[, TR]) onto the template instantiation F<R, TB[, TR]>.
#define TC_FWD_VARIANTS(X) X(2, 32) X(4, 32) X(8, 32) X(2, 64) X(4, 64) X(8, 64)
#define TC_FWDPOL_VARIANTS(X)                                                                   \
    X(2, 32, 1, 2) X(4, 32, 1, 2) X(2, 64, 1, 2) X(4, 64, 1, 2) X(2, 32, 1, 3) X(4, 32, 1, 3)  \
    X(2, 64, 1, 3) X(4, 64, 1, 3) X(2, 32, 2, 2) X(4, 32, 2, 2) X(2, 64, 2, 2) X(4, 64, 2, 2)  \
    X(2, 32, 3, 3) X(4, 32, 3, 3) X(2, 64, 3, 3) X(4, 64, 3, 3)
#define TC_ADJ_VARIANTS(X) X(2, 32, 4) X(4, 32, 4) X(8, 32, 4) X(2, 64, 4) X(4, 64, 4) X(8, 64, 4)

int launch_beam_symmetry(const double* blm, int lmax, int mbmax, int* sym, void* stream)
{
    hipLaunchKernelGGL(k_beam_symmetry, dim3(mbmax + 1), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const double2*>(blm), lmax, mbmax, sym);
    return (int)hipGetLastError();
}

int launch_fwd(const FwdArgs& a, Tile t, void* stream)
{
    const int blocks = a.ncol * a.ntile;
    if (a.npair == 1) {
#define X(r, tb)                                                                              \
    if (t.R == r && t.TB == tb) {                                                             \
        if (a.beam_sym[0]) {                                                                  \
            const int rc = launch_grid(k_fwd_rows<r, 256, tb>, a, blocks, 256, stream);       \
            if (rc) return rc;                                                                \
        }                                                                                     \
        return launch_grid(k_fwd<r, 256, tb, 1, 1>, a, blocks, 256, stream);                  \
    }
        TC_FWD_VARIANTS(X)
#undef X
        return (int)hipErrorInvalidValue;
    }
    const int nc = a.sum ? 1 : a.npair;
#define X(r, tb, c, p)                                                        \
    if (t.R == r && t.TB == tb && nc == c && a.npair == p)                    \
        return launch_grid(k_fwd<r, 256, tb, c, p>, a, blocks, 256, stream);
    TC_FWDPOL_VARIANTS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int launch_adj(const AdjArgs& a, Tile t, void* stream)
{
    const int blocks = a.ncol;   // every ring tile of a column in one workgroup
#define X(r, tb, tr) \
    if (t.R == r && t.TB == tb && t.TR == tr) return launch_grid(k_adj<r, 256, tb, tr>, a, blocks, 256, stream);
    TC_ADJ_VARIANTS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int launch_adj_epilogue(const EpiArgs& e, void* stream)
{
    const int nt = 256;
    if (e.alm_bar) {
        dim3 grid((e.sky_lmax + 1 + nt - 1) / nt, e.sky_lmax + 1);
        hipLaunchKernelGGL(k_adj_sky, grid, dim3(nt), 0, (hipStream_t)stream, e);
        const int rc = (int)hipGetLastError();
        if (rc) return rc;
    }
    if (e.blm_bar) return launch_adj_beam(e, stream);
    return 0;
}

int launch_adj_beam(const EpiArgs& e, void* stream)
{
    const int nt = 256;
    dim3 grid((e.lmax + 1 + nt - 1) / nt, 2 * e.mbmax + 1);
    hipLaunchKernelGGL(k_adj_beam, grid, dim3(nt), 0, (hipStream_t)stream, e);
    return (int)hipGetLastError();
}

int launch_fwd_items(const FwdArgs* walks, const int* items, int nitems, Tile t, void* stream)
{
    if (nitems <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
#define X(r, tb)                                                                                             \
    if (t.R == r && t.TB == tb) {                                                                            \
        hipLaunchKernelGGL((k_fwd_items<r, 256, tb>), dim3(nitems), dim3(256), 0, s, walks, items);            \
        return (int)hipGetLastError();                                                                       \
    }
    TC_FWD_VARIANTS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int fwd_walk_pairs(Tile t) { return t.R >= 8 ? walk_pairs<8>() : walk_pairs<4>(); }

int adj_walk_pairs_of(Tile t)
{
    if (t.TB > 32) return adj_walk_pairs<4, 64>();
    return t.R >= 8 ? adj_walk_pairs<8, 32>() : adj_walk_pairs<4, 32>();
}

int launch_adj_items(const AdjArgs* dets, const int* items, int nitems, Tile t, void* stream)
{
    if (nitems <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
#define X(r, tb, tr)                                                                                        \
    if (t.R == r && t.TB == tb && t.TR == tr) {                                                             \
        hipLaunchKernelGGL((k_adj_items<r, 256, tb, tr>), dim3(nitems), dim3(256), 0, s, dets, items);      \
        return (int)hipGetLastError();                                                                      \
    }
    TC_ADJ_VARIANTS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int launch_adj_sky_multi(const EpiArgs* eps, int ndet, int sky_lmax, bool accumulate, double* alm_bar, void* stream)
{
    const int nt = 256;
    dim3 grid((sky_lmax + 1 + nt - 1) / nt, sky_lmax + 1);
    hipLaunchKernelGGL(k_adj_sky_multi, grid, dim3(nt), 0, (hipStream_t)stream, eps, ndet, sky_lmax,
                       accumulate ? 1 : 0, alm_bar);
    return (int)hipGetLastError();
}

}  // namespace tc
