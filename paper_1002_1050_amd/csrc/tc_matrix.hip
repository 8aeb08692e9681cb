// gfx950 kernel of the full reduced Wigner matrix at one l (Sec. 3.1): every
// d^l_{m m'}(beta_j), -l <= m, m' <= l, for a set of rings.
//
// Sec. 3.1 walks a row of fixed l and m in m' with the three-term relation of
// Sec. 2 (eq. mrec), as ratios anchored at d^l_{00}.  Here the same relation runs
// on the values, downwards from the closed-form end point d^l_{m,l} = A c^{l+m}
// s^{l-m} (the seed of Sec. 3.2, as a logarithm, with exact power-of-two scaling
// while the values are tiny), on the triangle 0 <= m <= m' <= l only, where the
// wanted solution grows or oscillates in the direction of the walk:
//
//   d_{m,m'-1} = [2 (m' cot(beta) - m csc(beta)) d_{m,m'} - b_{m'} d_{m,m'+1}] / a_{m'},
//   a_{m'} = sqrt((l+m')(l-m'+1)),  b_{m'} = sqrt((l-m')(l+m'+1)).
//
// The rest of the matrix follows from the symmetries of the appendix:
//   d_{m',m} = (-1)^(m-m') d_{m,m'},  d_{-m,-m'} = (-1)^(m-m') d_{m,m'},
//   d_{m,-m'}(beta) = (-1)^(l+m) d_{m,m'}(pi - beta),
// so a workgroup walks the triangle at beta (side 0) or at pi - beta (side 1, rows
// m >= 1, whose images are the quadrants with m m' < 0) and writes each value to
// its images.  One lane owns R rows m of one ring; per-step coefficients depend on
// the ring and m' only and are staged in LDS.

#include <hip/hip_runtime.h>

#include "tc_internal.h"

namespace tc {
namespace {

constexpr int MS_TS = 8;          // steps between scale checks
constexpr int MS_FOLD = -900;     // scaled values fold into plain doubles at 2^-900

__device__ __forceinline__ bool wave_any_m(bool p) { return __ballot(p) != 0ull; }

__device__ __forceinline__ void two_sum_m(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (sh, sl) += n * (ah + al), n an integer held exactly in a double
__device__ __forceinline__ void dd_add_times_m(double& sh, double& sl, double n, double ah, double al)
{
    const double ph = n * ah;
    const double pl = fma(n, ah, -ph) + n * al;
    double s, e;
    two_sum_m(sh, ph, s, e);
    e += sl + pl;
    sh = s + e;
    sl = e - (sh - s);
}

// d^l_{m,l} = A c^p s^q (p = l+m, q = l-m, c, s > 0 here) as a significand in
// [1, 2) times 2^E (E < 0), or a plain double (E = 0) once >= 2^-900.
__device__ __forceinline__ void row_seed(double lnAh, double lnAl, int p, int q, double lch, double lcl,
                                         double lsh, double lsl, double& d, int& E)
{
    double h = lnAh, lo = lnAl;
    if (p > 0) dd_add_times_m(h, lo, (double)p, lch, lcl);
    if (q > 0) dd_add_times_m(h, lo, (double)q, lsh, lsl);
    // ln -> log2 in double-double
    const double L2h = 0x1.71547652b82fep+0, L2l = 0x1.777d0ffda0d24p-56;
    const double ph = h * L2h;
    const double pe = fma(h, L2h, -ph) + (h * L2l + lo * L2h);
    const double yh = ph + pe, yl = pe - (yh - ph);
    const double k = floor(yh);
    const double m = exp2((yh - k) + yl);
    const int ik = (int)k;
    if (ik >= MS_FOLD) { d = ldexp(m, ik); E = 0; }
    else { d = m; E = ik; }
}

// The four images of the walked element (m, mp) (mp >= m >= 0).  Side 0: v =
// d_{m,mp}(beta) goes to (m, mp), (mp, m), (-m, -mp), (-mp, -m) with signs 1, s, s, 1
// (s = (-1)^(m-mp)).  Side 1: u = (-1)^(l+m) v with v = d_{m,mp}(pi - beta) is
// d_{m,-mp}(beta) and goes to (m, -mp), (-mp, m), (-m, mp), (mp, -m), signs 1, s, s, 1.
// Images 1 and 3 run along a row as the lanes' m run (stored at once, coalesced);
// images 0 and 2 run along a row as mp runs, so they are gathered in LDS for FL
// steps and stored row by row (FL doubles per row segment).

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// element offset of image k of (m, mp) within one ring's (2l+1)^2 matrix
__device__ __forceinline__ unsigned image_off(int side, int k, int l, int W, int m, int mp)
{
    int row, col;
    if (side == 0) {
        row = k == 0 ? m : k == 1 ? mp : k == 2 ? -m : -mp;
        col = k == 0 ? mp : k == 1 ? m : k == 2 ? -mp : -m;
    } else {
        row = k == 0 ? m : k == 1 ? -mp : k == 2 ? -m : mp;
        col = k == 0 ? -mp : k == 1 ? m : k == 2 ? mp : -m;
    }
    return (unsigned)((row + l) * W + (col + l));
}

// Sync of the held values before and after a flush: within the wave for one-wave workgroups,
// a workgroup barrier otherwise.
template <int NT>
__device__ __forceinline__ void held_sync()
{
    if constexpr (NT == 64) wave_lds_fence();
    else __syncthreads();
}

template <int R, int NT, int TB, int FL>
__global__ void __launch_bounds__(NT) k_wigner_row(const MatrixArgs a)
{
    static_assert(NT % 64 == 0, "whole waves");
    static_assert(TB % FL == 0 && FL % MS_TS == 0 && (NT % FL == 0 || FL % NT == 0), "flush period");
    constexpr int LPR = FL < NT ? FL : NT;    // lanes per row segment in a flush
    constexpr int RPS = NT / LPR;             // rows per flush store
    __shared__ double4 cf[2][TB];             // per step: {A, nB, F2, -}: d_next = (m A + nB) d - F2 d_prev
    __shared__ double held[R][FL][NT + 1];    // values u of the last FL steps, per row
    const int tid = threadIdx.x;
    const int per_tile = 2 * a.nring;
    const int tile = blockIdx.x / per_tile;
    const int rem = blockIdx.x - tile * per_tile;
    const int j = rem >> 1, side = rem & 1;
    const int l = a.l;
    const int W = 2 * l + 1;
    double* __restrict__ out = a.d + (size_t)j * (size_t)W * (size_t)W;
    const double x = a.ring.x[j];
    const int m_base = tile * NT * R;
    const int m_lo = max(m_base, side);       // lowest row of the workgroup
    if (m_lo > l) return;

    int mrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = m_base + r * NT + tid;
        mrow[r] = (m <= l && m >= side) ? m : -1;
    }
    const bool pole = (x == 1.0 || x == -1.0);
    const bool ident = (side == 0) == (x == 1.0);   // at a pole: the walked triangle is at beta = 0

    double cot = 0.0, csc = 0.0, lch = 0.0, lcl = 0.0, lsh = 0.0, lsl = 0.0;
    if (!pole) {
        cot = side ? -a.trig[2 * j] : a.trig[2 * j];
        csc = a.trig[2 * j + 1];
        // c' = cos((pi - beta)/2) = sin(beta/2) on side 1
        lch = side ? a.ring.lsh[j] : a.ring.lch[j]; lcl = side ? a.ring.lsl[j] : a.ring.lcl[j];
        lsh = side ? a.ring.lch[j] : a.ring.lsh[j]; lsl = side ? a.ring.lcl[j] : a.ring.lsl[j];
    }
    double xm[R], d[R], dp[R], rs[R], s_r[R];
    int E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = mrow[r] < 0 ? 0 : mrow[r];
        xm[r] = (double)m;
        d[r] = 0.0; dp[r] = 0.0; E[r] = 0;
        if (!pole) row_seed(a.lnA[2 * m], a.lnA[2 * m + 1], l + m, l - m, lch, lcl, lsh, lsl, d[r], E[r]);
        rs[r] = (side == 1 && ((l + m) & 1)) ? -1.0 : 1.0;   // side 1 carries (-1)^(l+m)
        s_r[r] = ((m - l) & 1) ? -1.0 : 1.0;                  // (-1)^(m-mp) at mp = l
    }
    bool scaled = false;
#pragma unroll
    for (int r = 0; r < R; ++r) scaled |= (E[r] < 0);
    scaled = wave_any_m(scaled);

    // step s: from m' = l - s to m' - 1; steps needed: l - m_lo
    const int nsteps = l - m_lo;
    // Steps s <= full have m' = l - s >= every row of the workgroup; a group of MS_TS steps all
    // within them (and all followed by a step of the walk) takes the fast path below: no
    // per-step checks, the coefficients of the group read together, the two images along m'
    // through pointers moved by one output row per step (inc1 = +-W elements).
    const int m_hi = min(l, m_base + NT * R - 1);
    const int fast_last = pole ? -1 : min(nsteps - 1, l - m_hi);
    const long long inc1 = side ? (long long)W : -(long long)W;
    for (int t = tid; t < TB; t += NT) {
        const int mp = l - t;
        double4 c = make_double4(0.0, 0.0, 0.0, 0.0);
        if (!pole && t < nsteps) {
            const double av = sqrt((double)(l + mp) * (double)(l - mp + 1));
            const double bv = sqrt((double)(l - mp) * (double)(l + mp + 1));
            c = make_double4(-2.0 * csc / av, 2.0 * (double)mp * cot / av, bv / av, 0.0);
        }
        cf[0][t] = c;
    }
    __syncthreads();
    for (int s0 = 0, kb = 0; s0 <= nsteps; s0 += TB, ++kb) {
        const int buf = kb & 1;
        for (int t0 = 0; t0 < TB && s0 + t0 <= nsteps; t0 += MS_TS) {
            if (scaled) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // exact power-of-two rescale; fold into plain doubles at 2^-900
                    int e1, e2;
                    frexp(d[r], &e1);
                    frexp(dp[r], &e2);
                    const bool nz = (d[r] != 0.0) | (dp[r] != 0.0);
                    const int e = max(d[r] != 0.0 ? e1 : -(1 << 20), dp[r] != 0.0 ? e2 : -(1 << 20));
                    const bool sc = nz & (E[r] < 0);
                    const bool fold = (E[r] + e) >= MS_FOLD;
                    const int k = sc ? (fold ? E[r] : -e) : 0;
                    E[r] = sc ? (fold ? 0 : E[r] + e) : E[r];
                    d[r] = ldexp(d[r], k);
                    dp[r] = ldexp(dp[r], k);
                    any |= (E[r] < 0);
                }
                scaled = wave_any_m(any);
            }
            const int sg = s0 + t0;
            if (sg + MS_TS - 1 <= fast_last) {
                double4 kk[MS_TS];
#pragma unroll
                for (int t = 0; t < MS_TS; ++t) kk[t] = cf[buf][t0 + t];
                double* p1[R];
                double* p3[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int m = mrow[r] < 0 ? side : mrow[r];   // lanes without a row store nothing
                    p1[r] = out + image_off(side, 1, l, W, m, l - sg);
                    p3[r] = out + image_off(side, 3, l, W, m, l - sg);
                }
#pragma unroll
                for (int t = 0; t < MS_TS; ++t) {
                    const int h = (t0 + t) % FL;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double v = E[r] == 0 ? d[r] : ldexp(d[r], E[r]);
                        const double u = rs[r] * v;
                        held[r][h][tid] = u;
                        if (mrow[r] >= 0) {
                            p1[r][t * inc1] = s_r[r] * u;
                            p3[r][-t * inc1] = u;
                        }
                        s_r[r] = -s_r[r];
                        const double w = fma(xm[r], kk[t].x, kk[t].y);
                        const double dn = fma(-kk[t].z, dp[r], w * d[r]);
                        dp[r] = d[r];
                        d[r] = dn;
                    }
                }
            } else {
#pragma unroll
            for (int t = 0; t < MS_TS; ++t) {
                const int s = s0 + t0 + t;
                if (s > nsteps) break;
                const int mp = l - s;
                const int h = (t0 + t) % FL;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int m = mrow[r];
                    double v;
                    if (pole) v = ident ? (mp == m ? 1.0 : 0.0) : ((m == 0 && mp == 0) ? ((l & 1) ? -1.0 : 1.0) : 0.0);
                    else v = E[r] == 0 ? d[r] : ldexp(d[r], E[r]);
                    const double u = rs[r] * v;
                    held[r][h][tid] = u;
                    if (m >= 0 && mp >= m) {
                        out[image_off(side, 1, l, W, m, mp)] = s_r[r] * u;
                        out[image_off(side, 3, l, W, m, mp)] = u;
                    }
                    s_r[r] = -s_r[r];
                }
                if (s < nsteps && !pole) {
                    const double4 k = cf[buf][t0 + t];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double u = fma(xm[r], k.x, k.y);
                        const double dn = fma(-k.z, dp[r], u * d[r]);
                        dp[r] = d[r];
                        d[r] = dn;
                    }
                }
            }
            }
            // images 0 and 2 of the held steps, after every FL steps and after the last:
            // FL lanes per row, NT / FL rows per store
            const int done = s0 + t0 + MS_TS;
            if ((t0 + MS_TS) % FL == 0 || done > nsteps) {
                const int sb = s0 + ((t0 + MS_TS - 1) / FL) * FL;
                const int n = min(FL, nsteps + 1 - sb);
                held_sync<NT>();
                if (n == FL && sb + FL - 1 <= fast_last) {
                    // every held step has m' >= every row: per lane one m' (tq), rows q stepped by RPS,
                    // image 0 one output row further per RPS rows, image 2 one row back
                    const int q0 = tid / LPR;
                    const long long rstep = (long long)RPS * W;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
#pragma unroll
                        for (int c = 0; c < FL; c += LPR) {
                            const int tq = c + tid % LPR;
                            const int mpf = l - (sb + tq);
                            const int m0 = m_base + r * NT + q0;
                            double* p0 = out + image_off(side, 0, l, W, m0, mpf);
                            double* p2 = out + image_off(side, 2, l, W, m0, mpf);
                            bool odd = ((m0 - mpf) & 1) != 0;
                            for (int q = q0, k = 0; q < NT; q += RPS, ++k) {
                                const int m = m0 + (q - q0);
                                const double u = held[r][tq][q];
                                if (m >= side && m <= l) {
                                    p0[k * rstep] = u;
                                    p2[-k * rstep] = odd ? -u : u;
                                }
                                odd = (RPS & 1) ? !odd : odd;
                            }
                        }
                    }
                } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    for (int q = tid / LPR; q < NT; q += RPS) {
                        const int m = m_base + r * NT + q;
#pragma unroll
                        for (int c = 0; c < FL; c += LPR) {
                            const int tq = c + tid % LPR;
                            const int mpf = l - (sb + tq);
                            if (tq < n && m <= l && m >= side && mpf >= m) {
                                const double u = held[r][tq][q];
                                out[image_off(side, 0, l, W, m, mpf)] = u;
                                out[image_off(side, 2, l, W, m, mpf)] = ((m - mpf) & 1) ? -u : u;
                            }
                        }
                    }
                }
                }
                held_sync<NT>();
            }
        }
        if (s0 + TB <= nsteps) {
            for (int t = tid; t < TB; t += NT) {
                const int mp = l - (s0 + TB + t);
                double4 c = make_double4(0.0, 0.0, 0.0, 0.0);
                if (!pole && s0 + TB + t < nsteps) {
                    const double av = sqrt((double)(l + mp) * (double)(l - mp + 1));
                    const double bv = sqrt((double)(l - mp) * (double)(l + mp + 1));
                    c = make_double4(-2.0 * csc / av, 2.0 * (double)mp * cot / av, bv / av, 0.0);
                }
                cf[buf ^ 1][t] = c;
            }
        }
        __syncthreads();
    }
}

}  // namespace

// Built variants (id: R rows per lane, NT lanes, TB-step coefficient blocks, FL-step flushes).
// Id 0, the built-in: two-wave workgroups of 128 rows flushing every 128 steps, so that both
// image streams leave in 1 KB row segments (scattered 512-byte segments reach about two thirds
// of the write bandwidth of 1 KB ones on MI355X); the LDS of the flush buffer (133 KB) allows
// one workgroup per CU.  Ids 1 and 2: one-wave workgroups, 512-byte segments, R = 1 or 2.
#define TC_MATRIX_VARIANTS(X) X(0, 1, 128, 128, 128) X(1, 1, 64, 64, 64) X(2, 2, 64, 64, 64)

int matrix_rows_per_group(int v)
{
#define X(id, r, nt, tb, fl) if (v == id) return r * nt;
    TC_MATRIX_VARIANTS(X)
#undef X
    return 0;
}

int launch_matrix(const MatrixArgs& a, int v, void* stream)
{
    const int blocks = a.ntile * 2 * a.nring;
#define X(id, r, nt, tb, fl)                                                                                     \
    if (v == id) {                                                                                               \
        hipLaunchKernelGGL((k_wigner_row<r, nt, tb, fl>), dim3(blocks), dim3(nt), 0, (hipStream_t)stream, a);   \
        return (int)hipGetLastError();                                                                           \
    }
    TC_MATRIX_VARIANTS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

}  // namespace tc
