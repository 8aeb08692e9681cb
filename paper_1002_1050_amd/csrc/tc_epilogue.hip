// Sky gradients of several (sky, beam) pairs that share one cotangent, and so one set of
// per-column sums U, V: the polarised adjoint with summed outputs (the pairs' outputs add into
// one C, footnote of Sec. 4.1).  One launch reads U and V once for all pairs, where one launch
// per pair would read them once per pair.  Every pair's sums take the operations of the one-pair
// sky epilogue (k_adj_sky) in the same order, so each sky gradient equals, bit for bit, the one a
// scalar adjoint of the same cotangent returns for that pair.  (The beam gradients keep one
// launch per pair: a kernel that summed all three pairs' beam gradients in one pass over U, V
// ran 6.8 ms at lmax 4096, against 3 x 2.1 ms for one launch per pair.)
//
// u(mb, ms, l) = U[mb] + (-1)^(l-ms) V[-mb] at packed index (ms, l), defined for
// l >= max(|mb|, ms);  alm_bar_p{l,ms} = sum_mb b_p{l,mb} u(mb, ms, l), mb ascending.
#include <hip/hip_runtime.h>

#include "tc_internal.h"

namespace tc {
namespace {

// Global loads and stores of complex values through pointers held in the argument record, as
// native vectors in the global address space (the generic form would take flat instructions).
typedef double native_double2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld2(const double* base, size_t k)
{
    const native_double2 v = *(const __attribute__((address_space(1))) native_double2*)(base + 2 * k);
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ void st2(double* base, size_t k, double x, double y)
{
    native_double2 w;
    w.x = x;
    w.y = y;
    *(__attribute__((address_space(1))) native_double2*)(base + 2 * k) = w;
}

// Position of (l, m) in an array packed m-major for l = m .. lmax.
__device__ __forceinline__ size_t packed(int lmax, int l, int m)
{
    return (size_t)m * (size_t)(2 * lmax + 1 - m) / 2 + (size_t)l;
}

constexpr int ROWS = 8;   // beam rows whose U, V values a thread loads before using any

template <int NP>
__global__ void __launch_bounds__(256) k_adj_sky_pairs(const EpiPairsArgs e)
{
    const int ms = blockIdx.y;
    const int l = ms + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > e.sky_lmax) return;
    double ar[NP], ai[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) { ar[p] = 0.0; ai[p] = 0.0; }
    if (l <= e.lmax) {
        const size_t k = packed(e.lmax, l, ms);
        const int M = e.mbmax, lo = max(-M, -l), hi = min(M, l);   // rows with l >= |mb|
        const double sg = ((l - ms) & 1) ? -1.0 : 1.0;
        for (int mb0 = lo; mb0 <= hi; mb0 += ROWS) {
            double2 ua[ROWS], va[ROWS];
#pragma unroll
            for (int q = 0; q < ROWS; ++q) {
                const int mb = min(mb0 + q, hi);   // past the last row: a repeat of it, not added
                ua[q] = ld2(e.U, (size_t)(mb + M) * e.P + k);
                va[q] = ld2(e.V, (size_t)(-mb + M) * e.P + k);
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                double2 ba[ROWS];
#pragma unroll
                for (int q = 0; q < ROWS; ++q)
                    ba[q] = ld2(e.blm[p], (size_t)(min(mb0 + q, hi) + M) * (e.lmax + 1) + l);
#pragma unroll
                for (int q = 0; q < ROWS; ++q) {
                    if (mb0 + q <= hi) {
                        const double2 u = make_double2(ua[q].x + sg * va[q].x, ua[q].y + sg * va[q].y);
                        const double2 b = ba[q];
                        ar[p] += b.x * u.x - b.y * u.y;
                        ai[p] += b.x * u.y + b.y * u.x;
                    }
                }
            }
        }
    }
    const size_t o = packed(e.sky_lmax, l, ms);
#pragma unroll
    for (int p = 0; p < NP; ++p)
        if (e.alm_bar[p]) st2(e.alm_bar[p], o, ar[p], ai[p]);
}

template <int NP>
int launch_pairs(const EpiPairsArgs& e, void* stream)
{
    const int nt = 256;
    const dim3 grid((e.sky_lmax + 1 + nt - 1) / nt, e.sky_lmax + 1);
    hipLaunchKernelGGL(k_adj_sky_pairs<NP>, grid, dim3(nt), 0, (hipStream_t)stream, e);
    return (int)hipGetLastError();
}

}  // namespace

int launch_adj_sky_pairs(const EpiPairsArgs& e, void* stream)
{
    switch (e.npair) {
    case 2: return launch_pairs<2>(e, stream);
    case 3: return launch_pairs<3>(e, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace tc
