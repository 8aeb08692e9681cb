// gfx950 kernels of the data-cube stage (Sec. 4.1, eq. conviqt):
//
//   c(alpha_a, beta_j, gamma_g) = sum_{mb=-M}^{M} sum_{msky=-L}^{L}
//                                 e^{-i mb alpha_a} e^{-i msky gamma_g} C_{mb,msky}(beta_j)
//
// on alpha_a = 2 pi a / nalpha, gamma_g = 2 pi g / ngamma, with the columns msky < 0
// taken from C_{-mb,-msky} = conj(C_{mb,msky}) (real sky and beam, Sec. 4.2.3), so
// that c is real.
//
// Two passes, both bound by HBM bandwidth (the host runs them over ring chunks, the alpha pass of
// one chunk beside the gamma pass of the chunk before):
//  1. k_cube_alpha: P[j][a][k] = sum_mb E[mb][a] C[mb][k][j] for k = msky >= 0 -- the
//     short sum over mb, done directly with the host's phase table E (read into scalar
//     registers, four phases per load), and the
//     transpose from ring-fastest C to rows (ring, alpha) with msky fastest.
//  2. k_cube_gamma: one workgroup per row turns P_0..P_L into the real row
//     c[g] = Re P_0 + 2 Re sum_{k>=1} P_k e^{-2 pi i k g / N}: the Hermitian
//     spectrum is folded into its half X_0..X_{N/2}, packed into one complex
//     sequence of length H = N/2 (even outputs in the real part, odd outputs in the
//     imaginary part) and transformed by a Stockham FFT in LDS (radix-16 passes and
//     one smaller one), twiddles from the host's table W^m = e^{-2 pi i m / N}.

#include <hip/hip_runtime.h>

#include "tc_internal.h"

namespace tc {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Streaming store of a cube element (written once, read by no later pass here).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream(double2* p, double2 v)
{
    nt_d2 w;
    w.x = v.x; w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<nt_d2*>(p));
}

// ------------------------------------------------------------ alpha sums
constexpr int CA_T = 16;    // rings and msky values per workgroup tile (16 x 16 = 256 lanes)
constexpr int CA_Q = 8;     // alpha values per transposed store

// Each lane owns one (msky, ring) element and sums its 2M+1 values of C against the
// phases of QA values of alpha.  The C values are loaded CA_U at a time (all in flight
// together).  The phase table [mb][alpha] (alpha padded to a multiple of 4) is read with
// uniform 64-byte loads, four phases at a time, so the phases arrive in scalar registers
// and every C value feeds 4 QA fused multiply-adds without LDS traffic.
constexpr int CA_U = 8;

struct alignas(64) Phase4 {
    double2 v[4];
};

template <int QA>
__global__ void __launch_bounds__(256) k_cube_alpha(const CubeArgs c, const double2* __restrict__ C,
                                                    const Phase4* __restrict__ E4, double2* __restrict__ P)
{
    static_assert(QA % 4 == 0, "phases come in fours");
    __shared__ double2 tile[CA_Q][CA_T][CA_T + 1];
    const int nb = 2 * c.mbmax + 1;
    const int na4 = (c.nalpha + 3) / 4;     // Phase4 entries per mb row
    const int tid = threadIdx.x;
    const int jj = tid & (CA_T - 1), kk = tid / CA_T;
    const int j0 = blockIdx.x * CA_T, k0 = blockIdx.y * CA_T;
    const int j = j0 + jj, k = k0 + kk;
    const int L1 = c.lmax + 1;
    const bool in = (j < c.nring_chunk) && (k <= c.lmax);
    const size_t mb_stride = (size_t)L1 * c.nring;
    for (int a0 = 0; a0 < c.nalpha; a0 += QA) {
        double ar[QA], ai[QA];
#pragma unroll
        for (int q = 0; q < QA; ++q) { ar[q] = 0.0; ai[q] = 0.0; }
        if (in) {
            const double2* src = C + (size_t)k * c.nring + (c.ring0 + j);
            for (int mb0 = 0; mb0 < nb; mb0 += CA_U) {
                double2 v[CA_U];
#pragma unroll
                for (int u = 0; u < CA_U; ++u)
                    v[u] = (mb0 + u < nb) ? src[(size_t)(mb0 + u) * mb_stride] : make_double2(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < CA_U; ++u) {
                    if (mb0 + u < nb) {
                        const Phase4* row = E4 + (size_t)(mb0 + u) * na4 + a0 / 4;
#pragma unroll
                        for (int q4 = 0; q4 < QA / 4; ++q4) {
                            if (a0 + 4 * q4 < c.nalpha) {
                                const Phase4 e = row[q4];
#pragma unroll
                                for (int i = 0; i < 4; ++i) {
                                    const int q = 4 * q4 + i;
                                    ar[q] = fma(e.v[i].x, v[u].x, fma(-e.v[i].y, v[u].y, ar[q]));
                                    ai[q] = fma(e.v[i].x, v[u].y, fma(e.v[i].y, v[u].x, ai[q]));
                                }
                            }
                        }
                    }
                }
            }
        }
        // transposed stores, CA_Q values of alpha at a time: lanes with consecutive msky
#pragma unroll
        for (int q0 = 0; q0 < QA; q0 += CA_Q) {
            if (a0 + q0 >= c.nalpha) break;
#pragma unroll
            for (int q = 0; q < CA_Q; ++q) tile[q][kk][jj] = make_double2(ar[q0 + q], ai[q0 + q]);
            __syncthreads();
            const int jw = tid / CA_T, kw = tid & (CA_T - 1);
            if (j0 + jw < c.nring_chunk && k0 + kw <= c.lmax) {
                for (int q = 0; q < CA_Q && a0 + q0 + q < c.nalpha; ++q)
                    P[((size_t)(j0 + jw) * c.nalpha + (a0 + q0 + q)) * L1 + (k0 + kw)] = tile[q][kw][jw];
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------ gamma FFT
// Forward DFT of size R (sign -) in registers: bit-reversed reorder, then radix-2
// stages with the 16th roots of unity as constants.
__device__ __forceinline__ double2 root16(int m, double2 z)
{
    // z * e^{-2 pi i m / 16}, m in [0, 8)
    constexpr double C1 = 0.9238795325112867;   // cos(pi/8)
    constexpr double S1 = 0.3826834323650898;   // sin(pi/8)
    constexpr double H2 = 0.7071067811865476;   // cos(pi/4)
    switch (m) {
    case 0: return z;
    case 4: return make_double2(z.y, -z.x);
    case 1: return cmul(z, make_double2(C1, -S1));
    case 2: return cmul(z, make_double2(H2, -H2));
    case 3: return cmul(z, make_double2(S1, -C1));
    case 5: return cmul(z, make_double2(-S1, -C1));
    case 6: return cmul(z, make_double2(-H2, -H2));
    default: return cmul(z, make_double2(-C1, -S1));
    }
}

template <int R>
__device__ __forceinline__ void dft_regs(double2 (&v)[R])
{
    constexpr int LOG = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < LOG; ++b) r |= ((i >> b) & 1) << (LOG - 1 - b);
        if (i < r) {
            const double2 t = v[i];
            v[i] = v[r];
            v[r] = t;
        }
    }
#pragma unroll
    for (int half = 1; half < R; half <<= 1) {
#pragma unroll
        for (int b = 0; b < R; b += 2 * half) {
#pragma unroll
            for (int q = 0; q < half; ++q) {
                const double2 t = root16(q * (8 / half), v[b + q + half]);
                v[b + q + half] = csub(v[b + q], t);
                v[b + q] = cadd(v[b + q], t);
            }
        }
    }
}

constexpr int CG_HMAX = 8192;   // largest half length (ngamma <= 16384)

// LDS slot of element i: one pad slot per 16 elements, so that the first pass's
// stride-16 stores (and every other pass's accesses) spread over the banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Twiddles w_r = W^{r m1} for r < R from W^{m1}, W^{2 m1}, W^{4 m1}, W^{8 m1} of the
// host table: every w_r is a table entry or a product of at most three of them.
template <int R>
__device__ __forceinline__ void twiddle_base(const double2* __restrict__ tw, int m1, double2 (&b)[4])
{
    b[0] = tw[m1];
    if (R > 2) b[1] = tw[2 * m1];
    if (R > 4) b[2] = tw[4 * m1];
    if (R > 8) b[3] = tw[8 * m1];
}

template <int R>
__device__ __forceinline__ void apply_twiddles(double2 (&v)[R], const double2 (&b)[4])
{
    double2 w[R];
    w[1] = b[0];
    if (R > 2) { w[2] = b[1]; w[3] = cmul(b[0], b[1]); }
    if (R > 4) {
        w[4] = b[2];
#pragma unroll
        for (int r = 5; r < 8; ++r) w[r] = cmul(b[2], w[r - 4]);
    }
    if (R > 8) {
        w[8] = b[3];
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(b[3], w[r - 8]);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
}

// Entry b in [0, H] of the half spectrum: X_b = Z_b + Z_{b-N} with Z_0 = Re P_0,
// Z_k = P_k and Z_{-k} = conj(P_k) for 1 <= k <= L (zero beyond L).
__device__ __forceinline__ double2 half_spec(const double2* __restrict__ P, int b, int N, int L)
{
    double2 z = make_double2(0.0, 0.0);
    if (b == 0) z = make_double2(P[0].x, 0.0);
    else if (b <= L) z = P[b];
    if (b > 0 && N - b <= L) z = cadd(z, cconj(P[N - b]));
    return z;
}

// Packed input of the half-length transform: F_k = (X_k + conj X_{H-k}) + i W^k (X_k - conj X_{H-k}).
__device__ __forceinline__ double2 packed(double2 a, double2 b, double2 w)
{
    const double2 s = cadd(a, cconj(b)), d = cmul(w, csub(a, cconj(b)));
    return make_double2(s.x - d.y, s.y + d.x);
}

// First Stockham pass (stride Ns = 1, unit twiddles), fed straight from HBM: lane g
// forms F_{g + r H/R} for r < R from the row of P and transforms them in registers.
// All of a lane's loads are issued before the first is used.  The result goes to LDS,
// or, when this is the only pass, to the output row.
template <int R, int HMAX>
__device__ __forceinline__ void first_pass(const double2* __restrict__ P, const double2* __restrict__ tw,
                                           int H, int N, int L, double2* X, double2* out, bool last)
{
    constexpr int GM = HMAX / (R * 256) > 0 ? HMAX / (R * 256) : 1;
    const int tid = threadIdx.x;
    const int ng = H / R;
    double2 v[GM][R];
#pragma unroll
    for (int i = 0; i < GM; ++i) {
        const int g = tid + 256 * i;
        if (g < ng) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = g + r * ng;
                v[i][r] = packed(half_spec(P, k, N, L), half_spec(P, H - k, N, L), tw[k]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < GM; ++i) {
        const int g = tid + 256 * i;
        if (g < ng) {
            dft_regs<R>(v[i]);
            if (last) {
#pragma unroll
                for (int r = 0; r < R; ++r) store_stream(out + g * R + r, v[i][r]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) X[pad(g * R + r)] = v[i][r];
            }
        }
    }
    if (!last) __syncthreads();
}

// One later Stockham pass of radix R over X[0..H) in place (all reads, barrier, all
// writes, barrier); HMAX bounds H, hence the groups a lane handles.  The last pass
// (Ns = H / R, so each lane's outputs g + r Ns are contiguous across lanes) writes
// the output row instead.
template <int R, int HMAX, bool LAST>
__device__ __forceinline__ void stockham_pass(double2* X, int H, int Ns, int N, const double2* __restrict__ tw,
                                              double2* __restrict__ out)
{
    constexpr int GM = HMAX / (R * 256) > 0 ? HMAX / (R * 256) : 1;
    const int tid = threadIdx.x;
    const int ng = H / R;
    const int step = N / (Ns * R);
    double2 v[GM][R], b[GM][4];
    // twiddle loads first (their latency overlaps the LDS reads and the barrier)
#pragma unroll
    for (int i = 0; i < GM; ++i) {
        const int g = tid + 256 * i;
        if (g < ng) twiddle_base<R>(tw, (g & (Ns - 1)) * step, b[i]);
    }
#pragma unroll
    for (int i = 0; i < GM; ++i) {
        const int g = tid + 256 * i;
        if (g < ng) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = X[pad(g + r * ng)];
        }
    }
    if (!LAST) __syncthreads();
#pragma unroll
    for (int i = 0; i < GM; ++i) {
        const int g = tid + 256 * i;
        if (g < ng) {
            const int k = g & (Ns - 1);
            apply_twiddles<R>(v[i], b[i]);
            dft_regs<R>(v[i]);
            const int base = (g - k) * R + k;
            if (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) store_stream(out + base + r * Ns, v[i][r]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) X[pad(base + r * Ns)] = v[i][r];
            }
        }
    }
    if (!LAST) __syncthreads();
}

template <int HMAX>
__global__ void __launch_bounds__(256) k_cube_gamma(const CubeArgs c)
{
    extern __shared__ double2 X[];   // pad(H) + 1 entries
    const int row = blockIdx.x;      // (ring within the chunk) * nalpha + alpha
    const int N = c.ngamma, H = N / 2, L = c.lmax;
    const double2* P = reinterpret_cast<const double2*>(c.P) + (size_t)row * (L + 1);
    const double2* tw = reinterpret_cast<const double2*>(c.tw);
    // f_n = c[2n] + i c[2n+1] is the length-H transform of F
    double2* out = reinterpret_cast<double2*>(c.cube) + ((size_t)c.ring0 * c.nalpha + row) * (size_t)H;
    switch (H) {
    case 1:
        if (threadIdx.x == 0) out[0] = packed(half_spec(P, 0, N, L), half_spec(P, 1, N, L), tw[0]);
        return;
    case 2: first_pass<2, HMAX>(P, tw, H, N, L, X, out, true); return;
    case 4: first_pass<4, HMAX>(P, tw, H, N, L, X, out, true); return;
    case 8: first_pass<8, HMAX>(P, tw, H, N, L, X, out, true); return;
    default: break;
    }
    first_pass<16, HMAX>(P, tw, H, N, L, X, out, H == 16);
    int Ns = 16, rem = H / 16;
    while (rem > 16) { stockham_pass<16, HMAX, false>(X, H, Ns, N, tw, out); Ns *= 16; rem /= 16; }
    if (rem == 16) stockham_pass<16, HMAX, true>(X, H, Ns, N, tw, out);
    else if (rem == 8) stockham_pass<8, HMAX, true>(X, H, Ns, N, tw, out);
    else if (rem == 4) stockham_pass<4, HMAX, true>(X, H, Ns, N, tw, out);
    else if (rem == 2) stockham_pass<2, HMAX, true>(X, H, Ns, N, tw, out);
}

}  // namespace

int launch_cube_alpha(const CubeArgs& c, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    dim3 g1((c.nring_chunk + CA_T - 1) / CA_T, (c.lmax + 1 + CA_T - 1) / CA_T);
    const double2* C = reinterpret_cast<const double2*>(c.C);
    const Phase4* E = reinterpret_cast<const Phase4*>(c.phase);
    double2* P = reinterpret_cast<double2*>(c.P);
    if (c.nalpha <= 8)
        hipLaunchKernelGGL(k_cube_alpha<8>, g1, dim3(256), 0, s, c, C, E, P);
    else if (c.nalpha <= 16)
        hipLaunchKernelGGL(k_cube_alpha<16>, g1, dim3(256), 0, s, c, C, E, P);
    else
        hipLaunchKernelGGL(k_cube_alpha<32>, g1, dim3(256), 0, s, c, C, E, P);
    return (int)hipGetLastError();
}

int launch_cube_gamma(const CubeArgs& c, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int H = c.ngamma / 2;
    const size_t sh2 = sizeof(double2) * ((size_t)H + (H >> 4) + 1);
    if (H <= 4096)
        hipLaunchKernelGGL(k_cube_gamma<4096>, dim3(c.nring_chunk * c.nalpha), dim3(256), sh2, s, c);
    else
        hipLaunchKernelGGL(k_cube_gamma<CG_HMAX>, dim3(c.nring_chunk * c.nalpha), dim3(256), sh2, s, c);
    return (int)hipGetLastError();
}

int cube_set_lds_limits()
{
    // the gamma pass needs up to (8192 + 512 + 1) * 16 bytes of LDS
    int rc = (int)hipFuncSetAttribute((const void*)k_cube_gamma<4096>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (4096 + 4096 / 16 + 1) * (int)sizeof(double2));
    if (!rc)
        rc = (int)hipFuncSetAttribute((const void*)k_cube_gamma<CG_HMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (CG_HMAX + CG_HMAX / 16 + 1) * (int)sizeof(double2));
    return rc;
}

}  // namespace tc
