// Internal declarations of libtotalconv shared by the host-side table builder
// (tc_host.cpp) and the gfx950 kernels (tc_kernels.hip).  Not part of the ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace tc {

// Launch shape of the recursion kernels: each lane owns R chains (rings) of one
// (mb, msky) column and a workgroup has NT lanes, so one workgroup covers
// NT*R ring slots of one column.
struct Tile {
    int R;    // chains per lane
    int NT;   // lanes per workgroup
    int TB;   // l values per LDS coefficient block
    int TR;   // adjoint: steps per wave reduction of the lane sums
};

// Device-resident per-call tables, all inside the caller's workspace.
struct RingTables {
    const double* x;     // cos(beta_j)
    const double* lch;   // ln cos(beta_j/2), double-double (hi, lo); hi = -inf when cos(beta_j/2) = 0
    const double* lcl;
    const double* lsh;   // ln sin(beta_j/2), double-double; hi = -inf when sin(beta_j/2) = 0
    const double* lsl;
};

// Column list (processing order) with the seed normalisation of each column.
struct ColumnTables {
    const int* mb;       // [ncol]
    const int* ms;       // [ncol]
    const double* lnA;   // [ncol][2] double-double ln sqrt((2l0)!/((l0+m)!(l0-m)!))
};

struct WignerArgs {
    int lmax, npair, nring, ntile;
    RingTables ring;
    ColumnTables col;      // one "column" per requested (mb, msky) pair, in request order
    double* d;             // [npair][lmax+1][nring]
};

// (sky, beam) pairs that share one walk of the recursion: the polarised pairs (up to 3) or the
// detectors of a batched plan that share lmax and rings (up to 4).
constexpr int kMaxPairs = 4;

struct FwdArgs {
    int lmax, mbmax, nring, nslot, ncol, ntile;   // mbmax: of the column table (the largest pmbmax)
    int sky_lmax;          // packing lmax of the sky (>= lmax; detectors may share one sky)
    int skip_exp;          // accumulate from the first l-block that may hold |d| >= 2^-skip_exp; 0 = always
    RingTables ring;
    const int* slots;      // [nslot][2] (ring j, mirror ring or -1)
    ColumnTables col;
    int npair;             // pairs sharing the walk: 1 scalar, up to 3 polarised (temperature, gradient,
                           // curl), up to kMaxPairs detectors ordered by pmbmax, largest first
    int sum;               // polarised: 1 = one output, the sum over the pairs; 0 = one output per pair
    int pmbmax[kMaxPairs]; // rows of pair p's beam and output: mb = -pmbmax[p] .. pmbmax[p]
    const double* alm[kMaxPairs];  // packed sky of each pair (complex)
    const double* blm[kMaxPairs];  // [2 pmbmax+1][L+1] complex, per pair
    double* C[kMaxPairs];          // [2 pmbmax+1][L+1][nring] complex, per output
    const int* beam_sym[kMaxPairs];  // scalar convolution: per beam row mb + pmbmax, s = +-1 if
                           // b_{l,-mb} = s b_{l,mb} for every l >= |mb|, else 0 (from k_beam_symmetry);
                           // null: not used (polarised)
};

struct AdjArgs {
    int lmax, mbmax, nring, nslot, ncol, ntile;   // mbmax: of the column table (the largest pmbmax)
    int skip_exp;
    RingTables ring;
    const int* slots;
    ColumnTables col;
    int npair;             // cotangents sharing the walk: 1, or the detectors of a batched walk
                           // (same lmax and rings), ordered by pmbmax, largest first
    int pmbmax[kMaxPairs]; // rows of cotangent p and of its sums: mb = -pmbmax[p] .. pmbmax[p]
    const double* Cbar[kMaxPairs];  // layout of C, per cotangent
    double* U[kMaxPairs];  // complex [2 pmbmax+1][P] direct-ring sums u_l (all ring tiles of a column)
    double* V[kMaxPairs];  // complex [2 pmbmax+1][P] mirror-ring sums (before the (-1)^(l-msky) sign)
    long long P;           // (L+1)(L+2)/2
};

struct EpiArgs {
    int lmax, mbmax;
    int sky_lmax;          // packing lmax of alm and alm_bar
    long long P;
    const double* U;
    const double* V;
    const double* alm;
    const double* blm;
    double* alm_bar;       // may be null
    double* blm_bar;       // may be null
};

// The sky gradients of npair (2 or 3) (sky, beam) pairs that share one cotangent and so one U, V
// (the polarised adjoint with summed outputs); every beam has the rows -mbmax .. mbmax.
struct EpiPairsArgs {
    int lmax, mbmax;
    int sky_lmax;          // packing lmax of every alm_bar
    int npair;
    long long P;
    const double* U;
    const double* V;
    const double* blm[3];
    double* alm_bar[3];    // entries may be null (that pair's sky gradient is not stored)
};

// Full matrix d^l_{m m'} at one l: the m' recursion on the triangle 0 <= m <= m' <= l
// at beta (side 0) and at pi - beta (side 1), written out with its symmetric images.
struct MatrixArgs {
    int l, nring, ntile;   // ntile: row tiles per (ring, side)
    RingTables ring;       // x, ln cos(beta/2), ln sin(beta/2)
    const double* trig;    // [nring][2]: cot(beta), csc(beta) (unused at the poles)
    const double* lnA;     // [l+1][2] double-double ln sqrt((2l)! / ((l+m)! (l-m)!))
    double* d;             // [nring][2l+1][2l+1], d[j][m+l][m'+l]
};

int launch_matrix(const MatrixArgs& a, int variant, void* stream);
int matrix_rows_per_group(int variant);   // rows m one workgroup walks (0: no such variant)

// Data cube (eq. conviqt) of rings [ring0, ring0 + nring_chunk).
struct CubeArgs {
    int lmax, mbmax, nring, nalpha, ngamma;
    int ring0, nring_chunk;
    const double* C;       // [2M+1][L+1][nring] complex (totalconv_fwd output)
    const double* phase;   // [2M+1][nalpha rounded up to 4] complex, e^{-2 pi i mb a / nalpha} (pad: 0)
    const double* tw;      // [ngamma] complex, e^{-2 pi i m / ngamma}
    double* P;             // [nring_chunk][nalpha][L+1] complex, alpha sums of the chunk
    double* cube;          // [nring][nalpha][ngamma] real
};

// Data-cube launchers (tc_cube.hip).
int launch_cube_alpha(const CubeArgs& c, void* stream);   // P of the chunk from C
int launch_cube_gamma(const CubeArgs& c, void* stream);   // the chunk's cube rows from P
int cube_set_lds_limits();

// Kernel launchers (tc_kernels.hip).  Return a hipError_t value (0 on success).
int launch_wigner(const WignerArgs& a, Tile t, void* stream);
int launch_fwd(const FwdArgs& a, Tile t, void* stream);
int launch_beam_symmetry(const double* blm, int lmax, int mbmax, int* sym, void* stream);
int launch_adj(const AdjArgs& a, Tile t, void* stream);
int launch_adj_epilogue(const EpiArgs& e, void* stream);
// tc_epilogue.hip: the sky gradients of every pair in one launch, U and V read once.
int launch_adj_sky_pairs(const EpiPairsArgs& e, void* stream);

// Batched launches: one workgroup per item; forward items are (walk, column, ring tile) triples,
// adjoint items (detector, column) pairs (the workgroup walks every ring tile of the column).
int launch_fwd_items(const FwdArgs* walks, const int* items, int nitems, Tile t, void* stream);
// Detectors one batched forward / adjoint walk serves with tile t (at most kMaxPairs).
int fwd_walk_pairs(Tile t);
int adj_walk_pairs_of(Tile t);
int launch_adj_items(const AdjArgs* dets, const int* items, int nitems, Tile t, void* stream);
int launch_adj_sky_multi(const EpiArgs* eps, int ndet, int sky_lmax, bool accumulate, double* alm_bar,
                         void* stream);
int launch_adj_beam(const EpiArgs& e, void* stream);
bool tile_supported(int op, Tile t);

// The forward on colatitudes with its tables in `scratch` (scratch_bytes) instead of a caller
// workspace, copied from pageable host memory (no pinned cache, no allocation of device or pinned
// memory); TC_ENOMEM when the tables do not fit (tc_host.cpp).
int fwd_noalloc(int lmax, int mbmax, int nring, const double* beta, const double* alm, const double* blm, double* C,
                void* scratch, size_t scratch_bytes, void* stream);
// Records a failed HIP call as the calling thread's last error and returns TC_EHIP (tc_host.cpp).
int fail_hip(int rc, const char* what);

}  // namespace tc
