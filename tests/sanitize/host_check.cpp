// Host-side table preparation and argument checking of libtotalconv, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize_cpu.py.  No GPU is
// used: tc_host.cpp is compiled into this program, the kernel launchers below are stubs that
// fail, and the HIP runtime reports that no device is present.  Every check prints its name;
// the program ends with "ok" and exit status 0, or the first failed check and status 1.
#include "../../paper_1002_1050_amd/csrc/tc_host.cpp"

#include <cmath>
#include <cstdio>
#include <vector>

namespace tc {
// Launchers are never reached without a device; each returns hipErrorInvalidDeviceFunction.
constexpr int kNoKernel = 98;
int launch_matrix(const MatrixArgs&, int, void*) { return kNoKernel; }
int matrix_rows_per_group(int v) { return v == 0 ? 128 : 64 * v; }
int launch_cube_alpha(const CubeArgs&, void*) { return kNoKernel; }
int launch_cube_gamma(const CubeArgs&, void*) { return kNoKernel; }
int cube_set_lds_limits() { return kNoKernel; }
int launch_wigner(const WignerArgs&, Tile, void*) { return kNoKernel; }
int launch_fwd(const FwdArgs&, Tile, void*) { return kNoKernel; }
int launch_beam_symmetry(const double*, int, int, int*, void*) { return kNoKernel; }
int launch_adj(const AdjArgs&, Tile, void*) { return kNoKernel; }
int launch_adj_epilogue(const EpiArgs&, void*) { return kNoKernel; }
int launch_adj_sky_pairs(const EpiPairsArgs&, void*) { return kNoKernel; }
int launch_fwd_items(const FwdArgs*, const int*, int, Tile, void*) { return kNoKernel; }
int fwd_walk_pairs(Tile t) { return t.R >= 8 ? 2 : 4; }
int adj_walk_pairs_of(Tile t) { return (t.R <= 4 && t.TB <= 32) ? 2 : 1; }
int launch_adj_items(const AdjArgs*, const int*, int, Tile, void*) { return kNoKernel; }
int launch_adj_sky_multi(const EpiArgs*, int, int, bool, double*, void*) { return kNoKernel; }
int launch_adj_beam(const EpiArgs&, void*) { return kNoKernel; }
bool tile_supported(int, Tile) { return false; }
}  // namespace tc

namespace {

int g_failed = 0;

void check(bool ok, const char* what)
{
    std::printf("%s %s\n", ok ? "pass" : "FAIL", what);
    if (!ok) g_failed = 1;
}

// Equator-symmetric colatitudes (j + 1/2) pi / n, rounded to doubles.
std::vector<double> grid(int n)
{
    std::vector<double> b(n);
    for (int j = 0; j < n; ++j) b[j] = (double)((j + 0.5L) * kPiL / n);
    return b;
}

void rings_and_slots()
{
    for (int n : {1, 2, 7, 64, 301}) {
        const std::vector<double> beta = grid(n);
        std::vector<double> x;
        check(rings_from_beta(n, beta.data(), x) == TC_OK && (int)x.size() == n, "rings_from_beta accepts a grid");
        bool mirror = true;
        for (int j = 0; j < n - 1 - j; ++j) mirror = mirror && x[n - 1 - j] == -x[j];
        check(mirror, "grid rings are exact mirror pairs");
        check(count_slots(n, x.data()) == (n + 1) / 2, "one slot per mirror pair and per single ring");
        const Layout L = make_layout(TC_OP_FWD, 20, 3, n, x.data(), tc::Tile{4, 256, 32, 4});
        std::vector<char> img(L.tables_end, 0);
        build_rings(n, x.data(), img, L);
        build_slots(n, x.data(), img, L);
        const int* s = reinterpret_cast<const int*>(img.data() + L.slots);
        std::vector<int> seen(n, 0);
        for (int k = 0; k < L.nslot; ++k) {
            seen[s[2 * k]] += 1;
            if (s[2 * k + 1] >= 0) seen[s[2 * k + 1]] += 1;
        }
        bool once = true;
        for (int v : seen) once = once && v == 1;
        check(once, "every ring sits in exactly one slot");
        // the tables are functions of the ring cosine x: cos^2(beta/2) = (1 + x)/2, sin^2 = (1 - x)/2
        const double* r = reinterpret_cast<const double*>(img.data() + L.ring);
        bool logs = true;
        for (int j = 0; j < n; ++j) {
            const long double X = x[j];
            const long double lc = (long double)r[n + j] + r[2 * n + j];
            const long double ls = (long double)r[3 * n + j] + r[4 * n + j];
            const long double wc = 0.5L * logl((1.0L + X) / 2.0L), ws = 0.5L * logl((1.0L - X) / 2.0L);
            logs = logs && fabsl(lc - wc) <= 1e-17L * (1.0L + fabsl(wc));
            logs = logs && fabsl(ls - ws) <= 1e-17L * (1.0L + fabsl(ws));
        }
        check(logs, "ln cos(beta/2) and ln sin(beta/2) in double-double");
    }
    std::vector<double> x;
    const double bad[3] = {0.1, -1e-3, 1.0};
    check(rings_from_beta(3, bad, x) == TC_EINVAL, "a negative colatitude is refused");
    const double nan_beta[2] = {0.1, std::nan("")};
    check(rings_from_beta(2, nan_beta, x) == TC_EINVAL, "a NaN colatitude is refused");
    const double poles[2] = {0.0, (double)kPiL};
    check(rings_from_beta(2, poles, x) == TC_OK && x[0] == 1.0 && x[1] == -1.0, "the poles");
    const Layout L = make_layout(TC_OP_FWD, 5, 0, 2, x.data(), tc::Tile{4, 256, 32, 4});
    std::vector<char> img(L.tables_end, 0);
    build_rings(2, x.data(), img, L);
    const double* r = reinterpret_cast<const double*>(img.data() + L.ring);
    check(std::isinf(r[3 * 2 + 0]) && r[3 * 2 + 0] < 0 && std::isinf(r[2 + 1]) && r[2 + 1] < 0,
          "ln sin at the north pole and ln cos at the south pole are -inf");
}

void columns_and_layout()
{
    const std::vector<double> beta = grid(40);
    std::vector<double> x;
    rings_from_beta(40, beta.data(), x);
    for (int op : {TC_OP_FWD, TC_OP_ADJ}) {
        const int lmax = 33, mbmax = 5;
        const Layout L = make_layout(op, lmax, mbmax, 40, x.data(), tc::Tile{8, 256, 64, 4});
        check(L.ncol == (2 * mbmax + 1) * (lmax + 1) && L.ntile == 1, "column count and ring tiles");
        const size_t offs[] = {L.ring, L.slots, L.colmb, L.colms, L.lna, L.tables_end};
        bool order = true;
        for (int k = 0; k < 6; ++k) order = order && offs[k] % kAlign == 0 && (k == 0 || offs[k] >= offs[k - 1]);
        check(order, "table offsets aligned and in order");
        if (op == TC_OP_ADJ)
            check(L.U >= L.tables_end && L.V >= L.U + (size_t)16 * (2 * mbmax + 1) * (size_t)L.P &&
                      L.total >= L.V + (size_t)16 * (2 * mbmax + 1) * (size_t)L.P,
                  "U and V after the tables, one row per beam row");
        std::vector<char> img(L.tables_end, 0);
        build_columns(lmax, mbmax, img, L);
        const int* cmb = reinterpret_cast<const int*>(img.data() + L.colmb);
        const int* cms = reinterpret_cast<const int*>(img.data() + L.colms);
        const double* lna = reinterpret_cast<const double*>(img.data() + L.lna);
        bool sorted = true, norm = true;
        for (int i = 0; i < L.ncol; ++i) {
            const int l0 = std::max(std::abs(cmb[i]), cms[i]);
            if (i > 0) sorted = sorted && l0 >= std::max(std::abs(cmb[i - 1]), cms[i - 1]);
            const int m = std::abs(cms[i]) >= std::abs(cmb[i]) ? cmb[i] : cms[i];
            const double want = 0.5 * (std::lgamma(2.0 * l0 + 1) - std::lgamma(l0 + m + 1.0) - std::lgamma(l0 - m + 1.0));
            norm = norm && std::fabs(lna[2 * i] + lna[2 * i + 1] - want) <= 1e-13 * (1 + std::fabs(want));
        }
        check(sorted, "columns ordered by l0");
        check(norm, "seed normalisation ln A against lgamma");
    }
}

void entry_points()
{
    const std::vector<double> beta = grid(16);
    std::vector<double> alm(2 * 100), blm(2 * 64), C(2 * 64 * 16);
    check(totalconv_fwd(-1, 0, 16, beta.data(), alm.data(), blm.data(), C.data(), nullptr, 0, nullptr) == TC_EINVAL,
          "lmax < 0 is refused");
    check(totalconv_fwd(8, 9, 16, beta.data(), alm.data(), blm.data(), C.data(), nullptr, 0, nullptr) == TC_EINVAL,
          "mbmax > lmax is refused");
    check(tc_last_error() != nullptr && std::strlen(tc_last_error()) > 0, "the refusal is explained");
    const size_t ws = totalconv_workspace_bytes(TC_OP_ADJ, 64, 4, 16);
    check(ws > 0 && ws >= totalconv_workspace_bytes(TC_OP_FWD, 64, 4, 16), "workspace sizes");
    check(totalconv_workspace_bytes(TC_OP_FWD, -3, 0, 16) == 0, "no workspace size for bad sizes");
    std::vector<double> x(16);
    check(tc_rings_from_beta(16, beta.data(), x.data()) == TC_OK && x[15] == -x[0], "tc_rings_from_beta");
    // plans: a bad detector is refused; good ones get as far as the device allocation
    std::vector<tc_detector> d(3);
    std::vector<std::vector<double>> b(3);
    for (int i = 0; i < 3; ++i) {
        b[i] = grid(12 + 4 * i);
        d[i] = tc_detector{};
        d[i].lmax = 10; d[i].mbmax = i; d[i].nring = 12 + 4 * i;
        d[i].beta = b[i].data();
        d[i].blm = blm.data();
        d[i].C = C.data();
    }
    void* plan = nullptr;
    d[1].mbmax = 11;
    check(tc_plan_create(&plan, TC_OP_FWD, 3, d.data(), 10, alm.data(), nullptr, nullptr) == TC_EINVAL && !plan,
          "a plan with a bad detector is refused");
    d[1].mbmax = 1;
    const int rc = tc_plan_create(&plan, TC_OP_FWD, 3, d.data(), 10, alm.data(), nullptr, nullptr);
    check(rc != TC_OK && !plan, "without a device a plan fails cleanly");
    check(tc_plan_destroy(nullptr) == TC_OK, "destroying NULL");
}

}  // namespace

int main()
{
    rings_and_slots();
    columns_and_layout();
    entry_points();
    if (g_failed) return 1;
    std::printf("ok\n");
    return 0;
}
