"""Polarised total convolution (temperature, gradient and curl pairs sharing one
recursion) against the oracle, which evaluates eq. convdef for each pair (footnote of
Sec. 4.1), through the C ABI.  Gates as in test_gpu_parity: per column for C, normwise
(sky) and per mb row (beam) for the gradients, 1e-11."""
import sys

import numpy as np
import pytest

from paper_1002_1050_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GATE = 1e-11


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1002_1050_amd import _binding
    _binding.lib()
    yield _binding
    _binding.set_tile_ex(_binding.TC_OP_FWD_POL, 0, 0, 0)
    _binding.set_tile_ex(_binding.TC_OP_FWD, 0, 0, 0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def column_gate(got, ref):
    got = got.reshape(-1, got.shape[-1])
    ref = ref.reshape(-1, ref.shape[-1])
    num = np.abs(got - ref).max(axis=1)
    den = np.abs(ref).max(axis=1)
    assert np.all(num[den == 0] == 0), "non-zero result in an all-zero column"
    return float((num[den > 0] / den[den > 0]).max())


def pairs(L, M, n, seed):
    alms = [S.sky_alm(L, seed + p) for p in range(n)]
    blms = [S.random_beam(L, M, seed + 10 + p) for p in range(n)]
    return alms, blms


# 2600 rings: 1300 mirror slots, so two ring tiles at R = 4 and three at R = 2
CASES = [(120, 4, 2600), (70, 9, 301)]


@pytest.mark.parametrize("R,TB", [(2, 32), (4, 64)])
@pytest.mark.parametrize("npair", [2, 3])
def test_polarised_forward_separate_and_summed(B, orc, R, TB, npair):
    for L, M, n in CASES:
        x = S.ring_cosines(n)
        alms, blms = pairs(L, M, npair, 100 + L)
        da, db = [dev(a) for a in alms], [dev(b) for b in blms]
        B.set_tile_ex(B.TC_OP_FWD_POL, R, TB, 0)
        say(f"fwd_pol L={L} M={M} nring={n} npair={npair} R={R} TB={TB}")
        sep = [c.cpu().numpy() for c in B.totalconv_fwd_pol_x(L, M, x, da, db, B.TC_POL_SEPARATE)]
        tot = B.totalconv_fwd_pol_x(L, M, x, da, db, B.TC_POL_SUM)[0].cpu().numpy()
        ref = orc.totalconv_fwd_pol(L, M, x, alms, blms)
        gs = max(column_gate(sep[p], ref[p]) for p in range(npair))
        gt = column_gate(tot, sum(ref))
        say(f"  separate {gs:.2e}, summed {gt:.2e}")
        assert gs <= GATE and gt <= GATE
        # each separate output is the scalar forward of its pair, same tile: same arithmetic,
        # except on beam rows related to their mirror row by a sign (here the mb = 0 row of the
        # random beams), where the scalar forward sums even and odd l apart
        B.set_tile_ex(B.TC_OP_FWD, R, TB, 0)
        for p in range(npair):
            plain = B.totalconv_fwd_x(L, M, x, da[p], db[p]).cpu().numpy()
            rows = [r for r in range(2 * M + 1) if r != M]
            assert np.array_equal(plain[rows], sep[p][rows]), f"pair {p}: polarised output != scalar forward"
            assert column_gate(plain[M], sep[p][M]) <= 1e-13


def test_polarised_single_pair_is_scalar(B, orc):
    L, M, n = 90, 5, 400
    x = S.ring_cosines(n)
    alms, blms = pairs(L, M, 1, 7)
    da, db = [dev(alms[0])], [dev(blms[0])]
    say("fwd_pol npair=1")
    got = B.totalconv_fwd_pol_x(L, M, x, da, db, B.TC_POL_SUM)[0].cpu().numpy()
    ref = orc.totalconv_fwd(L, M, x, alms[0], blms[0])
    assert column_gate(got, ref) <= GATE


@pytest.mark.parametrize("summed", [True, False])
def test_polarised_adjoint(B, orc, summed):
    L, M, n = 150, 6, 1200
    x = S.ring_cosines(n)
    alms, blms = pairs(L, M, 3, 300)
    da, db = [dev(a) for a in alms], [dev(b) for b in blms]
    nG = 1 if summed else 3
    Gs = [S.random_cbar(L, M, n, 500 + k) for k in range(nG)]
    mode = B.TC_POL_SUM if summed else B.TC_POL_SEPARATE
    say(f"adj_pol L={L} M={M} nring={n} summed={summed}")
    ga, gb = B.totalconv_adj_pol_x(L, M, x, da, db, [dev(g) for g in Gs], mode)
    ra, rb = orc.totalconv_adj_pol(L, M, x, alms, blms, Gs, summed=summed)
    for p in range(3):
        a = ga[p].cpu().numpy()
        b = gb[p].cpu().numpy()
        ea = np.linalg.norm(a - ra[p]) / np.linalg.norm(ra[p])
        eb = max(np.linalg.norm(b[r] - rb[p][r]) / np.linalg.norm(rb[p][r])
                 for r in range(2 * M + 1) if np.any(rb[p][r] != 0))
        say(f"  pair {p}: sky {ea:.2e}, beam {eb:.2e}")
        assert ea <= GATE and eb <= GATE
    # only the beam gradients requested: the sky arrays stay untouched (None)
    ga2, gb2 = B.totalconv_adj_pol_x(L, M, x, da, db, [dev(g) for g in Gs], mode, want_alm=False)
    assert all(g is None for g in ga2)
    for p in range(3):
        assert torch.equal(gb2[p], gb[p])


@pytest.mark.parametrize("npair", [2, 3])
@pytest.mark.parametrize("L,M,n", [(150, 6, 1200), (300, 4, 701), (6, 6, 3), (0, 0, 1)])
def test_polarised_summed_adjoint_equals_scalar_adjoints(B, L, M, n, npair):
    """Summed outputs: the pairs share one cotangent and so one U, V, which one launch reads for
    every pair's sky gradient.  Each pair's sky and beam gradients equal, bit for bit, those of a
    scalar adjoint of that cotangent with the pair's sky and beam; requesting only the sky
    gradients gives the same sky gradients."""
    x = S.ring_cosines(n)
    alms, blms = pairs(L, M, npair, 700)
    da, db = [dev(a) for a in alms], [dev(b) for b in blms]
    G = dev(S.random_cbar(L, M, n, 800))
    say(f"adj_pol summed vs scalar adjoints L={L} M={M} nring={n} npair={npair}")
    ga, gb = B.totalconv_adj_pol_x(L, M, x, da, db, [G], B.TC_POL_SUM)
    for p in range(npair):
        sa, sb = B.totalconv_adj_x(L, M, x, da[p], db[p], G)
        assert torch.equal(ga[p], sa), f"sky gradient of pair {p}"
        assert torch.equal(gb[p], sb), f"beam gradient of pair {p}"
    ga2, gb2 = B.totalconv_adj_pol_x(L, M, x, da, db, [G], B.TC_POL_SUM, want_blm=False)
    assert all(g is None for g in gb2)
    for p in range(npair):
        assert torch.equal(ga2[p], ga[p])


def test_polarised_rejects_bad_arguments(B):
    L, M = 20, 2
    x = S.ring_cosines(41)
    alms, blms = pairs(L, M, 3, 1)
    da, db = [dev(a) for a in alms], [dev(b) for b in blms]
    lib = B.lib()
    arr = B._ptr_array
    out = [torch.empty((2 * M + 1, L + 1, x.size), dtype=torch.complex128, device="cuda") for _ in range(4)]
    ws = torch.empty(B.workspace_bytes_x(B.TC_OP_FWD_POL, L, M, x), dtype=torch.uint8, device="cuda")
    xp = x.ctypes.data_as(B.ctypes.c_void_p)
    for npair, mode in ((4, 0), (0, 0), (2, 2)):
        rc = lib.totalconv_fwd_pol_x(L, M, x.size, xp, npair, arr(da + da), arr(db + db), mode, arr(out),
                                   B._dptr(ws), ws.numel(), None)
        assert rc == -1, (npair, mode)
    rc = lib.totalconv_fwd_pol_x(L, M, x.size, xp, 3, arr(da[:2] + [None]), arr(db), 0, arr(out),
                               B._dptr(ws), ws.numel(), None)
    assert rc == -1 and "pair 2" in B.last_error()


@pytest.mark.parametrize("summed", [False, True])
def test_polarised_autograd_central_differences(B, summed):
    """TotalConvPol's backward (the polarised adjoint) against central differences of a quadratic
    loss, for every pair's sky and beam."""
    from paper_1002_1050_amd.autograd import TotalConvPolX as TotalConvPol
    L, M, n = 20, 2, 41
    x = S.ring_cosines(n)
    mode = B.TC_POL_SUM if summed else B.TC_POL_SEPARATE
    alms = [dev(S.sky_alm(L, 60 + p) + 0.0j).requires_grad_(True) for p in range(3)]
    blms = [dev(S.random_beam(L, M, 70 + p)).requires_grad_(True) for p in range(3)]
    Ts = [dev(S.random_cbar(L, M, n, 80 + k)) for k in range(1 if summed else 3)]
    say(f"polarised autograd, summed={summed}")

    def loss(a_list, b_list):
        outs = TotalConvPol.apply(mode, x, L, M, *a_list, *b_list)
        return 0.5 * sum(torch.sum(torch.abs(C - T) ** 2) for C, T in zip(outs, Ts))

    loss(alms, blms).backward()
    grads = [t.grad.clone() for t in alms + blms]
    gmax = max(g.abs().max().item() for g in grads)
    rng = np.random.Generator(np.random.PCG64(11))
    h = 1e-3
    with torch.no_grad():
        for p in range(3):
            for k in rng.choice(alms[p].numel(), 4, replace=False):
                for unit in (1.0, 1j):
                    d = torch.zeros_like(alms[p])
                    d[k] = h * unit
                    plus = [a + d if q == p else a for q, a in enumerate(alms)]
                    minus = [a - d if q == p else a for q, a in enumerate(alms)]
                    fd = ((loss(plus, blms) - loss(minus, blms)) / (2 * h)).item()
                    g = grads[p][k]
                    assert abs(fd - (g.real.item() if unit == 1.0 else g.imag.item())) <= 1e-8 * gmax
            for _ in range(4):
                r, l = int(rng.integers(0, 2 * M + 1)), int(rng.integers(0, L + 1))
                if l < abs(r - M):
                    continue
                for unit in (1.0, 1j):
                    d = torch.zeros_like(blms[p])
                    d[r, l] = h * unit
                    plus = [b + d if q == p else b for q, b in enumerate(blms)]
                    minus = [b - d if q == p else b for q, b in enumerate(blms)]
                    fd = ((loss(alms, plus) - loss(alms, minus)) / (2 * h)).item()
                    g = grads[3 + p][r, l]
                    assert abs(fd - (g.real.item() if unit == 1.0 else g.imag.item())) <= 1e-8 * gmax


def test_polarised_full_size_sampled(B, orc):
    """The benchmark's polarised launch at full size: lmax 4096, mbmax 14, 8192 rings, three
    pairs (the workload's sky and beam plus two seeded skies and random beams), built-in tile;
    sampled columns of every separate output and of the summed output against the oracle over
    every ring."""
    w = S.WORKLOADS["lmax4096"]
    L, M, x = w.lmax, w.mbmax, w.xring()
    alms = [w.alm()] + [S.sky_alm(L, w.sky_seed + 1 + p) for p in range(2)]
    blms = [w.blm()] + [S.random_beam(L, M, 77 + p) for p in range(2)]
    da, db = [dev(a) for a in alms], [dev(b) for b in blms]
    rng = np.random.Generator(np.random.PCG64(4096))
    mb = np.concatenate([[0, M, -M, 1], rng.integers(-M, M + 1, 8)]).astype(np.int32)
    ms = np.concatenate([[0, L, 1, L // 2], (rng.random(8) ** 0.7 * (L + 1)).astype(int)]).astype(np.int32)
    ms = np.minimum(ms, L)
    idx = torch.from_numpy(((mb + M) * (L + 1) + ms).astype(np.int64)).to("cuda")
    say(f"fwd_pol full size L={L} M={M} nring={x.size}, three pairs")
    sep = B.totalconv_fwd_pol_x(L, M, x, da, db, B.TC_POL_SEPARATE)
    got = [c.reshape(-1, x.size).index_select(0, idx).cpu().numpy() for c in sep]
    del sep
    torch.cuda.empty_cache()
    tot = B.totalconv_fwd_pol_x(L, M, x, da, db, B.TC_POL_SUM)[0]
    got_t = tot.reshape(-1, x.size).index_select(0, idx).cpu().numpy()
    del tot
    torch.cuda.empty_cache()
    ref = [orc.totalconv_fwd(L, M, x, alms[p], blms[p], cols=(mb, ms)) for p in range(3)]
    gs = max(column_gate(got[p], ref[p]) for p in range(3))
    gt = column_gate(got_t, ref[0] + ref[1] + ref[2])
    say(f"  {mb.size} columns: separate {gs:.2e}, summed {gt:.2e}")
    assert gs <= GATE and gt <= GATE


def test_polarised_summed_adjoint_full_size_equals_scalar_adjoints(B):
    """The summed-output adjoint at the lmax 4096 workload (three pairs, built-in tile): every
    pair's sky and beam gradients equal, bit for bit, those of a scalar adjoint of the same
    cotangent (the sky gradients of all pairs come from one launch over the shared U, V)."""
    w = S.WORKLOADS["lmax4096"]
    L, M, x = w.lmax, w.mbmax, w.xring()
    alms = [w.alm()] + [S.sky_alm(L, w.sky_seed + 1 + p) for p in range(2)]
    blms = [w.blm()] + [S.random_beam(L, M, 77 + p) for p in range(2)]
    da, db = [dev(a) for a in alms], [dev(b) for b in blms]
    g = torch.Generator(device="cuda")
    g.manual_seed(4096)
    G = torch.randn((2 * M + 1, L + 1, x.size), dtype=torch.complex128, device="cuda", generator=g)
    say(f"adj_pol summed full size L={L} M={M} nring={x.size}, three pairs, vs scalar adjoints")
    ga, gb = B.totalconv_adj_pol_x(L, M, x, da, db, [G], B.TC_POL_SUM)
    for p in range(3):
        sa, sb = B.totalconv_adj_x(L, M, x, da[p], db[p], G)
        assert torch.equal(ga[p], sa), f"sky gradient of pair {p}"
        assert torch.equal(gb[p], sb), f"beam gradient of pair {p}"
        del sa, sb
    del G
    torch.cuda.empty_cache()
