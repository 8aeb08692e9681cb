"""Pins for the oracle's total-convolution sum and its adjoint (CPU only).

C_{mb,msky}(beta) = sum_l conj(b_{l,mb}) d^l_{mb,msky}(beta) s_{l,msky}  (Sec. 4.1, eq. convdef).
Checked against an mpmath brute force built on Wigner's explicit sum, the
spherical-harmonic special case (Sec. 4), the symmetries of Sec. 4.2.3, linearity,
and for the adjoint the dot-product identity, exact central differences of a
quadratic loss, and an mpmath brute force.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_1002_1050_amd import synthetic as S


def rings(n):
    """Ring cosines of the equispaced grid, exactly mirror-symmetric."""
    return S.ring_cosines(n)


def sky_get(alm, lmax):
    def get(l, m):
        if m >= 0:
            return complex(alm[S.alm_index(lmax, l, m)])
        return (-1) ** m * complex(np.conj(alm[S.alm_index(lmax, l, -m)]))
    return get


def beam_get(blm, mbmax):
    return lambda l, mb: complex(blm[mb + mbmax, l])


def random_sky(lmax, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal(S.alm_size(lmax)) + 1j * rng.standard_normal(S.alm_size(lmax))
    a[: lmax + 1] = a[: lmax + 1].real
    return a


def test_brute_force_tiny(orc):
    """Every column, every ring, against mpmath sums of explicit-sum d (complex beam and sky,
    negative msky included through the sky's reality relation)."""
    mp.mp.dps = 40
    from oracle import mpref
    L, M, n = 9, 3, 7
    xr = rings(n)
    x = xr
    alm = random_sky(L, 3)
    blm = S.random_beam(L, M, 4)
    mbs = np.repeat(np.arange(-M, M + 1), 2 * L + 1).astype(np.int32)
    mss = np.tile(np.arange(-L, L + 1), 2 * M + 1).astype(np.int32)
    C = orc.totalconv_fwd(L, M, xr, alm, blm, cols=(mbs, mss))
    sg, bg = sky_get(alm, L), beam_get(blm, M)
    worst = 0.0
    for i in range(mbs.size):
        for j in range(n):
            ref = mpref.conv_brute(L, int(mbs[i]), int(mss[i]), x[j], sg, bg)
            worst = max(worst, abs(C[i, j] - ref))
    assert worst <= 5e-15, worst


def test_full_layout_and_delta_inputs(orc):
    """A unit sky at (l*, m*) and a unit beam at (l*, mb*) give C = d^{l*}_{mb*, m*} in that
    single column and zero elsewhere; checks layout, conjugation and the l-range."""
    L, M, n = 20, 4, 9
    xr = rings(n)
    for (ls, ms, mbs) in [(7, 3, -2), (20, 0, 4), (4, 4, 4), (13, 12, -3)]:
        alm = S.delta_sky(L, ls, ms, 1.0)
        blm = S.delta_beam(L, M, ls, mbs, 1.0)
        C = orc.totalconv_fwd(L, M, xr, alm, blm)
        d = orc.wigner_d(L, [mbs], [ms], xr)[0, ls]
        expect = np.zeros_like(C)
        expect[mbs + M, ms] = d
        np.testing.assert_allclose(C, expect, atol=1e-16, rtol=0)
        # complex weights: conj on the beam, none on the sky
        C2 = orc.totalconv_fwd(L, M, xr, S.delta_sky(L, ls, ms, 2 - 1j), S.delta_beam(L, M, ls, mbs, 1j))
        np.testing.assert_allclose(C2[mbs + M, ms], np.conj(1j) * (2 - 1j) * d, atol=1e-15)


def test_spherical_harmonic_special_case(orc):
    """mb = 0 with an axisymmetric beam: C_{0,m}(theta) = sum_l b_{l0} s_{lm} (-1)^m
    sqrt(4 pi/(2l+1)) Y_lm(theta, 0)  (Sec. 4 relation between Y_lm and D^l_{0m})."""
    mp.mp.dps = 30
    L, M, n = 24, 2, 5
    xr = rings(n)
    x = xr
    th = [mp.acos(mp.mpf(v)) for v in x]
    alm = S.sky_alm(L, 11)
    blm = S.beam_blm(L, M, 300.0, 0.0)           # e = 0: only mb = 0 is non-zero
    C = orc.totalconv_fwd(L, M, xr, alm, blm)
    for m in (0, 1, 5, 17):
        for j in range(n):
            ref = mp.mpc(0)
            for l in range(m, L + 1):
                y = mp.re(mp.spherharm(l, m, th[j], 0))
                ref += blm[M, l].real * complex(alm[S.alm_index(L, l, m)]) * (-1) ** m \
                    * mp.sqrt(4 * mp.pi / (2 * l + 1)) * y
            assert abs(C[M, m, j] - complex(ref)) <= 1e-15


def test_conjugate_symmetry(orc):
    """C_{-mb,-msky} = conj(C_{mb,msky}) for a real sky and a real-space beam (Sec. 4.2.3)."""
    L, M, n = 40, 6, 13
    xr = rings(n)
    alm = S.sky_alm(L, 5)
    blm = S.beam_blm(L, M, 200.0, 0.25)
    mbs = np.repeat(np.arange(-M, M + 1), L + 1).astype(np.int32)
    mss = np.tile(np.arange(0, L + 1), 2 * M + 1).astype(np.int32)
    C = orc.totalconv_fwd(L, M, xr, alm, blm, cols=(mbs, mss))
    Cn = orc.totalconv_fwd(L, M, xr, alm, blm, cols=(-mbs, -mss))
    np.testing.assert_allclose(Cn, np.conj(C), atol=1e-15, rtol=0)


def test_pi_minus_beta_pairing(orc):
    """C_{-mb,msky}(pi - beta) = sum_l conj(b_{l,-mb}) (-1)^{l-msky} d^l_{mb,msky}(beta) s_{l,msky}
    (appendix eq. pithetasym inside eq. convdef)."""
    L, M, n = 30, 4, 10
    xr = rings(n)
    alm = random_sky(L, 8)
    blm = S.random_beam(L, M, 9)
    C = orc.totalconv_fwd(L, M, xr, alm, blm)
    sg = sky_get(alm, L)
    lsign = (-1.0) ** np.arange(L + 1)
    for mb in range(-M, M + 1):
        for ms in (0, 3, 11, 30):
            d = orc.wigner_d(L, [mb], [ms], xr)[0]          # (L+1, n)
            w = np.array([np.conj(blm[-mb + M, l]) * sg(l, ms) for l in range(L + 1)])
            pair = ((w * lsign * (-1.0) ** ms)[:, None] * d).sum(axis=0)
            np.testing.assert_allclose(C[-mb + M, ms, ::-1], pair, atol=2e-15, rtol=0)


def test_linearity(orc):
    L, M, n = 25, 3, 6
    xr = rings(n)
    a1, a2 = random_sky(L, 1), random_sky(L, 2)
    b1, b2 = S.random_beam(L, M, 1), S.random_beam(L, M, 2)
    lam = 0.7 - 1.3j
    f = lambda a, b: orc.totalconv_fwd(L, M, xr, a, b)
    np.testing.assert_allclose(f(a1 + lam * a2, b1), f(a1, b1) + lam * f(a2, b1), atol=1e-14)
    np.testing.assert_allclose(f(a1, b1 + lam * b2), f(a1, b1) + np.conj(lam) * f(a1, b2), atol=1e-14)


def test_ring_and_column_selection(orc):
    """Sampled columns and rings equal the corresponding slice of the full result."""
    L, M, n = 33, 5, 17
    xr = rings(n)
    alm, blm = S.sky_alm(L, 2), S.beam_blm(L, M, 100.0, 0.2)
    full = orc.totalconv_fwd(L, M, xr, alm, blm)
    cols = (np.array([-5, 0, 3, 5], np.int32), np.array([33, 0, 7, 2], np.int32))
    sel = np.array([16, 0, 5], np.int32)
    part = orc.totalconv_fwd(L, M, xr, alm, blm, cols=cols, rings=sel)
    for i in range(4):
        np.testing.assert_array_equal(part[i], full[cols[0][i] + M, cols[1][i], sel])


def test_eps_skip_bound(orc):
    """The paper's accumulation skip (Sec. 4.2.1): neglecting d below eps before its first
    crossing changes C by at most eps * sum_l |w_l|."""
    L, M, n = 200, 4, 64
    xr = rings(n)
    alm, blm = S.sky_alm(L, 4), S.beam_blm(L, M, 60.0, 0.2)
    full = orc.totalconv_fwd(L, M, xr, alm, blm)
    eps = 1e-30
    skip = orc.totalconv_fwd(L, M, xr, alm, blm, eps=eps)
    bound = eps * np.abs(blm).sum(axis=1).max() * np.abs(alm).max() * (L + 1)
    assert np.max(np.abs(skip - full)) <= bound
    eps = 1e-3
    skip = orc.totalconv_fwd(L, M, xr, alm, blm, eps=eps)
    assert np.max(np.abs(skip - full)) > 0     # the switch does something


# ------------------------------------------------------------------ adjoint

def _inner(u, v):
    return np.vdot(u.ravel(), v.ravel())


def test_adjoint_dot_product(orc):
    """Re<C(s), G> = Re<s, sky_bar(G)> and Re<C(b), G> = Re<b, beam_bar(G)>."""
    L, M, n = 28, 4, 11
    xr = rings(n)
    alm = random_sky(L, 21)
    blm = S.random_beam(L, M, 22)
    G = S.random_cbar(L, M, n, 23)
    C = orc.totalconv_fwd(L, M, xr, alm, blm)
    sky_bar, beam_bar = orc.totalconv_adj(L, M, xr, alm, blm, G)
    lhs = _inner(G, C)
    assert abs(lhs - _inner(sky_bar, alm)) <= 1e-13 * abs(lhs)
    assert abs(lhs.real - _inner(blm, beam_bar).real) <= 1e-13 * abs(lhs)
    # C is antilinear in b: <G, C> = sum conj(b) . beam_bar (conjugated inner product)
    assert abs(lhs - np.sum(np.conj(blm) * beam_bar)) <= 1e-13 * abs(lhs)


def test_adjoint_central_differences(orc):
    """L = 0.5 ||C - T||^2 is quadratic in each coefficient, so central differences equal the
    gradient up to rounding (PyTorch convention: grad = dL/dRe + i dL/dIm)."""
    L, M, n = 16, 2, 9
    xr = rings(n)
    alm = random_sky(L, 31)
    blm = S.random_beam(L, M, 32)
    T = orc.totalconv_fwd(L, M, xr, random_sky(L, 33), blm)
    loss = lambda a, b: 0.5 * np.sum(np.abs(orc.totalconv_fwd(L, M, xr, a, b) - T) ** 2)
    G = orc.totalconv_fwd(L, M, xr, alm, blm) - T
    sky_bar, beam_bar = orc.totalconv_adj(L, M, xr, alm, blm, G)
    rng = np.random.Generator(np.random.PCG64(7))
    h = 1e-3
    gmax = max(np.abs(sky_bar).max(), np.abs(beam_bar).max())
    for k in rng.choice(alm.size, 12, replace=False):
        for unit in (1.0, 1j):
            da = np.zeros_like(alm)
            da[k] = h * unit
            fd = (loss(alm + da, blm) - loss(alm - da, blm)) / (2 * h)
            g = sky_bar[k].real if unit == 1.0 else sky_bar[k].imag
            assert abs(fd - g) <= 1e-9 * gmax
    for _ in range(12):
        r, l = int(rng.integers(0, 2 * M + 1)), int(rng.integers(0, L + 1))
        if l < abs(r - M):
            continue
        for unit in (1.0, 1j):
            db = np.zeros_like(blm)
            db[r, l] = h * unit
            fd = (loss(alm, blm + db) - loss(alm, blm - db)) / (2 * h)
            g = beam_bar[r, l].real if unit == 1.0 else beam_bar[r, l].imag
            assert abs(fd - g) <= 1e-9 * gmax


def test_adjoint_brute_force_tiny(orc):
    """sky_bar and beam_bar from their definitions with explicit-sum d (mpmath)."""
    mp.mp.dps = 30
    from oracle import mpref
    L, M, n = 6, 2, 4
    xr = rings(n)
    x = xr
    alm = random_sky(L, 41)
    blm = S.random_beam(L, M, 42)
    G = S.random_cbar(L, M, n, 43)
    sky_bar, beam_bar = orc.totalconv_adj(L, M, xr, alm, blm, G)
    sg = sky_get(alm, L)
    dd = {}
    for mb in range(-M, M + 1):
        for ms in range(0, L + 1):
            for l in range(max(abs(mb), ms), L + 1):
                for j in range(n):
                    dd[(l, mb, ms, j)] = complex(mpref.d_explicit(l, mb, ms, None, x=x[j]))
    for ms in range(L + 1):
        for l in range(ms, L + 1):
            ref = sum(blm[mb + M, l] * dd.get((l, mb, ms, j), 0.0) * G[mb + M, ms, j]
                      for mb in range(-M, M + 1) for j in range(n))
            assert abs(sky_bar[S.alm_index(L, l, ms)] - ref) <= 1e-14
    for mb in range(-M, M + 1):
        for l in range(L + 1):
            ref = sum(sg(l, ms) * dd.get((l, mb, ms, j), 0.0) * np.conj(G[mb + M, ms, j])
                      for ms in range(0, l + 1) for j in range(n))
            assert abs(beam_bar[mb + M, l] - ref) <= 1e-14


def test_invalid_conv_arguments(orc):
    xr = rings(3)
    with pytest.raises(ValueError):
        orc.totalconv_fwd(4, 5, xr, S.sky_alm(4, 1), np.zeros((11, 5), complex))
    with pytest.raises(ValueError):
        orc.totalconv_fwd(4, 1, xr, S.sky_alm(4, 1), np.zeros((3, 5), complex),
                          cols=(np.array([2], np.int32), np.array([0], np.int32)))


def test_polarised_pairs_against_brute_force(orc):
    """Footnote of Sec. 4.1: the polarised convolution is eq. convdef for each of the
    temperature, gradient and curl pairs.  Separate outputs and their sum against mpmath
    sums of explicit-sum d; the adjoint pairs against the dot-product identity."""
    mp.mp.dps = 40
    from oracle import mpref
    L, M, n = 7, 2, 5
    xr = rings(n)
    alms = [random_sky(L, 30 + p) for p in range(3)]
    blms = [S.random_beam(L, M, 40 + p) for p in range(3)]
    sep = orc.totalconv_fwd_pol(L, M, xr, alms, blms)
    tot = orc.totalconv_fwd_pol(L, M, xr, alms, blms, summed=True)
    assert len(sep) == 3 and len(tot) == 1
    worst = 0.0
    for mb in range(-M, M + 1):
        for ms in range(0, L + 1):
            for j in range(n):
                refs = [mpref.conv_brute(L, mb, ms, xr[j], sky_get(alms[p], L), beam_get(blms[p], M))
                        for p in range(3)]
                for p in range(3):
                    worst = max(worst, abs(sep[p][mb + M, ms, j] - refs[p]))
                worst = max(worst, abs(tot[0][mb + M, ms, j] - sum(refs)))
    assert worst <= 1e-14, worst
    # adjoint: <C(a, b), G> = <a, sky_bar> + (b-part) per pair, with the summed output's cotangent
    G = S.random_cbar(L, M, n, 50)
    sky_bar, beam_bar = orc.totalconv_adj_pol(L, M, xr, alms, blms, [G], summed=True)
    lhs = np.vdot(G, tot[0])                            # <G, C> = sum conj(G) C
    rhs = 0j
    for p in range(3):
        # C is complex-linear in s: <G, C(s)> = <sky_bar, s> restricted to the stored half-set
        rhs += np.vdot(sky_bar[p], alms[p])
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # conj-linear in b: <G, C> = sum conj(b) (s d conj(G)) = <b, beam_bar>
    rhs_b = sum(np.vdot(blms[p], beam_bar[p]) for p in range(3))
    assert abs(lhs - rhs_b) <= 1e-12 * abs(lhs)
