"""Pins for the oracle's reduced Wigner elements (CPU only).

Each check compares the oracle's l-recursion with something it does not share
code or formulas with: Wigner's explicit sum and the Jacobi form in mpmath,
closed forms from the paper (Sec. 3.2 seeds, Sec. 4.2.1 d(0) = delta), the
symmetries of the appendix, unitarity, the Legendre and spherical-harmonic
special cases (Sec. 2 eq. dl00, Sec. 4), and the qualitative facts stated with
Fig. 1 (Sec. 2).
"""
import collections
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rings(n):
    return np.pi * (np.arange(n) + 0.5) / n


# --------------------------------------------------------------- explicit sum

PAIRS = [(0, 0), (0, 1), (1, 0), (3, 1), (-3, 1), (2, 5), (-2, 5), (4, -6), (-7, 3), (7, 3),
         (5, 5), (-5, 5), (5, -5), (0, -4), (-6, -6), (9, -9), (-1, -8), (8, 2)]


def test_explicit_sum_small_l(orc):
    """Oracle vs Wigner's explicit sum (mpmath, 50 digits) for l <= 40, including the poles
    (the -infinity rule) and beta = pi/2."""
    mp.mp.dps = 50
    from oracle import mpref
    beta = np.array([0.0, 1e-3, 0.3, 0.7, math.pi / 2, 2.0, 2.9, math.pi - 1e-3, math.pi])
    x = orc.ring_x(beta)
    mb = [p[0] for p in PAIRS]
    ms = [p[1] for p in PAIRS]
    d = orc.wigner_d(40, mb, ms, x)
    worst = 0.0
    for i, (a, b) in enumerate(PAIRS):
        for j in range(beta.size):
            for l in range(41):
                ref = float(mpref.d_explicit(l, a, b, None, x=x[j]))
                worst = max(worst, abs(d[i, l, j] - ref))
    assert worst <= 2.3e-16, worst   # one ulp at |d| ~ 1 (both sides round to double)


def test_explicit_sum_many_columns(orc):
    """Every (m, m') with |m|, |m'| <= 12 at l <= 24 on three rings."""
    mp.mp.dps = 40
    from oracle import mpref
    beta = np.array([0.11, 1.3, 2.7])
    x = orc.ring_x(beta)
    pairs = [(a, b) for a in range(-12, 13, 3) for b in range(-12, 13, 2)]
    d = orc.wigner_d(24, [p[0] for p in pairs], [p[1] for p in pairs], x)
    worst = 0.0
    for i, (a, b) in enumerate(pairs):
        for j in range(3):
            for l in range(max(abs(a), abs(b)), 25, 3):
                worst = max(worst, abs(d[i, l, j] - float(mpref.d_explicit(l, a, b, None, x=x[j]))))
    assert worst <= 2.3e-16, worst   # one ulp at |d| ~ 1 (both sides round to double)


def test_zero_below_l0(orc):
    d = orc.wigner_d(30, [3, -7, 0], [10, 2, -5], orc.ring_x(rings(7)))
    assert np.all(d[0, :10] == 0) and np.all(d[1, :7] == 0) and np.all(d[2, :5] == 0)
    assert np.all(d[0, 10] != 0)


# --------------------------------------------------------------- closed forms

def test_diagonal_seed_closed_form(orc):
    """d^l_{ll}(beta) = cos^{2l}(beta/2) (Sec. 3.2, eq. ini1 with m = l)."""
    beta = rings(33)
    x = orc.ring_x(beta).astype(np.longdouble)
    c2 = (1 + x) / 2
    for l in (0, 1, 5, 60, 700):
        d = orc.wigner_d(l, [l], [l], orc.ring_x(beta))[0, l]
        ref = (c2 ** l).astype(np.float64)
        np.testing.assert_allclose(d, ref, rtol=2.3e-16, atol=0)   # one ulp: both round to double


def test_identity_at_beta_zero(orc):
    """d^l_{m m'}(0) = delta_{m m'} (Sec. 4.2.1); exercises the zero-base rule."""
    pairs = [(a, b) for a in range(-6, 7) for b in range(-6, 7)]
    d = orc.wigner_d(50, [p[0] for p in pairs], [p[1] for p in pairs], np.array([1.0]))
    for i, (a, b) in enumerate(pairs):
        l0 = max(abs(a), abs(b))
        expect = 1.0 if a == b else 0.0
        assert np.all(d[i, l0:, 0] == expect), (a, b)


def test_legendre_special_cases(orc):
    """d^l_{00} = P_l(x) (Sec. 2, eq. dl00 is Bonnet's recursion) and
    d^l_{m0} = sqrt((l-m)!/(l+m)!) P_l^m(x) at large l."""
    mp.mp.dps = 40
    from oracle import mpref
    beta = np.array([0.004, 0.9, 1.6, 3.1])
    x = orc.ring_x(beta)
    L = 1500
    d = orc.wigner_d(L, [0, 5, 12], [0, 0, 0], x)
    for j in range(beta.size):
        for l in (0, 1, 2, 77, 1499, 1500):
            assert abs(d[0, l, j] - float(mp.legendre(l, mp.mpf(x[j])))) <= 2e-15
        for i, m in ((1, 5), (2, 12)):
            for l in (m, m + 1, 400, 1500):
                assert abs(d[i, l, j] - float(mpref.d_legendre(l, m, x[j]))) <= 2e-15


def test_spherical_harmonic_relation(orc):
    """Y_lm(theta, 0) = (-1)^m sqrt((2l+1)/(4 pi)) d^l_{0m}(theta) (Sec. 4, with D = d at
    alpha = gamma = 0)."""
    mp.mp.dps = 30
    theta = np.array([0.25, 1.1, 2.4])
    x = orc.ring_x(theta)
    th = [mp.acos(mp.mpf(v)) for v in x]      # the ring's exact colatitude
    ms = [0, 1, 4, 9]
    d = orc.wigner_d(30, [0] * len(ms), ms, x)
    for i, m in enumerate(ms):
        for l in range(m, 31, 4):
            for j in range(3):
                y = mp.spherharm(l, m, th[j], 0)
                ref = float(mp.re(y)) / ((-1) ** m * math.sqrt((2 * l + 1) / (4 * math.pi)))
                assert abs(d[i, l, j] - ref) <= 1e-15


# --------------------------------------------------------------- symmetries

def test_appendix_symmetries(orc):
    """d_{m m'} = (-1)^{m-m'} d_{-m,-m'} = (-1)^{m-m'} d_{m' m} = d_{-m',-m}  (appendix)."""
    beta = orc.ring_x(rings(11))
    L = 120
    base = [(3, 1), (-4, 9), (10, -2), (0, 7), (-5, -5), (6, 6), (13, -13)]
    mb, ms = [], []
    for a, b in base:
        mb += [a, -a, b, -b]
        ms += [b, -b, a, -a]
    d = orc.wigner_d(L, mb, ms, beta)
    for k, (a, b) in enumerate(base):
        s = (-1) ** (a - b)
        d0, d1, d2, d3 = d[4 * k], d[4 * k + 1], d[4 * k + 2], d[4 * k + 3]
        assert np.max(np.abs(d0 - s * d1)) <= 1e-15
        assert np.max(np.abs(d0 - s * d2)) <= 1e-15
        assert np.max(np.abs(d0 - d3)) <= 1e-15


def test_pi_minus_beta(orc):
    """d^l_{m m'}(pi - beta) = (-1)^{l-m'} d^l_{-m,m'}(beta)  (appendix, eq. pithetasym)."""
    n = 40
    from paper_1002_1050_amd import synthetic as S
    beta = S.ring_cosines(n)                       # exactly mirror-symmetric: x[n-1-j] = -x[j]
    L = 60
    cols = [(2, 5), (-3, 1), (7, 7), (0, 0), (4, 0)]
    mb = [c[0] for c in cols] + [-c[0] for c in cols]
    ms = [c[1] for c in cols] * 2
    d = orc.wigner_d(L, mb, ms, beta)
    l = np.arange(L + 1)[:, None]
    for k, (a, b) in enumerate(cols):
        lhs = d[k][:, ::-1]                         # ring n-1-j is pi - beta_j
        rhs = ((-1.0) ** (l - b)) * d[len(cols) + k]
        rhs[: max(abs(a), abs(b))] = 0
        assert np.max(np.abs(lhs - rhs)) <= 1e-15


def test_row_orthonormality(orc):
    """sum_{m'} d^l_{m m'} d^l_{m'' m'} = delta_{m m''} (d is orthogonal)."""
    beta = np.array([0.37, 1.9])
    for l in (50, 333):
        mrows = [0, 3, -7, 20]
        mp_ = np.arange(-l, l + 1)
        mb = np.repeat(mrows, mp_.size)
        ms = np.tile(mp_, len(mrows))
        d = orc.wigner_d(l, mb, ms, orc.ring_x(beta))[:, l, :].reshape(len(mrows), mp_.size, beta.size)
        for j in range(beta.size):
            g = d[:, :, j] @ d[:, :, j].T
            np.testing.assert_allclose(g, np.eye(len(mrows)), atol=5e-15)


# --------------------------------------------------------------- large l

def test_jacobi_form_large_l(orc):
    """Oracle vs the Jacobi closed form (40 digits) at lmax 1024, 4096 and 8192, on rings at
    the poles, quarter points and the equator, including values far below the double range
    (compared as significand and exponent)."""
    with open(os.path.join(GOLDEN, "jacobi_large_l.json")) as f:
        doc = json.load(f)
    groups = collections.defaultdict(list)
    for p in doc["points"]:
        groups[(p["lmax"], p["mb"], p["msky"])].append(p)
    worst_abs = 0.0
    worst_rel_tiny = 0.0
    for (L, mb, ms), pts in groups.items():
        rr = sorted({p["ring"] for p in pts})
        nring = pts[0]["nring"]
        beta = np.pi * (np.array(rr, dtype=np.float64) + 0.5) / nring
        x = orc.ring_x(beta)
        mant, ex = orc.wigner_d(L, [mb], [ms], x, split=True)
        for p in pts:
            j = rr.index(p["ring"])
            assert float.fromhex(p["x"]) == x[j]
            ref = mp.mpf(p["d"])
            got = mp.ldexp(mp.mpf(float(mant[0, p["l"], j])), int(ex[0, p["l"], j]))
            err = abs(got - ref)
            worst_abs = max(worst_abs, float(err))
            if ref != 0 and abs(ref) < mp.mpf("1e-30"):
                worst_rel_tiny = max(worst_rel_tiny, float(err / abs(ref)))
    assert worst_abs <= 2e-14, worst_abs
    assert worst_rel_tiny <= 3e-14, worst_rel_tiny


# --------------------------------------------------------------- Fig. 1

def _first_peak_after(vals, start):
    for i in range(start + 1, len(vals) - 1):
        if vals[i] >= vals[i - 1] and vals[i] >= vals[i + 1]:
            return i
    return None


def test_fig1_l_transition(orc):
    """Sec. 2 / Fig. 1 top: d^l_{0,10}(0.0996687) turns classical at l = 100 and its tallest
    peak is the first one after the transition; below l = 100 it is exponentially small."""
    d = np.abs(orc.wigner_d(500, [0], [10], orc.ring_x([0.0996687]))[0, :, 0])
    lt = 0.5 * (math.sqrt(1 + 4 * 10 ** 2 / math.sin(0.0996687) ** 2) - 1)   # eq. classiccond
    assert abs(lt - 100) < 0.5
    arg = int(np.argmax(d[10:])) + 10
    assert arg == _first_peak_after(d, 100)
    assert 100 < arg < 130
    assert d[15] < 1e-7 * d[arg] and d[50] < 1e-2 * d[arg]   # monotone growth below l = 100
    assert np.all(np.diff(d[10:90]) > 0)


def test_fig1_m_transition(orc):
    """Sec. 2 / Fig. 1 middle: d^{1000}_{0,m'}(0.52331) turns non-classical at m' = 500 (the
    text's l = 1000); the tallest peak is the last one before m' = 500, and |d| decays
    quickly above it."""
    ms = np.arange(0, 1001)
    d = np.abs(orc.wigner_d(1000, np.zeros_like(ms), ms, orc.ring_x([0.52331]))[:, 1000, 0])
    mt = math.sin(0.52331) * math.sqrt(1000 * 1001)       # eq. classiccondm0
    assert abs(mt - 500) < 0.5
    arg = int(np.argmax(d))
    peaks = [m for m in range(1, 1000) if d[m] >= d[m - 1] and d[m] >= d[m + 1]]
    assert arg == max(p for p in peaks if p <= 500)
    assert 470 < arg <= 500
    assert d[600] < 1e-10 * d[arg]


def test_fig1_beta_transition(orc):
    """Sec. 2 / Fig. 1 bottom: d^{100}_{0,71}(beta) turns classical at beta = pi/4; the tallest
    peak on (0, pi/2] is the first one after it."""
    beta = np.linspace(math.pi / 2 / 2000, math.pi / 2, 2000)
    d = np.abs(orc.wigner_d(100, [0], [71], orc.ring_x(beta))[0, 100, :])
    bt = math.asin(71 / math.sqrt(100 * 101))
    assert abs(bt - math.pi / 4) < 2e-3
    arg = int(np.argmax(d))
    it = int(np.searchsorted(beta, bt))
    assert arg == _first_peak_after(d, it)
    assert math.pi / 4 < beta[arg] < math.pi / 4 + 0.1
    assert d[it // 2] < 1e-6 * d[arg]


# --------------------------------------------------------------- argument checks

def test_invalid_arguments(orc):
    with pytest.raises(ValueError):
        orc.wigner_d(5, [6], [0], np.array([0.1]))
    with pytest.raises(ValueError):
        orc.wigner_d(5, [0], [0], np.array([1.5]))     # |x| > 1 is not a ring
    with pytest.raises(ValueError):
        orc.wigner_d(5, [0], [-6], np.array([0.1]))


# ------------------------------------------------------------------- ring definition

def test_ring_x_is_cos_rounded_once(orc):
    """oracle.ring_x(beta) = cos(beta) rounded once to double (the ring definition x_j of the
    boundary; Sec. 4.2.2 precomputes cos(beta) per ring).  Reference: mpmath cos at 50 digits,
    rounded to nearest.  The oracle evaluates cosl in x87 long double and rounds that to double,
    so it may differ from the correctly rounded value only where the exact cosine lies within
    half a long-double ulp of a midpoint between two doubles (double rounding); any other
    difference is an error."""
    mp.mp.dps = 50
    rng = np.random.Generator(np.random.PCG64(1050))
    beta = np.concatenate([
        [0.0, np.pi, np.pi / 2, np.nextafter(np.pi, 0.0), np.nextafter(0.0, 1.0), 1e-300, 1e-9,
         np.pi - 1e-9, np.nextafter(np.pi / 2, 0.0), np.nextafter(np.pi / 2, 4.0)],
        rings(7), rings(64), rings(1025),
        rng.uniform(0.0, np.pi, 3000),
        rng.uniform(0.0, 1e-4, 200), np.pi - rng.uniform(0.0, 1e-4, 200),
        np.pi / 2 + rng.uniform(-1e-6, 1e-6, 200)])
    x = orc.ring_x(beta)
    mism = 0
    for b, xv in zip(beta, x):
        exact = mp.cos(mp.mpf(float(b)))
        cr = float(exact)                       # mpmath -> float rounds to nearest
        if xv == cr:
            continue
        mism += 1
        # double rounding only: the exact value sits within 2^-64 |x| of the midpoint
        assert abs(np.nextafter(cr, xv) - xv) == 0.0 or abs(xv - cr) <= abs(np.nextafter(cr, xv) - cr)
        mid = (mp.mpf(float(cr)) + mp.mpf(float(xv))) / 2
        assert abs(exact - mid) <= mp.mpf(2) ** -64 * abs(exact), (b, xv, cr)
    assert mism <= 3, f"{mism} double-rounding cases out of {beta.size}"
