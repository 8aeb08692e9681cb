"""The growth bound the GPU walks rely on, checked from the recursion's coefficients.

The kernels take the step of Sec. 4.2.2, d^{l+1} = F0 (x - F1) d^l - F2 d^{l-1}, with the closed
forms F0 = (l+1)(2l+1) / sqrt(((l+1)^2 - mb^2)((l+1)^2 - msky^2)), F1 = mb msky / (l (l+1)) and
F2 = (l+1) sqrt((l^2 - mb^2)(l^2 - msky^2)) / (l sqrt(((l+1)^2 - mb^2)((l+1)^2 - msky^2))), on the
normalised values e^l = c_l d^l with c_{l0} = c_{l0+1} = 1 and c_{l+1} = c_{l-1} / F2_l, so that a
step reads e^{l+1} = alpha_l F0 (x - F1) e^l - e^{l-1} with alpha_l = c_{l+1} / c_l.  For |x| <= 1
it multiplies max(|e^l|, |e^{l-1}|) by at most alpha F0 (1 + |F1|) + 1.  The skip test (a chain
below 2^-100 / 2^(17*8) cannot reach 2^-100 within 8 steps) and the rescale period of scaled
chains (32 steps: a significand below 1 stays below 2^544) both assume this factor is below 2^17
for every l <= 16384, and the skip tests on e assume c_l >= 1; the paper's coefficients are
evaluated here on a grid that holds the extreme columns (|mb| or msky equal to l0, and the two
equal) at every l.
"""
import numpy as np


def coefficients(l, mb, ms):
    l = l.astype(np.float64)
    l1 = l + 1.0
    b2, s2 = float(mb) ** 2, float(ms) ** 2
    den = np.sqrt(l1 * l1 - b2) * np.sqrt(l1 * l1 - s2)
    F0 = l1 * (2.0 * l + 1.0) / den
    F1 = np.where(l > 0, mb * ms / np.maximum(l * l1, 1.0), 0.0)
    F2 = np.where(l > 0, l1 * np.sqrt(np.maximum(l * l - b2, 0.0)) * np.sqrt(np.maximum(l * l - s2, 0.0))
                  / (np.maximum(l, 1.0) * den), 0.0)
    return F0, F1, F2


def growth_factor(l, mb, ms):
    """Factor of one step of the plain recursion."""
    F0, F1, F2 = coefficients(l, mb, ms)
    return F0 * (1.0 + np.abs(F1)) + F2


def normalisation(l, mb, ms):
    """c_l for l = l0 .. l0 + len(l) and alpha_l = c_{l+1} / c_l, l = l0 ..: c_{l+1} = c_{l-1} / F2_l."""
    _, _, F2 = coefficients(l, mb, ms)
    c = np.ones(l.size + 1)
    for i in range(1, l.size):
        c[i + 1] = c[i - 1] / F2[i]
    return c, c[1:] / c[:-1]


def columns(lmax):
    """(mb, msky) pairs with their own l0: the extremes at several sizes, and a seeded spread."""
    rng = np.random.Generator(np.random.PCG64(16384))
    out = [(0, 0), (0, lmax), (lmax, lmax), (-lmax, lmax), (14, 14), (-14, 14), (14, 0), (1, 1)]
    for m in (2, 17, 255, 1024, 4096, 8191):
        if m <= lmax:
            out += [(m, m), (-m, m), (0, m), (m, 0), (m, lmax), (min(16, m), m)]
    for _ in range(40):
        ms = int(rng.integers(0, lmax + 1))
        mb = int(rng.integers(-min(ms, 32), min(ms, 32) + 1)) if ms else 0
        out.append((mb, ms))
    return out


def test_step_growth_below_2l_plus_4():
    lmax = 16384
    worst = 0.0
    for mb, ms in columns(lmax):
        l0 = max(abs(mb), ms)
        l = np.arange(l0, lmax, dtype=np.int64)    # the step at l = lmax is switched off
        if l.size == 0:
            continue
        g = growth_factor(l, mb, ms)
        assert np.all(np.isfinite(g))
        assert np.all(g <= 2.0 * l + 4.0), (mb, ms, float(np.max(g - (2.0 * l + 4.0))))
        worst = max(worst, float(np.max(g)))
    assert worst < 2.0 ** 16


def test_normalised_step_growth_below_2_pow_17():
    """F2_l < 1 (so c_l >= 1: a skip test on e is conservative), alpha_l <= 2, and a step of the
    normalised walk grows max(|e^l|, |e^{l-1}|) by at most alpha F0 (1 + |F1|) + 1 < 2^17."""
    lmax = 16384
    worst_alpha, worst = 0.0, 0.0
    for mb, ms in columns(lmax):
        l0 = max(abs(mb), ms)
        l = np.arange(l0, lmax, dtype=np.int64)
        if l.size < 2:
            continue
        F0, F1, F2 = coefficients(l, mb, ms)
        assert np.all(F2[1:] < l[1:] / (l[1:] + 1.0) * (1 + 1e-15)), (mb, ms)
        c, alpha = normalisation(l, mb, ms)
        assert np.all(c >= 1.0) and np.all(np.isfinite(c)), (mb, ms)
        g = alpha * F0 * (1.0 + np.abs(F1)) + 1.0
        worst_alpha = max(worst_alpha, float(alpha.max()))
        worst = max(worst, float(g.max()))
    assert worst_alpha <= 2.0 * (1 + 1e-12)
    assert worst < 2.0 ** 17


def test_growth_bound_is_reached_in_order_of_magnitude():
    """The bound is not vacuous: at l = l0 of a column with mb = msky = l0 the first factor is
    l0 + 1 (F1 ~ 1 makes the step's factor about 2 l0), so the 16 bits per step are needed."""
    l0 = 16000
    g = growth_factor(np.array([l0]), l0, l0)[0]
    assert 1.5 * l0 < g <= 2.0 * l0 + 4.0


def test_rescale_period_margins():
    """The kernels' constants: 17 bits per step over a 32-step rescale period stays below the
    double range, and a chain left below 2^-900 stays 2^136 (one 8-step skip block) under 2^-100."""
    bits, rs, ts, fold, skip = 17, 32, 8, -900, 100
    assert bits * rs < 1023
    assert fold + bits * rs + bits * ts <= -skip
