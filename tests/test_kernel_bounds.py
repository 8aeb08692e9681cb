"""The growth bound the GPU walks rely on, checked from the recursion's coefficients.

The kernels take the step of Sec. 4.2.2, d^{l+1} = F0 (x - F1) d^l - F2 d^{l-1}, with the closed
forms F0 = (l+1)(2l+1) / sqrt(((l+1)^2 - mb^2)((l+1)^2 - msky^2)), F1 = mb msky / (l (l+1)) and
F2 = (l+1) sqrt((l^2 - mb^2)(l^2 - msky^2)) / (l sqrt(((l+1)^2 - mb^2)((l+1)^2 - msky^2))).
For |x| <= 1 a step multiplies max(|d^l|, |d^{l-1}|) by at most max(1, F0 (1 + |F1|) + F2).  The
skip test (a chain below 2^-100 / 2^(16*8) cannot reach 2^-100 within 8 steps) and the rescale
period of scaled chains (32 steps: a significand below 1 stays below 2^512) both assume this factor
is below 2l + 4 < 2^16 for every l <= 16384; the paper's coefficients are evaluated here on a grid
that holds the extreme columns (|mb| or msky equal to l0, and the two equal) at every l.
"""
import numpy as np


def growth_factor(l, mb, ms):
    l = l.astype(np.float64)
    l1 = l + 1.0
    b2, s2 = float(mb) ** 2, float(ms) ** 2
    den = np.sqrt(l1 * l1 - b2) * np.sqrt(l1 * l1 - s2)
    F0 = l1 * (2.0 * l + 1.0) / den
    F1 = np.where(l > 0, mb * ms / np.maximum(l * l1, 1.0), 0.0)
    F2 = np.where(l > 0, l1 * np.sqrt(np.maximum(l * l - b2, 0.0)) * np.sqrt(np.maximum(l * l - s2, 0.0))
                  / (np.maximum(l, 1.0) * den), 0.0)
    return F0 * (1.0 + np.abs(F1)) + F2


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


def test_growth_bound_is_reached_in_order_of_magnitude():
    """The bound is not vacuous: at l = l0 of a column with mb = msky = l0 the first factor is
    l0 + 1 (F1 ~ 1 makes the step's factor about 2 l0), so the 16 bits per step are needed."""
    l0 = 16000
    g = growth_factor(np.array([l0]), l0, l0)[0]
    assert 1.5 * l0 < g <= 2.0 * l0 + 4.0


def test_rescale_period_margins():
    """The kernels' constants: 16 bits per step over a 32-step rescale period stays below the
    double range, and a chain left below 2^-900 stays 2^128 (one 8-step skip block) under 2^-100."""
    bits, rs, ts, fold, skip = 16, 32, 8, -900, 100
    assert bits * rs < 1023
    assert fold + bits * rs + bits * ts <= -skip
