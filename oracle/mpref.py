"""Extended-precision textbook definitions used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  These are independent of
the l-recursion: they evaluate reduced Wigner elements straight from closed
forms with mpmath at high precision.

* ``d_explicit``: Wigner's explicit finite sum in the convention
  d^l_{m m'}(beta) = <l m| exp(-i beta J_y) |l m'> (Sec. 2, eq. reducedwignerdef):
      d^l_{m,m'} = sum_k (-1)^(m - m' + k)
                   sqrt((l+m)! (l-m)! (l+m')! (l-m')!)
                   / ((l+m'-k)! k! (m-m'+k)! (l-m-k)!)
                   c^(2l + m' - m - 2k) s^(m - m' + 2k),
  c = cos(beta/2), s = sin(beta/2).  Exact but cancelling: fine for l <= ~60 at
  50 digits.
* ``d_jacobi``: the Jacobi-polynomial form, valid for m' >= |m|:
      d^l_{m,m'} = sqrt((l+m')! (l-m')! / ((l+m)! (l-m)!)) s^(m'-m) c^(m'+m)
                   P^{(m'-m, m'+m)}_{l-m'}(cos beta)
  (mpmath evaluates the hypergeometric series exactly at working precision),
  for spot checks at large l.
* ``d_legendre``: d^l_{m,0} = sqrt((l-m)!/(l+m)!) P_l^m(cos beta) for m >= 0
  (mpmath ``legenp`` includes the Condon-Shortley phase).
"""

from __future__ import annotations

import mpmath as mp


def _cs(beta):
    b = mp.mpf(beta) / 2
    return mp.cos(b), mp.sin(b)


def d_explicit(l: int, m: int, mp_: int, beta, x=None):
    """Wigner's explicit sum.  If x is given, the ring is defined by x = cos(beta)."""
    if abs(m) > l or abs(mp_) > l:
        return mp.mpf(0)
    if x is not None:
        X = mp.mpf(x)
        c, s = mp.sqrt((1 + X) / 2), mp.sqrt((1 - X) / 2)
    else:
        c, s = _cs(beta)
    f = mp.factorial
    pre = mp.sqrt(f(l + m) * f(l - m) * f(l + mp_) * f(l - mp_))
    total = mp.mpf(0)
    kmin = max(0, mp_ - m)
    kmax = min(l + mp_, l - m)
    for k in range(kmin, kmax + 1):
        num = (-1) ** (m - mp_ + k)
        den = f(l + mp_ - k) * f(k) * f(m - mp_ + k) * f(l - m - k)
        pc = 2 * l + mp_ - m - 2 * k
        ps = m - mp_ + 2 * k
        term = num * (c ** pc if pc else mp.mpf(1)) * (s ** ps if ps else mp.mpf(1)) / den
        total += term
    return pre * total


def d_jacobi(l: int, m: int, mp_: int, x):
    """Jacobi form for mp_ >= |m|; the ring is given by x = cos(beta)."""
    if not mp_ >= abs(m):
        raise ValueError("d_jacobi needs m' >= |m|")
    if l < mp_:
        return mp.mpf(0)
    X = mp.mpf(x)
    c, s = mp.sqrt((1 + X) / 2), mp.sqrt((1 - X) / 2)
    f = mp.factorial
    pre = mp.sqrt(f(l + mp_) * f(l - mp_) / (f(l + m) * f(l - m)))
    a, b = mp_ - m, mp_ + m
    pa = s ** a if a else mp.mpf(1)
    pb = c ** b if b else mp.mpf(1)
    n = l - mp_
    if X < 0:   # P_n^{(a,b)}(-x) = (-1)^n P_n^{(b,a)}(x): keeps the series argument small
        poly = (-1) ** n * mp.jacobi(n, b, a, -X, maxprec=60000)
    else:
        poly = mp.jacobi(n, a, b, X, maxprec=60000)
    return pre * pa * pb * poly


def d_legendre(l: int, m: int, x):
    """d^l_{m,0} from the associated Legendre function, m >= 0."""
    X = mp.mpf(x)
    f = mp.factorial
    return mp.sqrt(f(l - m) / f(l + m)) * mp.legenp(l, m, X)


def sph_harm_theta(l: int, m: int, theta):
    """Y_lm(theta, phi=0) from mpmath (Condon-Shortley phase)."""
    return mp.spherharm(l, m, mp.mpf(theta), 0)


def conv_brute(lmax, mb, msky, beta_x, alm_get, blm_get):
    """C_{mb,msky} = sum_l conj(b_{l,mb}) d^l_{mb,msky} s_{l,msky}, every d from the
    explicit sum at the ring x = beta_x.  alm_get(l, m) and blm_get(l, mb) return
    Python complex numbers."""
    total = mp.mpc(0)
    for l in range(max(abs(mb), abs(msky)), lmax + 1):
        d = d_explicit(l, mb, msky, None, x=beta_x)
        total += mp.conj(mp.mpc(blm_get(l, mb))) * d * mp.mpc(alm_get(l, msky))
    return complex(total)


def d_jacobi_any(l: int, m: int, mp_: int, x):
    """Jacobi form for any (m, m'), mapped onto m' >= |m| with the symmetries
    d_{m,m'} = (-1)^(m-m') d_{m',m} = (-1)^(m-m') d_{-m,-m'} = d_{-m',-m}
    (appendix, eq. mmsym and the two lines after it)."""
    am, amp = abs(m), abs(mp_)
    if mp_ >= am:
        return d_jacobi(l, m, mp_, x)
    if m >= amp:
        return (-1) ** (m - mp_) * d_jacobi(l, mp_, m, x)
    if -mp_ >= am:
        return (-1) ** (m - mp_) * d_jacobi(l, -m, -mp_, x)
    return d_jacobi(l, -mp_, -m, x)
