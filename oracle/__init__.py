"""CPU oracle for the reduced-Wigner l-recursion and the total convolution.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product package never does.  The
arithmetic lives in ``totalconv_oracle.c`` (x87 long double, OpenMP); this
module builds it with gcc, loads it with ctypes and forms the two gradients
from the per-column sums u_l with numpy long doubles.

Functions follow Prezeau & Reinecke (arXiv:1002.1050): Sec. 3.2 (seeds and the
l-recursion with scaled values), Sec. 4.1 eq. convdef (the sum over l) and
Sec. 4.2.2 (the F0/F1/F2 form of the recursion).  The adjoint is the exact
transpose of that sum: with G = dL/dconj(C),
    sky_bar_{l,msky} = sum_{mb,j} b_{l,mb} d^l_{mb,msky}(beta_j) G_{mb,msky,j}
    beam_bar_{l,mb}  = sum_{msky,j} s_{l,msky} d^l_{mb,msky}(beta_j) conj(G_{mb,msky,j}).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "totalconv_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle_totalconv.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, IEEE semantics)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            I = ctypes.c_int
            lib.oracle_wigner_d.argtypes = [I, I, P, P, I, P, P, P, P, I]
            lib.oracle_totalconv_fwd.argtypes = [I, I, I, P, P, P, I, P, P, I, P, ctypes.c_double, P, I]
            lib.oracle_totalconv_u.argtypes = [I, I, I, P, P, I, P, P, P, I]
            lib.oracle_ring_x.argtypes = [I, P, P]
            lib.oracle_ring_grid_x.argtypes = [I, P, P]
            lib.oracle_ring_grid_x.restype = ctypes.c_int
            lib.oracle_datacube.argtypes = [I, I, I, P, I, I, I, P, P, P, P, I]
            lib.oracle_datacube.restype = ctypes.c_int
            lib.oracle_max_threads.argtypes = []
            for f in (lib.oracle_wigner_d, lib.oracle_totalconv_fwd, lib.oracle_totalconv_u,
                      lib.oracle_ring_x, lib.oracle_max_threads):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def max_threads() -> int:
    return _load().oracle_max_threads()


def ring_x(beta) -> np.ndarray:
    """Rings from colatitudes: x_j = cos(beta_j) evaluated in long double, rounded once."""
    beta = _c(beta, np.float64)
    x = np.empty_like(beta)
    _load().oracle_ring_x(beta.size, _ptr(beta), _ptr(x))
    return x


def ring_grid_x(beta) -> np.ndarray:
    """Rings of a colatitude grid: ring_x of each colatitude, and for every pair j < k =
    nring-1-j whose colatitudes add up to pi to within 2^-48 the ring with the larger colatitude
    set to exactly minus the other's x (an exact mirror pair, Sec. 4.2.3)."""
    beta = _c(beta, np.float64)
    x = np.empty_like(beta)
    _load().oracle_ring_grid_x(beta.size, _ptr(beta), _ptr(x))
    return x


def wigner_d(lmax: int, mb, msky, xring, nthreads: int = 0, split: bool = False):
    """d^l_{mb[i],msky[i]}(beta_j) for l in [0, lmax]; shape (npair, lmax+1, nring).

    Ring j is given by xring[j] = cos(beta_j) (use ring_x to turn colatitudes into rings).

    With split=True returns (mant, ex) with d = mant * 2^ex, mant in [0.5, 1),
    which represents values far outside the double range exactly."""
    mb = _c(np.atleast_1d(mb), np.int32)
    msky = _c(np.atleast_1d(msky), np.int32)
    xr = _c(np.atleast_1d(xring), np.float64)
    if mb.shape != msky.shape:
        raise ValueError("mb and msky must have the same length")
    shape = (mb.size, lmax + 1, xr.size)
    lib = _load()
    if split:
        mant = np.empty(shape, np.float64)
        ex = np.empty(shape, np.int64)
        rc = lib.oracle_wigner_d(lmax, mb.size, _ptr(mb), _ptr(msky), xr.size, _ptr(xr),
                                 None, _ptr(mant), _ptr(ex), nthreads)
        if rc:
            raise ValueError("oracle_wigner_d: invalid arguments (%d)" % rc)
        return mant, ex
    d = np.empty(shape, np.float64)
    rc = lib.oracle_wigner_d(lmax, mb.size, _ptr(mb), _ptr(msky), xr.size, _ptr(xr),
                             _ptr(d), None, None, nthreads)
    if rc:
        raise ValueError("oracle_wigner_d: invalid arguments (%d)" % rc)
    return d


def all_columns(lmax: int, mbmax: int):
    """(mb, msky) for mb in [-mbmax, mbmax] (outer) and msky in [0, lmax] (inner)."""
    mb = np.repeat(np.arange(-mbmax, mbmax + 1, dtype=np.int32), lmax + 1)
    ms = np.tile(np.arange(lmax + 1, dtype=np.int32), 2 * mbmax + 1)
    return mb, ms


def totalconv_fwd(lmax: int, mbmax: int, xring, alm, blm, cols=None, rings=None,
                  eps: float = 0.0, nthreads: int = 0) -> np.ndarray:
    """C_{mb,msky}(beta_j) = sum_l conj(b_{l,mb}) d^l_{mb,msky}(beta_j) s_{l,msky}.

    cols: (mb array, msky array) or None for every (mb, msky >= 0) column.
    rings: ring indices or None for all.  Returns complex128 (ncol, nsel); with
    cols=None and rings=None, shape (2*mbmax+1, lmax+1, nring).  Rings are given by
    xring[j] = cos(beta_j)."""
    xr = _c(xring, np.float64)
    alm = _c(alm, np.complex128)
    blm = _c(blm, np.complex128)
    if alm.size != (lmax + 1) * (lmax + 2) // 2 or blm.shape != (2 * mbmax + 1, lmax + 1):
        raise ValueError("alm/blm shape mismatch")
    full = cols is None and rings is None
    cmb, cms = all_columns(lmax, mbmax) if cols is None else (_c(cols[0], np.int32), _c(cols[1], np.int32))
    sel = np.arange(xr.size, dtype=np.int32) if rings is None else _c(rings, np.int32)
    out = np.empty((cmb.size, sel.size), np.complex128)
    rc = _load().oracle_totalconv_fwd(lmax, mbmax, xr.size, _ptr(xr), _ptr(alm), _ptr(blm),
                                      cmb.size, _ptr(cmb), _ptr(cms), sel.size, _ptr(sel),
                                      float(eps), _ptr(out), nthreads)
    if rc:
        raise ValueError("oracle_totalconv_fwd: invalid arguments (%d)" % rc)
    if full:
        return out.reshape(2 * mbmax + 1, lmax + 1, xr.size)
    return out


def column_sums(lmax: int, mbmax: int, xring, G, cols, nthreads: int = 0) -> np.ndarray:
    """u_l(col) = sum_j d^l_col(beta_j) G[col, j]; G has shape (ncol, nring).
    Returns complex long double as an array of shape (ncol, lmax+1, 2) (re, im)."""
    xr = _c(xring, np.float64)
    cmb, cms = _c(cols[0], np.int32), _c(cols[1], np.int32)
    G = _c(G, np.complex128)
    if G.shape != (cmb.size, xr.size):
        raise ValueError("G must have shape (ncol, nring)")
    u = np.empty((cmb.size, lmax + 1, 2), np.longdouble)
    if u.itemsize != ctypes.sizeof(ctypes.c_longdouble):
        raise RuntimeError("numpy longdouble does not match C long double")
    rc = _load().oracle_totalconv_u(lmax, mbmax, xr.size, _ptr(xr), _ptr(G),
                                    cmb.size, _ptr(cmb), _ptr(cms), _ptr(u), nthreads)
    if rc:
        raise ValueError("oracle_totalconv_u: invalid arguments (%d)" % rc)
    return u


def totalconv_adj(lmax: int, mbmax: int, xring, alm, blm, Gbar, nthreads: int = 0):
    """Exact gradients (sky_bar, beam_bar) of the full forward for cotangent Gbar.

    Gbar has the layout of C, shape (2*mbmax+1, lmax+1, nring).  Returns complex128
    sky_bar (packed like alm) and beam_bar (shaped like blm)."""
    xr = _c(xring, np.float64)
    nring = xr.size
    Gbar = _c(Gbar, np.complex128).reshape(2 * mbmax + 1, lmax + 1, nring)
    cmb, cms = all_columns(lmax, mbmax)
    u = column_sums(lmax, mbmax, xr, Gbar.reshape(-1, nring), (cmb, cms), nthreads)
    u = u.reshape(2 * mbmax + 1, lmax + 1, lmax + 1, 2)     # [mb][msky][l][re/im]
    ure, uim = u[..., 0], u[..., 1]
    blm = _c(blm, np.complex128)
    bre = blm.real.astype(np.longdouble)[:, None, :]        # [mb][1][l]
    bim = blm.imag.astype(np.longdouble)[:, None, :]
    # sky_bar_{l,msky} = sum_mb b_{l,mb} u_l(mb,msky)
    sre = (bre * ure - bim * uim).sum(axis=0)               # [msky][l]
    sim = (bre * uim + bim * ure).sum(axis=0)
    sky_bar = np.zeros((lmax + 1) * (lmax + 2) // 2, np.complex128)
    for m in range(lmax + 1):
        start = m * (2 * lmax + 1 - m) // 2 + m      # packed index of (l = m, m)
        sky_bar[start:start + lmax + 1 - m] = (sre[m, m:].astype(np.float64)
                                              + 1j * sim[m, m:].astype(np.float64))
    # beam_bar_{l,mb} = sum_msky s_{l,msky} conj(u_l(mb,msky))
    alm = _c(alm, np.complex128)
    s_full = np.zeros((lmax + 1, lmax + 1), np.complex128)   # [msky][l]
    for m in range(lmax + 1):
        start = m * (2 * lmax + 1 - m) // 2 + m      # packed index of (l = m, m)
        s_full[m, m:] = alm[start:start + lmax + 1 - m]
    sre_ = s_full.real.astype(np.longdouble)[None]
    sim_ = s_full.imag.astype(np.longdouble)[None]
    bbre = (sre_ * ure + sim_ * uim).sum(axis=1)            # s * conj(u)
    bbim = (sim_ * ure - sre_ * uim).sum(axis=1)
    beam_bar = bbre.astype(np.float64) + 1j * bbim.astype(np.float64)
    return sky_bar, beam_bar


def totalconv_fwd_pol(lmax: int, mbmax: int, xring, alms, blms, summed: bool = False,
                      nthreads: int = 0):
    """Polarised total convolution (footnote of Sec. 4.1): eq. convdef evaluated for each
    (sky, beam) pair -- temperature, gradient, curl.  Returns the list of per-pair C, or
    (summed) a one-element list holding their sum, the polarised detector's coefficients."""
    if not 1 <= len(alms) <= 3 or len(blms) != len(alms):
        raise ValueError("1 to 3 (alm, blm) pairs")
    outs = [totalconv_fwd(lmax, mbmax, xring, a, b, nthreads=nthreads) for a, b in zip(alms, blms)]
    if summed:
        total = outs[0].copy()
        for c in outs[1:]:
            total += c
        return [total]
    return outs


def totalconv_adj_pol(lmax: int, mbmax: int, xring, alms, blms, Gbars, summed: bool = False,
                      nthreads: int = 0):
    """Gradients of totalconv_fwd_pol: pair p gets the scalar adjoint of its own sky and beam
    for its cotangent (summed: the one cotangent of the summed output).  Returns
    ([sky_bar per pair], [beam_bar per pair])."""
    if len(Gbars) != (1 if summed else len(alms)):
        raise ValueError("one cotangent per output")
    sky, beam = [], []
    for p, (a, b) in enumerate(zip(alms, blms)):
        sb, bb = totalconv_adj(lmax, mbmax, xring, a, b, Gbars[0 if summed else p], nthreads=nthreads)
        sky.append(sb)
        beam.append(bb)
    return sky, beam


def datacube(lmax: int, mbmax: int, C, nalpha: int, ngamma: int, points=None, nthreads: int = 0):
    """Data cube of eq. conviqt (Sec. 4.1) by its definition, the double sum over mb and
    msky in [-lmax, lmax] with C_{mb,msky<0} = conj(C_{-mb,-msky}); real part.

    C: complex (2*mbmax+1, lmax+1, nring).  points: (ring, a, g) index arrays, or None
    for the whole cube, shape (nring, nalpha, ngamma)."""
    C = _c(C, np.complex128)
    nring = C.shape[-1]
    if C.shape != (2 * mbmax + 1, lmax + 1, nring):
        raise ValueError("C must have shape (2*mbmax+1, lmax+1, nring)")
    if points is None:
        j, a, g = np.meshgrid(np.arange(nring), np.arange(nalpha), np.arange(ngamma), indexing="ij")
        pts = [_c(v.ravel(), np.int32) for v in (j, a, g)]
    else:
        pts = [_c(v, np.int32) for v in points]
    out = np.empty(pts[0].size, np.float64)
    rc = _load().oracle_datacube(lmax, mbmax, nring, _ptr(C), nalpha, ngamma, pts[0].size,
                                 _ptr(pts[0]), _ptr(pts[1]), _ptr(pts[2]), _ptr(out), nthreads)
    if rc:
        raise ValueError("oracle_datacube: invalid arguments (%d)" % rc)
    return out.reshape(nring, nalpha, ngamma) if points is None else out
