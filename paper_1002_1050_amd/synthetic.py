"""Seeded synthetic inputs: colatitude rings, skies and beams.

This module only draws and tabulates inputs.  It holds none of the method's
arithmetic (no Wigner elements, no recursion, no contraction), so both the HIP
path and the CPU oracle may be fed from it.

Layouts (all complex arrays are complex128, i.e. interleaved FP64 pairs):

* rings: colatitudes ``beta[j] = pi * (j + 1/2) / nring`` for ``j = 0 .. nring-1``, an
  open equispaced grid in (0, pi).  A ring is handed to the library as
  ``x[j] = cos(beta[j])`` (a double): ``ring_cosines`` evaluates the cosine in long
  double, rounds it once, and makes the set exactly mirror-symmetric,
  ``x[nring-1-j] = -x[j]`` (and ``x = 0`` on the equator ring when nring is odd),
  so that ring pairs (beta, pi - beta) are exact pairs.
* sky ``alm``: the coefficients s_{l,m} for 0 <= m <= l <= lmax, packed m-major
  (index ``m*(2*lmax+1-m)//2 + l``).  s_{l,-m} = (-1)^m conj(s_{l,m}) is implied
  (a real sky, Sec. 4.2.3 of the paper), so a_{l,0} is real.
* beam ``blm``: shape ``(2*mbmax+1, lmax+1)``, row ``mb + mbmax`` holds b_{l,mb}
  for every l (entries with l < |mb| are zero).

Recipes (seeded with numpy ``Generator(PCG64(seed))``):

* sky: C_l = 1/(l(l+1)+1), optionally times exp(-l^2/taper^2).  Drawn m-major
  with l inner; for m = 0 one standard normal per l, a_{l0} = sqrt(C_l) N; for
  m >= 1 two normals per l (real part first), a_{lm} = sqrt(C_l/2) (N + iN).
* beam: an elliptical Gaussian beam of full width at half maximum ``fwhm``
  (arcmin) and ellipticity ``e``: b_{l,0} = exp(-l(l+1) sigma^2 / 2) with
  sigma = fwhm / sqrt(8 ln 2) in radians, and for even m > 0
  b_{l,m} = b_{l,0} (e^2 l^2 / 8)^(m/2) / (m/2)!, zero for odd m and for l < m;
  b_{l,-m} = (-1)^m conj(b_{l,m}).  The formula is applied literally (it is a
  shape recipe, not a normalised beam).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SKY_SEED = 1002
TARGET_SKY_SEED = 1050


def ring_colatitudes(nring: int) -> np.ndarray:
    """Equispaced open ring grid beta_j = pi (j + 1/2) / nring."""
    if nring < 1:
        raise ValueError("nring must be >= 1")
    j = np.arange(nring, dtype=np.float64)
    return np.pi * (j + 0.5) / nring


def ring_cosines(nring: int) -> np.ndarray:
    """x_j = cos(beta_j) on the equispaced grid, exactly mirror-symmetric."""
    if nring < 1:
        raise ValueError("nring must be >= 1")
    pi = np.arccos(np.longdouble(-1.0))
    j = np.arange(nring, dtype=np.longdouble)
    x = np.cos(pi * (j + np.longdouble(0.5)) / np.longdouble(nring)).astype(np.float64)
    h = nring // 2
    x[nring - 1 - np.arange(h)] = -x[:h]
    if nring % 2:
        x[h] = 0.0
    return x


def alm_index(lmax: int, l, m):
    """Packed m-major index of (l, m), 0 <= m <= l <= lmax."""
    return m * (2 * lmax + 1 - m) // 2 + l


def alm_size(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def sky_alm(lmax: int, seed: int = SKY_SEED, taper: float | None = None) -> np.ndarray:
    """Gaussian random sky with power spectrum C_l = 1/(l(l+1)+1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    l_all = np.arange(lmax + 1, dtype=np.float64)
    cl = 1.0 / (l_all * (l_all + 1.0) + 1.0)
    if taper is not None:
        cl = cl * np.exp(-(l_all / taper) ** 2)
    out = np.zeros(alm_size(lmax), dtype=np.complex128)
    # m = 0: real
    out[0 : lmax + 1] = np.sqrt(cl) * rng.standard_normal(lmax + 1)
    for m in range(1, lmax + 1):
        n = lmax + 1 - m
        z = rng.standard_normal(2 * n).reshape(n, 2)
        start = alm_index(lmax, m, m)
        out[start : start + n] = np.sqrt(cl[m:] / 2.0) * (z[:, 0] + 1j * z[:, 1])
    return out


def beam_blm(lmax: int, mbmax: int, fwhm_arcmin: float, ellipticity: float) -> np.ndarray:
    """Elliptical Gaussian beam coefficients, shape (2*mbmax+1, lmax+1)."""
    if mbmax > lmax:
        raise ValueError("mbmax must not exceed lmax")
    sigma = math.radians(fwhm_arcmin / 60.0) / math.sqrt(8.0 * math.log(2.0))
    l_all = np.arange(lmax + 1, dtype=np.float64)
    b0 = np.exp(-0.5 * l_all * (l_all + 1.0) * sigma * sigma)
    out = np.zeros((2 * mbmax + 1, lmax + 1), dtype=np.complex128)
    out[mbmax, :] = b0
    e2 = ellipticity * ellipticity
    for m in range(2, mbmax + 1, 2):
        k = m // 2
        row = b0 * (e2 * l_all * l_all / 8.0) ** k / math.factorial(k)
        row[:m] = 0.0
        out[mbmax + m, :] = row
        out[mbmax - m, :] = ((-1) ** m) * np.conj(row)
    return out


def delta_sky(lmax: int, l: int, m: int, value: complex = 1.0) -> np.ndarray:
    out = np.zeros(alm_size(lmax), dtype=np.complex128)
    out[alm_index(lmax, l, m)] = value
    return out


def delta_beam(lmax: int, mbmax: int, l: int, mb: int, value: complex = 1.0) -> np.ndarray:
    out = np.zeros((2 * mbmax + 1, lmax + 1), dtype=np.complex128)
    out[mb + mbmax, l] = value
    return out


def random_beam(lmax: int, mbmax: int, seed: int) -> np.ndarray:
    """Complex Gaussian beam coefficients (no symmetry imposed), zero for l < |mb|."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((2 * mbmax + 1, lmax + 1, 2))
    out = (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)
    for r in range(2 * mbmax + 1):
        out[r, : abs(r - mbmax)] = 0.0
    return out


def random_cbar(lmax: int, mbmax: int, nring: int, seed: int) -> np.ndarray:
    """Complex Gaussian cotangent for C, shape (2*mbmax+1, lmax+1, nring)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((2 * mbmax + 1, lmax + 1, nring, 2))
    return (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)


def random_cbar_row(lmax: int, mbmax: int, nring: int, seed: int, mb: int) -> np.ndarray:
    """Row mb of a complex Gaussian cotangent for C, shape (lmax+1, nring), drawn from its own
    stream PCG64([seed, mb + mbmax]) so that one row can be drawn without the others."""
    rng = np.random.Generator(np.random.PCG64([seed, mb + mbmax]))
    z = rng.standard_normal((lmax + 1, nring, 2))
    return (z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0)


def count_terms(lmax: int, mbmax: int, nring: int) -> int:
    """Number of (l, mb, msky, beta) terms: sum over chains of lmax - max(|mb|, msky) + 1."""
    t = 0
    for mb in range(-mbmax, mbmax + 1):
        a = abs(mb)
        t += a * (lmax + 1 - a) + (lmax + 1 - a) * (lmax + 2 - a) // 2
    return t * nring


@dataclass
class Detector:
    lmax: int
    mbmax: int
    nring: int
    fwhm_arcmin: float
    ellipticity: float

    def xring(self) -> np.ndarray:
        return ring_cosines(self.nring)

    def colatitudes(self) -> np.ndarray:
        return ring_colatitudes(self.nring)

    def blm(self) -> np.ndarray:
        return beam_blm(self.lmax, self.mbmax, self.fwhm_arcmin, self.ellipticity)


@dataclass
class Workload:
    name: str
    lmax: int
    mbmax: int
    nring: int
    fwhm_arcmin: float
    ellipticity: float
    sky_seed: int = SKY_SEED
    target_seed: int | None = None
    sky_taper: float | None = None
    detectors: list = field(default_factory=list)

    def xring(self) -> np.ndarray:
        return ring_cosines(self.nring)

    def colatitudes(self) -> np.ndarray:
        return ring_colatitudes(self.nring)

    def alm(self) -> np.ndarray:
        return sky_alm(self.lmax, self.sky_seed, self.sky_taper)

    def blm(self) -> np.ndarray:
        return beam_blm(self.lmax, self.mbmax, self.fwhm_arcmin, self.ellipticity)

    def terms(self) -> int:
        if self.detectors:
            return sum(count_terms(d.lmax, d.mbmax, d.nring) for d in self.detectors)
        return count_terms(self.lmax, self.mbmax, self.nring)


def sixteen_detectors() -> list:
    """Sixteen detectors, one per (lmax, mbmax) combination."""
    ls = [512, 1024, 2048, 4096]
    ms = [4, 6, 9, 14]
    dets = []
    for i in range(16):
        lmax = ls[i % 4]
        mbmax = ms[i // 4]
        dets.append(Detector(lmax, mbmax, 2 * lmax, 4.0 + 26.0 * i / 15.0, 0.3 * ((5 * i) % 16) / 15.0))
    return dets


def four_large_detectors(seed: int = 5) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(4):
        fwhm = float(rng.uniform(4.0, 30.0))
        e = float(rng.uniform(0.0, 0.3))
        out.append(Detector(8192, 16, 16384, fwhm, e))
    return out


WORKLOADS = {
    # small forward case: lmax 64, mbmax 4, 129 rings, FWHM 10 deg, e = 0.1
    "small": Workload("small", 64, 4, 129, 600.0, 0.1),
    # forward case: lmax 1024, mbmax 9, 2048 rings, FWHM 5', e = 0.2
    "medium": Workload("medium", 1024, 9, 2048, 5.0, 0.2),
    # forward + adjoint case: lmax 2048, mbmax 14, 4096 rings, target sky seed 1050
    "adjoint": Workload("adjoint", 2048, 14, 4096, 5.0, 0.2, target_seed=TARGET_SKY_SEED),
    # headline case: lmax 4096, mbmax 14, 8192 rings, forward + adjoint
    "lmax4096": Workload("lmax4096", 4096, 14, 8192, 5.0, 0.2, target_seed=TARGET_SKY_SEED),
    # sixteen detectors with mixed lmax / mbmax, one sky at lmax 4096
    "batched16": Workload("batched16", 4096, 14, 8192, 0.0, 0.0, detectors=sixteen_detectors()),
    # four detectors at lmax 8192, mbmax 16, 16384 rings, tapered sky
    "large4": Workload("large4", 8192, 16, 16384, 0.0, 0.0, sky_taper=8192.0,
                       detectors=four_large_detectors()),
}
