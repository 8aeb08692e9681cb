"""Write the stored expected values under tests/golden/.

Calls only the oracle package: ``oracle.ring_x`` for the ring definition and
``oracle.mpref`` (mpmath, 40 significant digits) for reduced Wigner elements
from the Jacobi-polynomial closed form, which is independent of the
l-recursion; and ``oracle.column_sums`` for one row of the adjoint's beam gradient
(inputs from the seeded generators of ``paper_1002_1050_amd.synthetic``, which hold
none of the method's arithmetic).  Run from the repository root:
    python tests/golden/make_golden.py             (Jacobi points)
    python tests/golden/make_golden.py beam_row    (beam-gradient row, minutes of CPU)
"""
import json
import os
import sys

import mpmath as mp
import numpy as np

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
import oracle  # noqa: E402
from oracle import mpref  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def jacobi_points():
    mp.mp.dps = 40
    out = []
    for L in (1024, 4096, 8192):
        nring = 2 * L
        rings = [0, 1, 3, 17, nring // 4, nring // 2 - 1, 3 * nring // 4, nring - 1]
        beta = np.pi * (np.array(rings, dtype=np.float64) + 0.5) / nring
        x = oracle.ring_x(beta)
        cols = [(0, 0), (14, 14), (-14, 300), (3, L // 4), (16, L - 1000), (0, L - 96),
                (-9, 5), (7, -2), (-12, -L // 2)]
        for (mb, ms) in cols:
            for l in sorted({max(abs(mb), abs(ms)), max(abs(mb), abs(ms)) + 7, L // 2 + 1, L}):
                if l < max(abs(mb), abs(ms)):
                    continue
                for j, xj in zip(rings, x):
                    v = mpref.d_jacobi_any(l, mb, ms, mp.mpf(float(xj)))
                    out.append({"lmax": L, "nring": nring, "ring": j, "l": l, "mb": mb, "msky": ms,
                                "x": float(xj).hex(), "d": mp.nstr(v, 30)})
    return out


def beam_gradient_row():
    """One row of the beam gradient at the lmax 4096 workload (mbmax 14, 8192 rings, sky seed
    1002): beam_bar_{l,mb} = sum_{msky <= l} s_{l,msky} conj(u_l(mb, msky)) with the oracle's
    column sums u_l over every ring, for the seeded cotangent row synthetic.random_cbar_row
    (seed 4096, mb 13; every other row zero).  About 7e10 oracle terms."""
    from paper_1002_1050_amd import synthetic as S
    L, M, nring, mb, seed = 4096, 14, 8192, 13, 4096
    x = S.ring_cosines(nring)
    alm = S.sky_alm(L, S.SKY_SEED)
    G = S.random_cbar_row(L, M, nring, seed, mb)
    ms = np.arange(L + 1, dtype=np.int32)
    u = oracle.column_sums(L, M, x, G, (np.full(L + 1, mb, np.int32), ms))   # [msky][l][re, im]
    ure, uim = u[..., 0], u[..., 1]
    bre = np.zeros(L + 1, np.longdouble)
    bim = np.zeros(L + 1, np.longdouble)
    for m in range(L + 1):
        start = S.alm_index(L, m, m)
        s = alm[start:start + L + 1 - m]
        sr, si = s.real.astype(np.longdouble), s.imag.astype(np.longdouble)
        bre[m:] += sr * ure[m, m:] + si * uim[m, m:]      # s conj(u)
        bim[m:] += si * ure[m, m:] - sr * uim[m, m:]
    bre[:abs(mb)] = 0
    bim[:abs(mb)] = 0
    return {
        "what": "beam-gradient row mb of the total-convolution adjoint (Sec. 4.1 eq. convdef, its exact "
                "transpose) at lmax 4096, mbmax 14, 8192 rings synthetic.ring_cosines, sky "
                "synthetic.sky_alm(4096, 1002), cotangent row synthetic.random_cbar_row(4096, 14, 8192, "
                "4096, 13) and every other row zero; oracle column sums in x87 long double",
        "lmax": L, "mbmax": M, "nring": nring, "mb": mb, "seed": seed,
        "re": [float(v).hex() for v in bre.astype(np.float64)],
        "im": [float(v).hex() for v in bim.astype(np.float64)],
    }


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "beam_row":
        doc = beam_gradient_row()
        with open(os.path.join(HERE, "beam_gradient_row_lmax4096.json"), "w") as f:
            json.dump(doc, f)
        print("wrote beam-gradient row of", len(doc["re"]), "values")
        return
    pts = jacobi_points()
    doc = {
        "what": "reduced Wigner elements d^l_{mb,msky}(beta_ring) from the Jacobi closed form "
                "(mpmath, 40 digits) on rings beta_j = pi (j+1/2)/nring, x = cos(beta_j) rounded to double",
        "convention": "d^l_{m m'}(beta) = <l m|exp(-i beta J_y)|l m'>, Sec. 2 eq. reducedwignerdef",
        "points": pts,
    }
    with open(os.path.join(HERE, "jacobi_large_l.json"), "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote", len(pts), "points")


if __name__ == "__main__":
    main()
