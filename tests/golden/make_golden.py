"""Write the stored expected values under tests/golden/.

Calls only the oracle package: ``oracle.ring_x`` for the ring definition and
``oracle.mpref`` (mpmath, 40 significant digits) for reduced Wigner elements
from the Jacobi-polynomial closed form, which is independent of the
l-recursion.  Run from the repository root:  python tests/golden/make_golden.py
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


def main():
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
