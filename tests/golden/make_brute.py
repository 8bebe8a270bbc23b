"""Writes the brute-force fixtures in this folder.

Calls only ``oracle.brute`` (exact rational r^2, 50-digit mpmath cosine of
Eq. (1), Section 1).  Run from the repository root:
    python tests/golden/make_brute.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import brute  # noqa: E402

CASES = [
    # name, nx, ny, pitch, wavelength, points (x, y, z, A)
    ("tiny_near", 5, 4, 8e-6, 633e-9,
     [(1.25, 2.5, 2.0e-4, 0.75), (3.0, 0.0, 3.5e-4, -0.5), (-2.375, 5.125, 1.5e-4, 1.0)]),
    ("tiny_far", 7, 3, 8e-6, 633e-9,
     [(1900.3125, 1000.75, 0.3, 0.625), (-700.5, 40.25, 0.55, 0.875),
      (3.5, 1.0, 0.45, -0.25), (2500.125, -900.0, 0.35, 0.5)]),
]


def main():
    for name, nx, ny, pitch, wl, pts in CASES:
        x, y, z, a = (np.array([p[i] for p in pts], dtype=np.float32) for i in range(4))
        vals = brute.hologram(x, y, z, a, nx, ny, pitch, wl)
        rec = {
            "source": "Eq. (1), Section 1: exact rational r^2, mpmath cos at %d digits" % brute.DIGITS,
            "nx": nx, "ny": ny, "pitch": pitch, "wavelength": wl,
            "x": [float(v) for v in x], "y": [float(v) for v in y],
            "z": [float(v) for v in z], "a": [float(v) for v in a],
            "I": [[brute.mpmath.nstr(v, 40) for v in row] for row in vals],
        }
        with open(os.path.join(HERE, "brute_%s.json" % name), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
