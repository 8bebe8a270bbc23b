"""High-precision brute force of Eq. (1) for tiny grids (test infrastructure).

Independent of ``cgh_oracle.c``: the squared distance is formed exactly in
rational arithmetic from the binary values of the inputs, P_j = pi p^2 /
(lambda z_j) (Section 1) and the cosine are evaluated by mpmath at 50 decimal
digits.  Used to pin the C oracle and to write the stored fixtures under
``tests/golden/``.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath

DIGITS = 50


def _mp(v: float) -> mpmath.mpf:
    # A binary64 value is a dyadic rational; mpf holds it exactly at 50 digits.
    return mpmath.mpf(float(v))


def hologram(x, y, z, a, nx, ny, pitch, wavelength):
    """Return ``I[k][i]`` (row k = y_h, column i = x_h) as mpmath numbers."""
    with mpmath.workdps(DIGITS):
        p = _mp(pitch)
        lam = _mp(wavelength)
        coeff = [mpmath.pi * p * p / (lam * _mp(zj)) for zj in z]
        out = []
        for k in range(ny):
            row = []
            for i in range(nx):
                s = mpmath.mpf(0)
                for j in range(len(x)):
                    r2 = (Fraction(i) - Fraction(float(x[j]))) ** 2 + \
                         (Fraction(k) - Fraction(float(y[j]))) ** 2
                    r2m = mpmath.mpf(r2.numerator) / mpmath.mpf(r2.denominator)
                    s += _mp(a[j]) * mpmath.cos(coeff[j] * r2m)
                row.append(s)
            out.append(row)
        return out
