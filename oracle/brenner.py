"""Brenner's series for the force on each of two equal spheres moving along
their line of centres with equal and opposite velocities (Section 3,
eq. Brenner), for unit radius and unit viscosity (test infrastructure).

Each term is evaluated with numerator and denominator scaled by
exp(-(2n+1) alpha) so that large n does not overflow.  Pinned in the tests
by its two limits: the far-field expansion 6 pi |v| (1 + 3/(2 d) + ...) and
the lubrication expansion 6 pi |v| (1/(2 delta) + (9/20) log(1/delta) + O(1)).
"""
from __future__ import annotations

import math


def brenner_force(delta: float, v: float = 1.0, tol: float = 1e-18, n_max: int = 200000) -> float:
    alpha = math.acosh(1.0 + delta / 2.0)
    sa, s2a = math.sinh(alpha), math.sinh(2.0 * alpha)
    total = 0.0
    for n in range(1, n_max):
        q = math.exp(-(2 * n + 1) * alpha)
        # 4 cosh^2((n+1/2) a) e^{-(2n+1) a} = (1 + e^{-(2n+1) a})^2
        num = (1.0 + q) ** 2 + (2 * n + 1) ** 2 * sa * sa * q
        # 2 sinh((2n+1) a) e^{-(2n+1) a} = 1 - e^{-2(2n+1) a}
        den = (1.0 - q * q) - (2 * n + 1) * s2a * q
        term = n * (n + 1) / ((2 * n - 1) * (2 * n + 3)) * (num / den - 1.0)
        total += term
        if n > 3 and abs(term) < tol * abs(total):
            break
    return 8.0 * math.pi * abs(v) * sa * total
