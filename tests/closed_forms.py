"""Closed forms from the Stokes-flow literature for two equal spheres, used
as pins by the tests (of the oracle and of the library alike).  They come
from bispherical-coordinate solutions, not from the paper, and share
nothing with either implementation."""
import math


def stimson_jeffery(h):
    """Drag factor F / (6 pi mu a U) of two equal spheres translating with the
    same velocity along their line of centres, half centre distance h radii
    (Stimson & Jeffery 1926, bispherical coordinates, cosh(alpha) = h).  The
    bracket of each term is written as one quotient,
    [2 - 2 exp(-(2n+1) alpha) + (2n+1) sinh(2 alpha) + (2n+1)^2 sinh^2(alpha)]
    / [2 sinh((2n+1) alpha) + (2n+1) sinh(2 alpha)], which is 1 minus the
    published ratio without its cancellation."""
    al = math.acosh(h)
    sa, s2 = math.sinh(al), math.sinh(2 * al)
    tot = 0.0
    for n in range(1, 100000):
        k = 2 * n + 1
        x = k * al
        if x > 700.0:           # the remaining terms are below exp(-700) relative
            break
        num = 2.0 - 2.0 * math.exp(-x) + k * s2 + k * k * sa * sa
        tot += n * (n + 1) / ((2 * n - 1) * (2 * n + 3)) * num / (2.0 * math.sinh(x) + k * s2)
    return 4.0 / 3.0 * sa * tot


def jeffery_axial_torque(h, same_sense):
    """Torque factor T / (8 pi mu a^3 Omega) of two equal spheres spinning
    about their line of centres, half centre distance h radii (Jeffery 1915,
    bispherical coordinates, cosh(alpha) = h): sinh^3(alpha) times the sum
    over n >= 1 of cosech^3(n alpha), with alternating signs (+, -, +, ...)
    when both spin in the same sense.  Spinning in opposite senses is a
    sphere spinning at distance h from a no-slip wall."""
    al = math.acosh(h)
    tot = 0.0
    for n in range(1, 100000):
        if n * al > 230.0:         # cosech^3 below exp(-690)
            break
        tot += (-1.0 if same_sense and n % 2 == 0 else 1.0) / math.sinh(n * al) ** 3
    return math.sinh(al) ** 3 * tot
