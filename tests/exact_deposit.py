"""Exact-rational brute-force deposit for tiny meshes (a pin for the oracle).

Independent formulation: the segment is laid out in unwrapped coordinates
[a, a + d] (d the minimum-image separation) and intersected with every
unwrapped cell [j dx, (j+1) dx], whose charge is added to cell j mod nc.
All arithmetic is in ``fractions.Fraction``, so the result is exact.
"""
from fractions import Fraction
import math


def exact_deposit(L, nc, sheets):
    """sheets: list of (q, closed, [x_t as Fraction]).  Returns [Fraction] * nc."""
    L = Fraction(L)
    dx = L / nc
    Q = [Fraction(0)] * nc
    for q, closed, xs in sheets:
        q = Fraction(q)
        n = len(xs)
        nseg = n if closed else n - 1
        for t in range(nseg):
            a = Fraction(xs[t])
            b = Fraction(xs[(t + 1) % n])
            d = b - a
            if d >= L / 2:
                d -= L
            elif d < -L / 2:
                d += L
            if d == 0:
                j = math.ceil(a / dx) - 1
                Q[j % nc] += q
                continue
            lo, hi = (a, a + d) if d > 0 else (a + d, a)
            length = hi - lo
            for j in range(math.floor(lo / dx) - 1, math.floor(hi / dx) + 2):
                left = max(lo, j * dx)
                right = min(hi, (j + 1) * dx)
                if right > left:
                    Q[j % nc] += q * (right - left) / length
    return Q
