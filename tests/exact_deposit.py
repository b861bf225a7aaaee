"""Exact-rational brute-force deposit for tiny meshes (a pin for the oracle).

Independent formulation: the segment is laid out in unwrapped coordinates
[a, a + d] (d the minimum-image separation) and intersected with every
unwrapped cell [j dx, (j+1) dx], whose charge is added to cell j mod nc.
All arithmetic is in ``fractions.Fraction``, so the result is exact.
"""
from fractions import Fraction
import math


def _seg_charge(q, t):
    """q is one charge for every segment of the sheet, or a list of
    per-segment charges (entry t: the segment that starts at tracer t)."""
    return Fraction(q[t]) if isinstance(q, (list, tuple)) else Fraction(q)


def exact_deposit(L, nc, sheets):
    """sheets: list of (q, closed, [x_t as Fraction]); q is a charge per
    segment, or a list of them.  Returns [Fraction] * nc."""
    L = Fraction(L)
    dx = L / nc
    Q = [Fraction(0)] * nc
    for q, closed, xs in sheets:
        qs = q
        n = len(xs)
        nseg = n if closed else n - 1
        for t in range(nseg):
            q = _seg_charge(qs, t)
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


def _min_image(d, L):
    if d >= L / 2:
        return d - L
    if d < -L / 2:
        return d + L
    return d


def exact_deposit_linear(L, nc, sheets):
    """Piecewise-linear segments (section 2.5) in exact rational arithmetic:
    segment i carries rho0_i + (x - c_i) g_i with rho0_i = q / length_i, c_i
    its midpoint, and g_i the central difference of the neighbours' rho0 over
    their centroid separation when the three centroids are in monotone order
    (else 0); each cell gets the exact integral over its overlap."""
    L = Fraction(L)
    dx = L / nc
    Q = [Fraction(0)] * nc
    for q, closed, xs in sheets:
        qs = q
        n = len(xs)
        nseg = n if closed else n - 1
        segs = []
        for t in range(nseg):
            a = Fraction(xs[t])
            d = _min_image(Fraction(xs[(t + 1) % n]) - a, L)
            segs.append((a, d, a + d / 2, (_seg_charge(qs, t) / abs(d)) if d != 0 else None))
        for t, (a, d, c, r0) in enumerate(segs):
            if d == 0:
                Q[(math.ceil(a / dx) - 1) % nc] += _seg_charge(qs, t)
                continue
            g = Fraction(0)
            has_prev = (nseg >= 3) if closed else t > 0
            has_next = (nseg >= 3) if closed else t + 1 < nseg
            if has_prev and has_next:
                ap, dp_, cp, rp = segs[(t - 1) % nseg]
                an, dn_, cn, rn = segs[(t + 1) % nseg]
                if rp is not None and rn is not None:
                    dm = _min_image(cp - c, L)
                    dpp = _min_image(cn - c, L)
                    if (dm < 0 < dpp) or (dpp < 0 < dm):
                        g = (rn - rp) / (dpp - dm)
            lo, hi = (a, a + d) if d > 0 else (a + d, a)
            for j in range(math.floor(lo / dx) - 1, math.floor(hi / dx) + 2):
                al = max(lo, j * dx)
                be = min(hi, (j + 1) * dx)
                if be > al:
                    w = be - al
                    Q[j % nc] += r0 * w + g * w * ((al + be) / 2 - c)
    return Q


def _hat_antiderivative(t):
    """Integral of max(0, 1 - |s|) from -infinity to t."""
    if t <= -1:
        return Fraction(0)
    if t <= 0:
        return (1 + t) ** 2 / 2
    if t <= 1:
        return 1 - (1 - t) ** 2 / 2
    return Fraction(1)


def exact_deposit_cic(L, nc, sheets):
    """First-order weighting of segments (section 2.4) in exact arithmetic,
    through the antiderivative of the hat: grid point j (at (j + 1/2) dx)
    gets h dx [H((hi - X_j)/dx) - H((lo - X_j)/dx)], h = q / length; a
    zero-length segment gives its point the hat weights."""
    L = Fraction(L)
    dx = L / nc
    Q = [Fraction(0)] * nc
    for q, closed, xs in sheets:
        qs = q
        n = len(xs)
        nseg = n if closed else n - 1
        for t in range(nseg):
            q = _seg_charge(qs, t)
            a = Fraction(xs[t])
            d = _min_image(Fraction(xs[(t + 1) % n]) - a, L)
            if d == 0:
                for j in range(math.floor(a / dx) - 2, math.floor(a / dx) + 3):
                    w = 1 - abs(a - (j + Fraction(1, 2)) * dx) / dx
                    if w > 0:
                        Q[j % nc] += q * w
                continue
            lo, hi = (a, a + d) if d > 0 else (a + d, a)
            h = q / (hi - lo)
            for j in range(math.floor(lo / dx) - 2, math.floor(hi / dx) + 3):
                X = (j + Fraction(1, 2)) * dx
                Q[j % nc] += h * dx * (_hat_antiderivative((hi - X) / dx) - _hat_antiderivative((lo - X) / dx))
    return Q
