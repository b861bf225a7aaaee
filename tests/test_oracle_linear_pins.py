"""Pins of the oracle's piecewise-linear segment deposit (paper section 2.5)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import inputs as I
from tests.exact_deposit import exact_deposit, exact_deposit_linear
from tests.test_oracle_pins import _dyadic_sheets
from tests.test_oracle_golden import load_golden

CV = load_golden("convergence_section_3_3.txt")

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("nc", [1, 2, 3, 5, 8, 16])
def test_linear_deposit_matches_exact_rational(nc):
    rng = np.random.default_rng(500 + nc)
    for L in (Fraction(1), Fraction(5, 2)):
        sheets = _dyadic_sheets(rng, 14, L)
        exact = exact_deposit_linear(L, nc, sheets)
        nts = [len(s[2]) for s in sheets]
        q = [float(s[0]) for s in sheets]
        cl = [1 if s[1] else 0 for s in sheets]
        x = np.array([float(v) for s in sheets for v in s[2]])
        Q, _ = O.deposit(float(L), nc, nts, q, cl, x, order=1)
        total = float(sum(s[0] * (len(s[2]) if s[1] else len(s[2]) - 1) for s in sheets))
        err = np.max(np.abs(Q - np.array([float(v) for v in exact])))
        assert err <= 1e-12 * total, (nc, float(L), err)


def test_linear_and_constant_differ_only_by_the_gradient_terms():
    """With every gradient zero (a sheet whose segments all have equal
    length), the linear deposit is the constant one."""
    L, nc = Fraction(1), 8
    xs = [Fraction(k, 16) for k in range(16)]
    sheets = [(Fraction(1, 16), True, xs)]
    assert exact_deposit_linear(L, nc, sheets) == exact_deposit(L, nc, sheets)


def test_linear_deposit_conserves_charge():
    p = I.random_sheets(17, 30, [int(n) for n in np.random.default_rng(4).integers(2, 300, 30)], 77, L=4.0,
                        jitter=0.9, closed=[int(c) for c in np.random.default_rng(5).integers(0, 2, 30)])
    Q, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0, order=1)
    nseg = np.where(p.closed == 1, p.n_tracers, p.n_tracers - 1)
    expect = float(np.sum(p.q * nseg))
    assert abs(Q.sum() - expect) <= 1e-13 * expect


def test_linear_density_is_reproduced_exactly():
    """Tracers placed at the exact inverse cumulative of a linear density
    n(x) = a + b x: every interior segment's mean density is n at its
    centroid and the central difference is exactly b, so the piecewise-linear
    reconstruction is n itself and cells covered by interior segments receive
    their exact integral of n (an open sheet on part of the box)."""
    L, nc = 8.0, 64
    dx = L / nc
    a, b = 1.0, 0.25
    x0, x1 = 1.0, 6.0
    N = 41
    total = a * (x1 - x0) + 0.5 * b * (x1 ** 2 - x0 ** 2)
    targets = np.linspace(0.0, total, N)
    # inverse of a(x - x0) + b/2 (x^2 - x0^2) = s
    xs = (-a + np.sqrt(a * a + 2 * b * (targets + a * x0 + 0.5 * b * x0 * x0))) / b
    q = total / (N - 1)
    Q, _ = O.deposit(L, nc, [N], [q], [0], xs, order=1)
    lo, hi = xs[1], xs[N - 2]  # covered by interior segments only
    for j in range(nc):
        fa, fb = j * dx, (j + 1) * dx
        if fa >= lo and fb <= hi:
            exact = a * (fb - fa) + 0.5 * b * (fb ** 2 - fa ** 2)
            assert abs(Q[j] - exact) < 1e-13, j
    Q0, _ = O.deposit(L, nc, [N], [q], [0], xs, order=0)
    j = int((0.5 * (lo + hi)) // dx)
    exact = a * dx + 0.5 * b * (((j + 1) * dx) ** 2 - (j * dx) ** 2)
    assert abs(Q0[j] - exact) > 1e-6  # the constant scheme does not


def test_fold_corner_drops_the_gradient():
    """Open sheet 0.10 -> 0.20 -> 0.30 -> 0.25 -> 0.15 (q = 1 per segment),
    worked by hand: segment 0 and segment 3 lack a neighbour (flat boxes of
    density 10); segment 1 has centroids 0.15 < 0.25 < 0.275, so it carries
    10 + 80 (x - 0.25) on [0.2, 0.3]; segment 2 is the corner of the fold
    (centroids 0.25, 0.275, 0.2 not monotone), a flat box of density 20 on
    [0.25, 0.3]."""
    L, nc = 1.0, 100
    dx = L / nc
    xs = np.array([0.10, 0.20, 0.30, 0.25, 0.15])
    Q, _ = O.deposit(L, nc, [5], [1.0], [0], xs, order=1)

    def integral(lo, hi, f0, g, c, a, b):
        al, be = max(lo, a), min(hi, b)
        if be <= al:
            return 0.0
        return f0 * (be - al) + g * (be - al) * (0.5 * (al + be) - c)

    for j in range(nc):
        a, b = j * dx, (j + 1) * dx
        expect = (integral(0.10, 0.20, 10.0, 0.0, 0.15, a, b) + integral(0.20, 0.30, 10.0, 80.0, 0.25, a, b)
                  + integral(0.25, 0.30, 20.0, 0.0, 0.275, a, b) + integral(0.15, 0.25, 10.0, 0.0, 0.2, a, b))
        assert abs(Q[j] - expect) < 1e-12, (j, Q[j], expect)


def _sheet_density_error(N, nc, order, alpha=0.3, k=0.5):
    """Max cell-density error of one cold sheet x = q + (alpha/k) sin kq with
    N tracers on nc cells, against the exact cell averages."""
    L = 2 * math.pi / k
    qs = np.arange(N) * (L / N)
    xs = qs + (alpha / k) * np.sin(k * qs)
    Q, _ = O.deposit(L, nc, [N], [L / N], [1], np.mod(xs, L), order=order)
    # exact: charge between faces = Lagrangian extent q(x_{j+1}) - q(x_j)
    faces = np.arange(nc + 1) * (L / nc)
    qf = faces.copy()
    for _ in range(60):
        qf = qf - (qf + (alpha / k) * np.sin(k * qf) - faces) / (1 + alpha * np.cos(k * qf))
    exact = np.diff(qf)
    return np.max(np.abs(Q - exact)) / (L / nc)


def test_linear_segments_converge_one_order_faster():
    """Density error against the exact cell averages, with fewer tracers
    than cells: first order for constant segments, second for linear ones
    (section 3.3, convergence study; the orders from the golden fixture)."""
    Ns = np.array([16, 32, 64, 128])
    e0 = np.array([_sheet_density_error(N, 512, 0) for N in Ns])
    e1 = np.array([_sheet_density_error(N, 512, 1) for N in Ns])
    s0 = np.polyfit(np.log(Ns), np.log(e0), 1)[0]
    s1 = np.polyfit(np.log(Ns), np.log(e1), 1)[0]
    assert abs(s0 - CV["field_order_constant"]) < 0.3, s0
    assert s1 < CV["field_order_linear"] + 0.3, s1
    assert np.all(e1 < e0)
