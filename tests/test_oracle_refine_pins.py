"""Pins of the oracle's per-segment charges, refinement (paper section 2.6)
and vertically connected sheets (section 3.3.2)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import inputs as I
from tests.exact_deposit import exact_deposit, exact_deposit_cic, exact_deposit_linear
from tests.test_oracle_pins import _dyadic_sheets, landau_root, log_peaks

EPS = np.finfo(np.float64).eps


def _with_segment_charges(rng, sheets):
    """The same sheets with a different dyadic charge on every segment."""
    out = []
    for _, closed, xs in sheets:
        n = len(xs)
        nseg = n if closed else n - 1
        cs = [Fraction(int(rng.integers(1, 17)), 16) for _ in range(nseg)]
        out.append((cs + [Fraction(0)] * (n - nseg), closed, xs))
    return out


@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("nc", [1, 3, 4, 13])
def test_segment_charges_match_exact_rational(order, nc):
    rng = np.random.default_rng(1300 + 10 * nc + order)
    exact_fn = {0: exact_deposit, 1: exact_deposit_linear, 2: exact_deposit_cic}[order]
    for L in (Fraction(1), Fraction(5, 4)):
        sheets = _with_segment_charges(rng, _dyadic_sheets(rng, 10, L))
        exact = exact_fn(L, nc, sheets)
        nts = [len(s[2]) for s in sheets]
        cl = [1 if s[1] else 0 for s in sheets]
        c = np.array([float(v) for s in sheets for v in s[0]])
        x = np.array([float(v) for s in sheets for v in s[2]])
        Q, _ = O.deposit(float(L), nc, nts, np.zeros(len(nts)), cl, x, order=order, c=c)
        total = float(np.sum(np.abs(c)))
        err = np.max(np.abs(Q - np.array([float(v) for v in exact])))
        if order == 1:
            # the gradient divides by centroid separations: allow their
            # conditioning (dyadic inputs keep it small)
            assert err <= 1e-12 * total, (nc, err)
        else:
            assert err <= 16 * EPS * total, (nc, err)


def test_uniform_segment_charges_reduce_to_sheet_charges():
    p = I.random_sheets(5, 6, [3, 64, 65, 2, 130, 7], 37, L=2.0, jitter=0.6, closed=[1, 0, 1, 0, 1, 1])
    c = p.seg_charges
    for order in (0, 1, 2):
        a, ma = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0, order=order)
        b, mb = O.deposit(p.L, p.n_cells, p.n_tracers, np.zeros(p.n_sheets), p.closed, p.x0, order=order, c=c)
        assert np.array_equal(a, b) and ma == mb
    r1 = O.run_problem(p, 12)
    r2 = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, c, p.x0, p.v0, 12)
    assert np.array_equal(r1["hist"], r2["hist"], equal_nan=True)
    assert np.array_equal(r1["x"], r2["x"]) and np.array_equal(r1["v"], r2["v"])


def test_tracer_masses_carry_the_segment_charges():
    """With equal charge-to-mass ratio the mass of the system is its charge:
    sheets moving at one common velocity u carry momentum u * (total charge)
    and kinetic energy u^2/2 * (total charge), open sheets included (whose
    end tracers bound one segment only)."""
    p = I.random_sheets(8, 5, [2, 9, 64, 3, 100], 20, L=1.5, jitter=0.4, closed=[0, 1, 0, 1, 0])
    rng = np.random.default_rng(3)
    c = p.seg_charges * rng.uniform(0.5, 2.0, p.total_tracers)
    ends = np.cumsum(p.n_tracers) - 1
    c[ends[p.closed == 0]] = 0.0
    u = 0.37
    v = np.full(p.total_tracers, u)
    _, _, ke, mom = O.push(p.L, p.n_cells, 0.1, p.n_tracers, p.q, p.closed, np.zeros(p.n_cells), p.x0, v, c=c)
    total = np.sum(c)
    assert abs(mom - u * total) < 1e-14 * abs(u * total)
    assert abs(ke - 0.5 * u * u * total) < 1e-14 * abs(ke)
    # a segment's momentum is its charge times the mean velocity of its ends
    v = rng.standard_normal(p.total_tracers)
    _, _, _, mom = O.push(p.L, p.n_cells, 0.1, p.n_tracers, p.q, p.closed, np.zeros(p.n_cells), p.x0, v, c=c)
    seg_mom, b = 0.0, 0
    for s in range(p.n_sheets):
        nt = int(p.n_tracers[s])
        for t in range(nt if p.closed[s] else nt - 1):
            seg_mom += c[b + t] * 0.5 * (v[b + t] + v[b + (t + 1) % nt])
        b += nt
    assert abs(mom - seg_mom) < 1e-13 * np.sum(np.abs(c) * 2)


def test_refinement_splits_long_segments_at_their_centre():
    """A segment longer than l_max gains a tracer at its centre (the shorter
    way round) with the mean velocity of its ends; both halves carry half the
    charge.  On dyadic positions every quantity is exact."""
    L = 1.0
    x = np.array([0.0, 0.25, 0.6875, 0.875, 0.5, 0.5 + 1 / 64, 0.9375, 0.0625])
    v = np.array([1.0, 2.0, -1.0, 0.5, 0.25, 0.75, 3.0, -3.0])
    nts = np.array([4, 2, 2], dtype=np.int32)
    cl = np.array([1, 0, 1], dtype=np.int32)
    c = np.array([0.5, 0.25, 0.125, 1.0, 2.0, 0.0, 4.0, 8.0])
    nt2, x2, v2, c2, added = O.refine(L, 0.2, nts, cl, x, v, c)
    # sheet 0: 0 -> .25 (split), .25 -> .6875 (split), .6875 -> .875 and .875 -> 0 (short)
    # sheet 1 (open): .5 -> .515625 (short); sheet 2: .9375 -> .0625 (.125 across 0) and back
    assert added == 2 and list(nt2) == [6, 2, 2]
    assert list(x2[:6]) == [0.0, 0.125, 0.25, 0.46875, 0.6875, 0.875]
    assert list(v2[:6]) == [1.0, 1.5, 2.0, 0.5, -1.0, 0.5]
    assert list(c2[:6]) == [0.25, 0.25, 0.125, 0.125, 0.125, 1.0]
    assert np.array_equal(x2[6:], x[4:]) and np.array_equal(c2[6:], c[4:])
    # a separation of exactly L/2 is taken downwards: .25 -> .75 runs through 0
    _, xt, _, _, added = O.refine(L, 0.2, [2], [0], np.array([0.25, 0.75]), np.zeros(2), np.array([1.0, 0.0]))
    assert added == 1 and list(xt) == [0.25, 0.0, 0.75]
    # across the periodic boundary: .875 -> .375 is 0.5 long downwards; centre .625
    nt3, x3, _, _, added = O.refine(L, 0.3, [2], [0], np.array([0.875, 0.375]), np.array([0.0, 1.0]),
                                    np.array([1.0, 0.0]))
    assert added == 1 and list(x3) == [0.875, 0.625, 0.375]
    nt3, x3, _, _, added = O.refine(L, 0.3, [2], [0], np.array([0.875, 0.25]), np.array([0.0, 1.0]),
                                    np.array([1.0, 0.0]))
    assert added == 1 and list(x3) == [0.875, 0.0625, 0.25]
    # "longer than" is strict: a segment of exactly l_max (dyadic, so the
    # length is exact) stays whole, one a rounding unit longer is split
    seg = np.array([0.25, 0.5])
    _, xt, _, _, added = O.refine(L, 0.25, [2], [0], seg, np.zeros(2), np.array([1.0, 0.0]))
    assert added == 0 and list(xt) == [0.25, 0.5]
    _, xt, _, _, added = O.refine(L, np.nextafter(0.25, 0.0), [2], [0], seg, np.zeros(2), np.array([1.0, 0.0]))
    assert added == 1 and list(xt) == [0.25, 0.375, 0.5]


@pytest.mark.parametrize("order", [0, 2])
def test_refinement_keeps_charge_momentum_and_deposit(order):
    """Halving a segment leaves its box function unchanged (half the charge
    over half the length), so the constant and first-order weighted deposits
    do not change; total charge is exact and momentum is unchanged."""
    p = I.random_sheets(11, 7, [40, 3, 64, 65, 2, 128, 9], 50, L=2.5, jitter=1.5, closed=[1, 0, 1, 1, 0, 1, 1])
    c = p.seg_charges
    dx = p.L / p.n_cells
    nt2, x2, v2, c2, added = O.refine(p.L, 0.8 * dx, p.n_tracers, p.closed, p.x0, p.v0, c)
    assert added > 20
    assert math.fsum(c2) == math.fsum(c)
    Q1, m1 = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0, order=order, c=c)
    Q2, m2 = O.deposit(p.L, p.n_cells, nt2, p.q, p.closed, x2, order=order, c=c2)
    assert np.max(np.abs(Q2 - Q1)) < 1e-12 * np.max(np.abs(Q1)) * max(1, added / 100)
    assert m2 <= 0.5 * m1 + 1e-15 or m2 <= 0.8 * dx
    E = np.zeros(p.n_cells)
    _, _, _, mom1 = O.push(p.L, p.n_cells, 0.0, p.n_tracers, p.q, p.closed, E, p.x0, p.v0, c=c)
    _, _, _, mom2 = O.push(p.L, p.n_cells, 0.0, nt2, p.q, p.closed, E, x2, v2, c=c2)
    assert abs(mom2 - mom1) < 1e-14 * np.sum(np.abs(c) * np.abs(p.v0).max())


def _refined_run(l_max_cells, n_steps=550):
    p = I.refinement_two_stream(n_steps=n_steps)
    dx = p.L / p.n_cells
    r = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps,
                  l_max=l_max_cells * dx, capacity=2_000_000)
    return p, r


def _lengths(p, r):
    out, b = [], 0
    for nt in r["n_tracers"]:
        xs = r["x"][b:b + nt]
        d = np.roll(xs, -1) - xs
        out.append(np.abs(d - p.L * np.floor(d / p.L + 0.5)))
        b += nt
    return np.concatenate(out)


def test_refinement_two_stream_follows_section_2_6():
    """Section 2.6's two-stream experiment: little refinement while the
    instability grows linearly, then roughly exponential growth of the tracer
    count once the vortex folds the sheets; the refinement length moves the
    onset, not the rate; the mean segment length settles slightly above half
    the refinement length.  Charge is conserved exactly throughout."""
    rates, onsets = {}, {}
    for lm in (1.0, 0.5):
        p, r = _refined_run(lm)
        f = r["count"] / r["count"][0]
        t = r["hist"][:, 1]
        W = r["hist"][:, 2]
        linear = t <= 20.0  # field energy still far below saturation here
        assert W[linear].max() < 0.1 * W.max()
        assert np.all(f[linear] == 1.0)
        onsets[lm] = t[np.argmax(f > 1.01)]
        grow = f >= 2.0
        slope, icpt = np.polyfit(t[grow], np.log(f[grow]), 1)
        resid = np.log(f[grow]) - (slope * t[grow] + icpt)
        assert np.std(resid) < 0.2, (lm, np.std(resid))
        assert f[-1] > 20.0
        rates[lm] = slope
        ratio = _lengths(p, r).mean() / (lm * p.L / p.n_cells)
        assert 0.5 < ratio < 0.75, (lm, ratio)
        assert np.all(r["hist"][:, 5] == r["hist"][0, 5]) or \
            np.max(np.abs(r["hist"][:, 5] - r["hist"][0, 5])) < 1e-13 * r["hist"][0, 5]
        assert math.fsum(r["c"]) == math.fsum(p.seg_charges)  # halving is exact
    assert onsets[0.5] < onsets[1.0]
    assert abs(rates[0.5] / rates[1.0] - 1.0) < 0.15, rates


def test_vertical_sheets_start_as_point_charges():
    """Vertically connected sheets join tracers at one position, so every
    segment starts with zero length and its charge goes to the cell that owns
    that position (the zero-length reading)."""
    p = I.landau_vertical(n_streams=26, n_positions=160, n_cells=40)
    c = p.seg_charges
    Q, ms = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0, order=0, c=c)
    assert ms == 0.0
    expect = np.zeros(p.n_cells)
    col = np.sum(c[:26])
    dx = p.L / p.n_cells
    for xp in p.x0[::26]:
        expect[(math.ceil(xp / dx) - 1) % p.n_cells] += col
    assert np.max(np.abs(Q - expect)) < 1e-14 * col


def test_vertical_sheets_damp_at_the_landau_rate_with_refinement():
    """Landau damping (k = 0.5) with vertically connected sheets (section
    3.3.2): with refinement at one cell they reproduce the kinetic damping
    rate and frequency; without it the stretched sheets lose the density
    information and the rate is far off."""
    root = landau_root(0.5)
    p = I.landau_vertical(n_streams=64, n_positions=256, n_cells=64, n_steps=260, vmax_units=6.0)
    dx = p.L / p.n_cells
    fits = {}
    for lm in (dx, 0.0):
        r = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps,
                      l_max=lm, capacity=4_000_000)
        h = r["hist"]
        tp, lp = log_peaks(h[:, 1], h[:, 2], 2.0, 25.0)
        fits[lm] = (np.polyfit(tp, lp, 1)[0] / 2, math.pi / np.mean(np.diff(tp)))
    gamma, omega = fits[dx]
    assert abs(gamma / root.imag - 1.0) < 0.02, gamma
    assert abs(omega / root.real - 1.0) < 0.01, omega
    assert abs(fits[0.0][0] / root.imag - 1.0) > 0.1, fits[0.0]
