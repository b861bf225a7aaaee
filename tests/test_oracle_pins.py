"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: exact
rational arithmetic, closed forms of the discrete Poisson problem, invariants
of the deposit, dispersion relations of the paper's test problems (section 3)
solved here with an independent root finder, and leapfrog reversibility.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import wofz

from oracle import oracle as O
from paper_1506_07207_amd import inputs as I
from tests.exact_deposit import exact_deposit

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------- helpers

def landau_root(k, guess=1.4 - 0.15j):
    """Root of the Maxwellian dielectric function 1 + (1 + z Z(z)) / k^2 = 0,
    z = omega / (sqrt(2) k), Z(z) = i sqrt(pi) w(z) (v_th = 1, omega_p = 1)."""

    def D(w):
        z = w / (math.sqrt(2.0) * k)
        return 1.0 + (1.0 + z * 1j * math.sqrt(math.pi) * wofz(z)) / k ** 2

    w = guess
    for _ in range(80):
        h = 1e-7
        step = D(w) / ((D(w + h) - D(w - h)) / (2 * h))
        w -= step
        if abs(step) < 1e-14:
            break
    return w


def multibeam_root(k, v, wts, guess):
    """Root of 1 = sum_m w_m / (omega - k v_m)^2 (cold beams, section 3.2)."""
    om = complex(guess)
    for _ in range(200):
        D = 1.0 - np.sum(wts / (om - k * v) ** 2)
        dD = np.sum(2.0 * wts / (om - k * v) ** 3)
        step = D / dD
        om -= step
        if abs(step) < 1e-15:
            break
    return om


def log_peaks(t, W, t0, t1):
    """Local maxima of W in [t0, t1], refined by a parabola through log W."""
    dt = t[1] - t[0]
    tp, lp = [], []
    for i in range(1, len(W) - 1):
        if W[i] > W[i - 1] and W[i] >= W[i + 1] and t0 <= t[i] <= t1:
            y0, y1, y2 = np.log(W[i - 1:i + 2])
            den = y0 - 2 * y1 + y2
            off = 0.5 * (y0 - y2) / den if den != 0 else 0.0
            tp.append(t[i] + off * dt)
            lp.append(y1 - 0.25 * (y0 - y2) * off)
    return np.array(tp), np.array(lp)


# ---------------------------------------------------------------- deposit

def _dyadic_sheets(rng, n_sheets, L, den=64):
    sheets = []
    for _ in range(n_sheets):
        n = int(rng.integers(2, 12))
        ks = rng.integers(0, den, n)
        if rng.uniform() < 0.5:  # mostly ordered with folds
            ks = np.sort(ks)
            ks[rng.integers(0, n)] = rng.integers(0, den)
        if rng.uniform() < 0.3 and n > 2:  # a zero-length segment
            ks[1] = ks[0]
        if rng.uniform() < 0.3 and n > 2:  # a segment of exactly L/2
            ks[2] = (ks[1] + den // 2) % den
        xs = [Fraction(int(k), den) * L for k in ks]
        q = Fraction(int(rng.integers(1, 9)), 8)
        sheets.append((q, bool(rng.uniform() < 0.8), xs))
    return sheets


def test_wrap_lands_in_the_box_at_the_nearest_point():
    """Every position wraps into [0, L) and lands on the representable point
    nearest to it on the circle (exact rationals): x - L is exact on [L, 2L),
    and a tiny negative x, whose x + L rounds up to L, is the point 0."""
    for L in (1.0, 4.0 * math.pi, 0.1):
        ulp = np.spacing(L)
        xs = [0.0, -1e-300, -2.0 ** -60 * L, -L, -L + ulp, -0.5 * L, L - ulp, L, L + ulp, 2.0 * L - 2 * ulp,
              2.0 * L, 7.3 * L, -5.1 * L, 1e6 * L + 0.3]
        for x in xs:
            r = O.wrap(x, L)
            assert 0.0 <= r < L, (x, L, r)
            d = (Fraction(r) - Fraction(x)) % Fraction(L)
            d = min(d, Fraction(L) - d)  # distance on the circle
            assert d <= Fraction(np.spacing(max(abs(x), L))), (x, L, r)
    assert O.wrap(-1e-300, 1.0) == 0.0
    assert O.wrap(1.0, 1.0) == 0.0 and O.wrap(-1.0, 1.0) == 0.0


@pytest.mark.parametrize("nc", [1, 2, 3, 4, 8, 13])
def test_deposit_matches_exact_rational(nc):
    """Overlap deposit (eqs. overlap/rho_sum) equals exact rational brute force."""
    rng = np.random.default_rng(100 + nc)
    for L in (Fraction(1), Fraction(3, 2)):
        sheets = _dyadic_sheets(rng, 12, L)
        exact = exact_deposit(L, nc, sheets)
        nts = [len(s[2]) for s in sheets]
        q = [float(s[0]) for s in sheets]
        cl = [1 if s[1] else 0 for s in sheets]
        x = np.array([float(v) for s in sheets for v in s[2]])
        Q, _ = O.deposit(float(L), nc, nts, q, cl, x)
        total = float(sum(s[0] * (len(s[2]) if s[1] else len(s[2]) - 1) for s in sheets))
        err = np.max(np.abs(Q - np.array([float(v) for v in exact])))
        assert err <= 8 * EPS * total, (nc, float(L), err)


def test_deposit_conserves_charge():
    """Every segment deposits exactly its charge (box normalisation, section 2.3)."""
    p = I.random_sheets(7, 40, [int(n) for n in np.random.default_rng(1).integers(2, 300, 40)], 97,
                        L=5.0, jitter=0.8)
    Q, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0)
    nseg = np.where(p.closed == 1, p.n_tracers, p.n_tracers - 1)
    expect = float(np.sum(p.q * nseg))
    assert abs(Q.sum() - expect) <= 64 * EPS * expect


@pytest.mark.parametrize("nt,nc", [(1024, 128), (100, 37), (37, 100), (8, 8)])
def test_uniform_sheet_gives_uniform_density(nt, nc):
    """An unperturbed sheet deposits the same charge into every cell and has no field."""
    L = 2.0 * math.pi
    for shift in (0.0, 0.123, L / nc):
        p = I.uniform_sheet(nt, nc, L, shift=shift)
        Q, _ = O.deposit(p.L, nc, p.n_tracers, p.q, p.closed, p.x0)
        dx = L / nc
        assert np.max(np.abs(Q / dx - 1.0)) < 1e-12
        E, W, _ = O.solve(p.L, nc, Q)
        assert np.max(np.abs(E)) < 1e-12 and W < 1e-24


def test_zero_length_segment_tie_rule():
    """A zero-length segment puts all of its charge into the cell that owns the
    point, a point on a face belonging to the lower cell (W_0 tie rule)."""
    L, nc = 1.0, 8
    Q = O.deposit_segment(0.25, 0.25, 1.0, L, nc)  # on face 2 -> cell 1
    assert Q[1] == 1.0 and Q.sum() == 1.0
    Q = O.deposit_segment(0.0, 0.0, 1.0, L, nc)  # face 0 -> cell -1 = 7
    assert Q[7] == 1.0
    Q = O.deposit_segment(0.3, 0.3, 1.0, L, nc)
    assert Q[2] == 1.0


def test_segment_takes_shorter_way_round():
    L, nc = 1.0, 4
    Q = O.deposit_segment(0.9, 0.1, 1.0, L, nc)  # 0.9 -> 1.1 across the boundary
    np.testing.assert_allclose(Q, [0.5, 0.0, 0.0, 0.5], atol=1e-15)
    Q = O.deposit_segment(0.25, 0.75, 1.0, L, nc)  # exactly L/2: taken downwards, 0.25 -> -0.25
    np.testing.assert_allclose(Q, [0.5, 0.0, 0.0, 0.5], atol=1e-15)


def test_translation_by_one_cell_rolls_the_mesh():
    p = I.random_sheets(3, 10, 200, 64, L=2.0, jitter=0.6)
    dx = p.L / p.n_cells
    Q0, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0)
    xs = np.array([O.wrap(v + dx, p.L) for v in p.x0])
    Q1, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, xs)
    assert np.max(np.abs(Q1 - np.roll(Q0, 1))) < 1e-13


def test_reflection_mirrors_mesh_and_field():
    p = I.random_sheets(4, 10, 150, 50, L=3.0, jitter=0.4)
    Q0, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0)
    xr = np.array([O.wrap(p.L - v, p.L) for v in p.x0])
    Q1, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, xr)
    assert np.max(np.abs(Q1 - Q0[::-1])) < 1e-13
    E0, W0, _ = O.solve(p.L, p.n_cells, Q0)
    E1, W1, _ = O.solve(p.L, p.n_cells, Q1)
    assert np.max(np.abs(E1 + E0[::-1])) < 1e-12 * max(1.0, np.max(np.abs(E0)))
    assert abs(W1 - W0) < 1e-12 * W0


# ---------------------------------------------------------------- solve

@pytest.mark.parametrize("nc", [8, 37, 128, 256, 1024])
def test_poisson_single_mode_closed_form(nc):
    """For rho_j = A cos(k x_j) + B sin(k x_j) the 3-point Poisson equation with a
    centred-difference field gives E_j = sin(k dx) (A sin - B cos)(k x_j) / (dx K^2),
    K = (2/dx) sin(k dx / 2)."""
    L = 7.0
    dx = L / nc
    xc = (np.arange(nc) + 0.5) * dx
    modes = sorted({1, 2, 3, max(1, nc // 3), nc // 2})
    for m in modes:
        k = 2 * math.pi * m / L
        A, B = 0.3, -0.2
        rho = A * np.cos(k * xc) + B * np.sin(k * xc)
        Q = dx * (1.0 + rho)
        E, W, qt = O.solve(L, nc, Q)
        K2 = (2.0 / dx * math.sin(k * dx / 2)) ** 2
        expect = math.sin(k * dx) * (A * np.sin(k * xc) - B * np.cos(k * xc)) / (dx * K2)
        scale = max(1.0, np.max(np.abs(expect)))
        assert np.max(np.abs(E - expect)) < 1e-12 * scale, (nc, m)
        assert abs(W - 0.5 * dx * np.sum(E * E)) < 1e-14 * max(W, 1e-30) + 1e-300


@pytest.mark.parametrize("nc", [16, 33, 200])
def test_poisson_random_density_invariants(nc):
    """For any density: the field has zero mean, no Nyquist component, and its
    centred difference equals the [1, 2, 1]/4 smoothed charge density, which
    together determine E uniquely."""
    rng = np.random.default_rng(nc)
    L = 3.3
    dx = L / nc
    Q = dx * (1.0 + 0.2 * rng.standard_normal(nc))
    E, W, qt = O.solve(L, nc, Q)
    rho = Q / dx - Q.sum() / L
    lhs = (np.roll(E, -1) - np.roll(E, 1)) / (2 * dx)
    rhs = 0.25 * (np.roll(rho, 1) + 2 * rho + np.roll(rho, -1))
    assert np.max(np.abs(lhs - rhs)) < 1e-12
    assert abs(E.sum()) < 1e-12 * nc
    if nc % 2 == 0:
        assert abs(np.sum(E * (-1.0) ** np.arange(nc))) < 1e-12 * nc
    assert abs(qt - Q.sum()) <= 16 * EPS * abs(Q).sum()


# ---------------------------------------------------------------- gather / push

def test_gather_is_first_order_weighting():
    """Brute-force sum over every grid point and its periodic images of
    E_j W_1(x - X_j) (section 2.4) equals the two-point gather."""
    rng = np.random.default_rng(5)
    L, nc = 2.5, 11
    dx = L / nc
    E = rng.standard_normal(nc)
    xs = np.concatenate([rng.uniform(0, L, 200), (np.arange(nc) + 0.5) * dx, np.arange(nc) * dx, [0.0]])
    got = O.gather(L, nc, E, xs)
    for x, g in zip(xs, got):
        s = 0.0
        for img in (-1, 0, 1):
            for j in range(nc):
                Xj = (j + 0.5) * dx + img * L
                w = 1.0 - abs(x - Xj) / dx
                if w > 0:
                    s += E[j] * w
        assert abs(s - g) < 1e-14 * max(1.0, np.max(np.abs(E)))
    nodes = O.gather(L, nc, E, (np.arange(nc) + 0.5) * dx)
    assert np.max(np.abs(nodes - E)) < 8 * EPS * np.max(np.abs(E))


def test_cold_uniform_sheet_is_static_and_drifting_sheet_stays_uniform():
    p = I.uniform_sheet(256, 64, 4.0, v=0.0, n_steps=50)
    r = O.run_problem(p)
    assert np.max(np.abs(r["x"] - p.x0)) < 1e-13
    assert np.max(r["hist"][:, 2]) < 1e-26
    p = I.uniform_sheet(256, 64, 4.0, v=0.37, n_steps=50)
    r = O.run_problem(p)
    expect = np.mod(p.x0 + 0.37 * 50 * p.dt, p.L)
    d = np.abs(r["x"] - expect)
    d = np.minimum(d, p.L - d)
    assert np.max(d) < 1e-12
    assert np.max(r["hist"][:, 2]) < 1e-24


def test_leapfrog_is_reversible():
    """Running the leapfrog map backwards (drift back, then kick back with the
    field recomputed at x^n) recovers the initial state."""
    p = I.landau(n_sheets=16, n_tracers=128, n_cells=64, alpha=0.05, n_steps=40)
    r = O.run_problem(p)
    x, v = r["x"].copy(), r["v"].copy()
    for _ in range(p.n_steps):
        x = np.array([O.wrap(a - p.dt * b, p.L) for a, b in zip(x, v)])
        Q, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, x)
        E, _, _ = O.solve(p.L, p.n_cells, Q)
        v = v - p.dt * O.gather(p.L, p.n_cells, E, x)
    x0 = np.array([O.wrap(a, p.L) for a in p.x0])
    d = np.abs(x - x0)
    d = np.minimum(d, p.L - d)
    assert np.max(d) < 1e-11 * p.L
    Q, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, x0)
    E, _, _ = O.solve(p.L, p.n_cells, Q)
    vhalf0 = p.v0 - 0.5 * p.dt * O.gather(p.L, p.n_cells, E, x0)
    assert np.max(np.abs(v - vhalf0)) < 1e-11


def test_long_segment_flag():
    L = 1.0
    x = np.array([0.0, 0.46, 0.5, 0.7])
    r = O.run(L, 8, 0.01, [4], [0.25], [1], x, np.zeros(4), 0)
    assert int(r["hist"][0, 7]) & 2
    r = O.run(L, 8, 0.01, [4], [0.25], [1], np.array([0.0, 0.25, 0.5, 0.75]), np.zeros(4), 0)
    assert int(r["hist"][0, 7]) == 0


# ---------------------------------------------------------------- physics (section 3)

def test_cold_plasma_oscillation():
    """Single cold sheet (section 3.1): field energy starts at the continuum value
    times the cell-averaging x finite-difference factor [sinc(z) z / tan z]^2,
    oscillates at the plasma frequency, and total energy is conserved."""
    p = I.cold_oscillation()
    r = O.run_problem(p)
    h = r["hist"]
    t, W = h[:, 1], h[:, 2]
    k, a = p.meta["k"], p.meta["alpha"]
    W_cont = 0.5 * (a / k) ** 2 * p.L / 2
    z = k * (p.L / p.n_cells) / 2
    factor = (math.sin(z) / z * z / math.tan(z)) ** 2
    assert abs(W[0] / W_cont - factor) < 5e-5
    tp, lp = log_peaks(t, W, 0.5, t[-1])
    assert len(tp) >= 5
    omega = math.pi / np.mean(np.diff(tp))
    assert abs(omega - 1.0) < 2e-3
    assert np.max(np.abs(np.exp(lp) / W[0] - 1.0)) < 0.03
    total = h[:-1, 2] + h[:-1, 3]
    assert np.max(np.abs(total - total[0])) / np.max(W) < 2e-2
    assert np.max(np.abs(h[:-1, 4])) < 1e-12  # symmetric: momentum stays zero
    assert np.max(np.abs(h[:, 5] - p.L)) < 1e-12 * p.L  # charge conserved


def test_landau_damping_rate_and_frequency():
    """Warm plasma, k = 0.5 (section 3.3): the field energy peaks decay at 2 gamma
    and are spaced pi / omega, with (omega, gamma) the root of the Maxwellian
    dispersion relation."""
    p = I.landau(n_steps=260)
    root = landau_root(0.5)
    assert abs(root.real - 1.41566) < 1e-4 and abs(root.imag + 0.15336) < 1e-4
    r = O.run_problem(p)
    h = r["hist"]
    tp, lp = log_peaks(h[:, 1], h[:, 2], 2.0, 25.0)
    assert len(tp) >= 8
    gamma = np.polyfit(tp, lp, 1)[0] / 2
    omega = math.pi / np.mean(np.diff(tp))
    assert abs(gamma / root.imag - 1.0) < 0.02, gamma
    assert abs(omega / root.real - 1.0) < 0.01, omega
    total = h[:-1, 2] + h[:-1, 3]
    assert np.max(np.abs(total - total[0])) / total[0] < 1e-5


def test_cold_two_stream_growth_rate():
    """Two cold beams of plasma frequency sqrt(1/2) at the fastest-growing k v0
    grow at half the beam plasma frequency (section 3.2)."""
    p = I.cold_two_stream(alpha=1e-7, n_steps=540)
    r = O.run_problem(p)
    t, W = r["hist"][:, 1], r["hist"][:, 2]
    sel = (t >= 14) & (t <= 26)
    gamma = np.polyfit(t[sel], np.log(W[sel]), 1)[0] / 2
    expect = 0.5 * math.sqrt(0.5)
    root = multibeam_root(p.meta["k"], p.sheet_v, p.q * p.n_tracers / p.L, 0.3j)
    assert abs(root.imag - expect) < 1e-12
    assert abs(gamma / expect - 1.0) < 0.01, gamma


def test_warm_two_stream_growth_rate():
    """Warm beams at +-2.4 (v_th 0.5), k = 0.2: growth at the root of the
    discrete multi-beam dispersion relation of the sheets actually loaded."""
    p = I.two_stream(alpha=1e-6, n_sheets=64, n_tracers=1024, n_cells=256, n_steps=600)
    root = multibeam_root(0.2, p.sheet_v, p.q * p.n_tracers / p.L, 0.31j)
    assert abs(root.imag - 0.3132016) < 1e-6
    r = O.run_problem(p)
    t, W = r["hist"][:, 1], r["hist"][:, 2]
    sel = (t >= 16) & (t <= 30)
    gamma = np.polyfit(t[sel], np.log(W[sel]), 1)[0] / 2
    assert abs(gamma / root.imag - 1.0) < 0.02, gamma


def test_nonfinite_state_flags():
    """A non-finite velocity makes the tracer's position non-finite after the
    next move: its two segments deposit nothing, the longest segment and the
    kinetic energy are NaN, and every row from then on has the NONFINITE bit.
    A velocity so large that its kinetic energy overflows, with every
    position still finite, sets the bit through the kinetic energy alone."""
    p = I.landau(n_sheets=4, n_tracers=32, n_cells=16, n_steps=3)
    v0 = np.array(p.v0)
    v0[5] = np.nan
    r = O.run(p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, v0, 3)
    h = r["hist"]
    assert h[0, 7] == 0 and np.isfinite(h[0, 2])
    assert np.all(h[1:, 7] == 1)
    assert np.all(np.isnan(h[1:, 6])) and np.all(np.isfinite(h[1:, 2]))
    assert np.isnan(h[0, 3])  # the move from step 0 had a NaN velocity
    # the two segments of tracer 5 (sheet 0) carry no charge after the move
    assert abs(h[1, 5] - (h[0, 5] - 2 * p.q[0])) < 1e-12 * h[0, 5]
    v0 = np.array(p.v0)
    v0[7] = 1e300
    r = O.run(p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, v0, 2)
    h = r["hist"]
    assert np.all(np.isfinite(r["x"]))
    assert h[0, 7] == 0 and np.isinf(h[0, 3])
    assert np.all(h[1:, 7].astype(int) & 1)
