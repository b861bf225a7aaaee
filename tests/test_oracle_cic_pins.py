"""Pins of the oracle's first-order weighting of segments (paper section 2.4)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import inputs as I
from tests.exact_deposit import exact_deposit_cic
from tests.test_oracle_pins import _dyadic_sheets

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("nc", [1, 2, 3, 4, 8, 13])
def test_cic_deposit_matches_exact_rational(nc):
    rng = np.random.default_rng(900 + nc)
    for L in (Fraction(1), Fraction(7, 4)):
        sheets = _dyadic_sheets(rng, 12, L)
        exact = exact_deposit_cic(L, nc, sheets)
        nts = [len(s[2]) for s in sheets]
        q = [float(s[0]) for s in sheets]
        cl = [1 if s[1] else 0 for s in sheets]
        x = np.array([float(v) for s in sheets for v in s[2]])
        Q, _ = O.deposit(float(L), nc, nts, q, cl, x, order=2)
        total = float(sum(s[0] * (len(s[2]) if s[1] else len(s[2]) - 1) for s in sheets))
        err = np.max(np.abs(Q - np.array([float(v) for v in exact])))
        assert err <= 16 * EPS * total, (nc, float(L), err)


def test_cic_deposit_conserves_charge_and_keeps_uniform_sheets_uniform():
    p = I.random_sheets(21, 25, [int(n) for n in np.random.default_rng(8).integers(2, 200, 25)], 61, L=3.0,
                        jitter=0.8, closed=[int(c) for c in np.random.default_rng(9).integers(0, 2, 25)])
    Q, _ = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0, order=2)
    nseg = np.where(p.closed == 1, p.n_tracers, p.n_tracers - 1)
    assert abs(Q.sum() - np.sum(p.q * nseg)) < 1e-13 * np.sum(p.q * nseg)
    for nt, nc, shift in [(100, 37, 0.01), (5, 64, 0.3), (1024, 128, 0.0)]:
        u = I.uniform_sheet(nt, nc, 3.0, shift=shift)
        Q, _ = O.deposit(u.L, nc, u.n_tracers, u.q, u.closed, u.x0, order=2)
        assert np.max(np.abs(Q / (u.L / nc) - 1.0)) < 1e-12


def test_short_segment_tends_to_the_cic_point_weights():
    """A segment of length eps away from a grid point deposits the
    first-order (CIC) weights of its midpoint up to O(eps^2) (the hat is
    linear there); centred on a grid point, where the hat has its kink, the
    grid point gets 1 - eps/(4 dx) and each neighbour eps/(8 dx)."""
    L, nc = 1.0, 10
    dx = L / nc
    eps = 1e-4
    Q, _ = O.deposit(L, nc, [2], [1.0], [0], np.array([0.55 - eps / 2, 0.55 + eps / 2]), order=2)
    assert abs(Q[5] - (1 - eps / (4 * dx))) < 1e-12
    assert abs(Q[4] - eps / (8 * dx)) < 1e-12 and abs(Q[6] - eps / (8 * dx)) < 1e-12
    for m in (0.123, 0.5712, 0.0777, 0.999):
        for eps in (1e-4, 1e-5):
            Q = np.zeros(nc)
            Q, _ = O.deposit(L, nc, [2], [1.0], [0], np.array([m - eps / 2, m + eps / 2]) % L, order=2)
            expect = np.zeros(nc)
            j0 = int(np.floor(m / dx - 0.5))
            s = m / dx - 0.5 - j0
            expect[j0 % nc] += 1 - s
            expect[(j0 + 1) % nc] += s
            assert np.max(np.abs(Q - expect)) < 10 * (eps / dx) ** 2 + 1e-12


@pytest.mark.parametrize("nc", [1024, 4096])
def test_cic_deposit_conserves_charge_on_fine_meshes(nc):
    """The hats sum to one at every point, so the W_1 deposit of a segment is
    exactly its charge.  Short jittered segments on a fine mesh (lengths down
    to a small fraction of a cell, folds) keep the total to rounding."""
    ragged = [2, 3, 4, 63, 64, 65, 127, 128, 129, 300]
    closed = [1, 1, 0, 1, 0, 1, 1, 0, 1, 1]
    p = I.random_sheets(70 + nc, len(ragged), ragged, nc, L=2.3, jitter=0.8, closed=closed)
    Q, _ = O.deposit(p.L, nc, p.n_tracers, p.q, p.closed, p.x0, order=2)
    nseg = np.where(np.asarray(p.closed) == 1, p.n_tracers, np.asarray(p.n_tracers) - 1)
    exact = float(np.sum(np.asarray(p.q) * nseg))
    assert abs(Q.sum() - exact) < 1e-14 * exact
    # and segment by segment: a single short segment anywhere on the mesh
    rng = np.random.default_rng(nc)
    dx = p.L / nc
    for _ in range(200):
        a = rng.uniform(0, p.L)
        b = (a + rng.choice([-1.0, 1.0]) * dx * 10.0 ** rng.uniform(-9, 0.5)) % p.L
        Q, _ = O.deposit(p.L, nc, [2], [1.0], [0], np.array([a, b]), order=2)
        assert abs(Q.sum() - 1.0) < 4 * EPS and np.all(Q >= -4 * EPS)
