"""Small simulations run their steps in one resident workgroup (registers and
LDS, one launch per call).  The same steps through the fused two-kernel path
(forced here by timing mode, which always takes it) must give the same
result: the same bits in the split forms, FP64 to the rounding of the
deposit sums.  Runs cross the resident path's launch boundary, alternate the
two paths, and include open sheets, ragged sheets, a one-chunk closed sheet
(its own partner) and per-segment charges."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import envelope_rel, periodic_diff

pytestmark = pytest.mark.gpu


def _ragged():
    return I.random_sheets(17, 6, [64, 2, 65, 130, 37, 300], 48, L=2.5, dt=0.05, jitter=0.6, vscale=0.4,
                           closed=[1, 0, 1, 0, 1, 1])


def _with_charges(p):
    rng = np.random.default_rng(3)
    c = rng.uniform(0.2, 1.0, p.total_tracers) / p.total_tracers
    ends = np.cumsum(p.n_tracers.astype(np.int64)) - 1
    c[ends[p.closed == 0]] = 0.0
    p.c_full = c
    return p


CASES = [
    ("cold", lambda: I.cold_oscillation(n_steps=60)),
    ("ragged", _ragged),
    ("charges", lambda: _with_charges(_ragged())),
    # the largest mesh (16 cells per solve thread) and the smallest (one cell)
    ("cells4096", lambda: I.random_sheets(5, 3, [700, 640, 690], 4096, L=3.0, dt=0.02, jitter=0.3,
                                          vscale=0.2)),
    # the widest workgroup's largest mesh (1024 cells: 8 wavefronts) and one
    # cell more (the 4-wavefront kernel with 16 cells per solve thread)
    ("cells1024", lambda: I.random_sheets(8, 4, [512, 300, 450, 700], 1024, L=2.0, dt=0.03, jitter=0.4,
                                          vscale=0.3)),
    ("cells1025", lambda: I.random_sheets(9, 4, [512, 300, 450, 700], 1025, L=2.0, dt=0.03, jitter=0.4,
                                          vscale=0.3)),
    ("cells1", lambda: I.random_sheets(6, 2, [129, 64], 1, L=1.5, dt=0.05, jitter=0.8, closed=[1, 0])),
]


def _run(p, prec, plan):
    """plan: list of (steps, fused) pieces; fused=True takes the two-kernel path."""
    with B.Simulation(p, precision=prec, history_rows=8400) as s:
        for n, fused in plan:
            B.sic_set_timing(s.h, fused)
            s.step(n)
        x, v, step = s.state()
        d = s.diagnostics()
    return x, v, step, d


@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_SPLIT_F32, B.SIC_FP64])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_resident_steps_equal_fused_steps(name, make, prec):
    p = make()
    assert sum((int(n) + 63) // 64 for n in p.n_tracers) <= 32
    print(f"case {name} prec={prec} tracers={p.total_tracers}", flush=True)
    xa, va, sa, da = _run(p, prec, [(37, False), (5, True), (11, False)])
    xb, vb, sb, db = _run(p, prec, [(53, True)])
    assert sa == sb == 53
    ha, hb = da["history"], db["history"]
    ke_a, ke_b = ha["KE"][:-1], hb["KE"][:-1]
    # the kinetic-energy and momentum sums run in another order
    assert np.max(np.abs(ke_a - ke_b)) <= 1e-12 * np.max(np.abs(ke_b))
    assert np.max(np.abs(ha["momentum"][:-1] - hb["momentum"][:-1])) <= 1e-12 * max(np.max(np.abs(ke_b)), 1e-300)
    if prec == B.SIC_FP64:
        assert np.max(periodic_diff(xa, xb, p.L)) < 1e-12 * p.L
        assert np.max(np.abs(va - vb)) < 1e-12 * max(1.0, np.max(np.abs(vb)))
        if np.max(hb["W_E"]) > 0.0:
            assert envelope_rel(ha["W_E"], hb["W_E"], p.dt) < 1e-11
        else:  # one cell: no field
            assert np.max(ha["W_E"]) == 0.0
        assert np.max(np.abs(ha["max_segment"] - hb["max_segment"])) < 1e-12 * p.L
    else:
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
        assert np.array_equal(ha["W_E"], hb["W_E"])
        assert np.array_equal(ha["total_charge"], hb["total_charge"])
        assert np.array_equal(ha["max_segment"], hb["max_segment"])
        assert np.array_equal(da["E"], db["E"]) and np.array_equal(da["rho"], db["rho"])
    np.testing.assert_array_equal(ha["step"], hb["step"])
    assert np.all(np.isnan(ha["KE"][-1:])) and np.all(np.isnan(hb["KE"][-1:]))


def test_resident_run_across_launches_equals_fused():
    """More steps than one resident launch takes (8192): split U32, so the
    resident and the fused paths must agree to the bit through the launch
    boundary."""
    p = I.cold_oscillation(n_steps=8300)
    xa, va, sa, da = _run(p, B.SIC_SPLIT_U32, [(8300, False)])
    xb, vb, sb, db = _run(p, B.SIC_SPLIT_U32, [(8300, True)])
    assert sa == sb == 8300
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert np.array_equal(da["history"]["W_E"], db["history"]["W_E"])


def test_resident_cold_oscillation_matches_oracle():
    """500 steps: within the horizon where the oracle itself still answers a
    1-ulp change of one position below 1e-12 (2.7e-13 at step 500, 3.4e-7 at
    1000, 0.56 at 2000: grid heating drives the sheet model chaotic)."""
    p = I.cold_oscillation(n_steps=500)
    ref = O.run_problem(p, 500)
    with B.Simulation(p, history_rows=501) as s:
        s.step(500)
        h = s.diagnostics()["history"]
    assert len(h) == 501
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"cold oscillation 500 steps, resident: field-energy envelope error {err:.3e}", flush=True)
    assert err < 1e-10
