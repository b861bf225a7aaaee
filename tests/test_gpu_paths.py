"""Launch paths of a single simulation's steps: the resident launch of a
small simulation gives the fused launches' bits in the split forms and the
same run to rounding in FP64; sic_last_step_path reports the path taken and
fused_only forces the fused launches."""
import numpy as np
import pytest

from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import periodic_diff

pytestmark = pytest.mark.gpu


def _run(p, prec, steps, fused_only):
    with B.Simulation(p, precision=prec) as s:
        assert B.sic_last_step_path(s.h) == B.SIC_PATH_NONE
        B.sic_set_tuning(s.h, fused_only=fused_only)
        assert B.sic_get_tuning(s.h)["fused_only"] == fused_only
        s.step(steps)
        path = B.sic_last_step_path(s.h)
        x, v, st = s.state()
        d = s.diagnostics()
    return path, x, v, st, d


@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_SPLIT_F32, B.SIC_FP64])
def test_resident_and_fused_paths_agree(prec):
    # 8 sheets of 250 tracers: 32 chunks, the largest resident simulation
    p = I.landau(n_sheets=8, n_tracers=250, n_cells=64, alpha=0.05)
    print(f"case resident vs fused prec={prec}", flush=True)
    r = _run(p, prec, 80, 0)
    f = _run(p, prec, 80, 1)
    assert r[0] == B.SIC_PATH_RESIDENT and f[0] == B.SIC_PATH_FUSED
    assert r[3] == f[3] == 80
    if prec == B.SIC_FP64:
        assert np.max(periodic_diff(r[1], f[1], p.L)) < 1e-11 * p.L
        np.testing.assert_allclose(r[4]["history"]["W_E"], f[4]["history"]["W_E"], rtol=1e-10)
    else:
        assert np.array_equal(r[1], f[1]) and np.array_equal(r[2], f[2])
        assert np.array_equal(r[4]["history"]["W_E"], f[4]["history"]["W_E"])


def test_larger_simulation_takes_the_solve_first_path():
    p = I.landau(n_sheets=64, n_tracers=256, n_cells=64)
    path, *_ = _run(p, B.SIC_FP64, 3, 0)
    assert path == B.SIC_PATH_SOLVE_FIRST
    path, *_ = _run(p, B.SIC_FP64, 3, 1)
    assert path == B.SIC_PATH_FUSED


def _timed_classic(p, prec, steps):
    """The same steps as tracer/solve launch pairs (timing mode)."""
    with B.Simulation(p, precision=prec) as s:
        B.sic_set_timing(s.h, True)
        s.step(steps)
        assert B.sic_last_step_path(s.h) == B.SIC_PATH_FUSED
        x, v, st = s.state()
        d = s.diagnostics()
    return x, v, st, d


SF_CASES = {
    # 2048 chunks on 256 cells (one solve thread per cell)
    "landau_256x512": lambda: I.landau(),
    # ragged sheets, 100 cells
    "ragged_37x300": lambda: I.landau(n_sheets=37, n_tracers=300, n_cells=100, alpha=0.05),
    # 1024 cells (four cells per solve thread), two-stream
    "two_stream_64x1024": lambda: I.two_stream(n_sheets=64, n_tracers=1024, n_cells=1024, n_steps=100),
    # 4096 cells (16 cells per solve thread; a work item's LDS above 64 KB)
    "landau_32x1024_4096cells": lambda: I.landau(n_sheets=32, n_tracers=1024, n_cells=4096, n_steps=60),
}


@pytest.mark.parametrize("case", sorted(SF_CASES))
@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_SPLIT_F32, B.SIC_FP64])
def test_solve_first_steps_give_the_fused_bits(case, prec):
    """Steps in calls of 1, 2, 33 and 9 (graphs of one step, of two, across
    the 32-step graph size, and a remainder), then one launch pair, against
    46 steps of launch pairs: the same state, history rows and step count."""
    p = SF_CASES[case]()
    print(f"case solve-first {case} prec={prec}", flush=True)
    with B.Simulation(p, precision=prec) as s:
        for n in (1, 2, 33, 9):
            s.step(n)
            assert B.sic_last_step_path(s.h) == B.SIC_PATH_SOLVE_FIRST
        # one more step as a launch pair: it deposits into the pool's own
        # accumulators, which the solve-first steps must have left clear
        B.sic_set_timing(s.h, True)
        s.step(1)
        x, v, st = s.state()
        d = s.diagnostics()
    xr, vr, sr, dr = _timed_classic(p, prec, 46)
    assert st == sr == 46
    h, hr = d["history"], dr["history"]
    assert np.array_equal(h["step"], hr["step"])
    if prec == B.SIC_FP64:
        # float64 atomics may add in another order
        assert np.max(periodic_diff(x, xr, p.L)) < 1e-11 * p.L
        np.testing.assert_allclose(h["W_E"], hr["W_E"], rtol=1e-10)
        np.testing.assert_allclose(h["KE"][:-1], hr["KE"][:-1], rtol=1e-12)
    else:
        assert np.array_equal(x, xr) and np.array_equal(v, vr)
        for col in ("W_E", "KE", "momentum", "total_charge", "max_segment"):
            assert np.array_equal(h[col], hr[col], equal_nan=True), col
        assert np.array_equal(h["flags"], hr["flags"])


def test_refining_simulation_reports_its_path():
    p = I.two_stream(n_sheets=8, n_tracers=64, n_cells=64, n_steps=5)
    with B.Simulation(p, l_max=p.L / 16, max_tracers=16 * p.total_tracers) as s:
        s.step(3)
        assert B.sic_last_step_path(s.h) == B.SIC_PATH_REFINING


def test_single_simulation_launch_shapes_and_paths():
    """The item rules of a single simulation and the path they lead to:
    256-cell Landau, 256 items of 8 chunks (one per CU); two-stream on 1024
    cells, 512 items of 64 chunks; a million tracers on 100 cells, items
    capped at 256 (contention on a small mesh) instead of 2048; a 4096-cell
    simulation of 2048 workgroups keeps the launch pairs (solve-first only up
    to 512)."""
    cases = [
        (I.landau(), 8, 512, 256, B.SIC_PATH_SOLVE_FIRST),
        (I.two_stream(n_steps=2), 64, 512, 512, B.SIC_PATH_SOLVE_FIRST),
        (I.landau(n_sheets=2, n_tracers=524288, n_cells=100, n_steps=2), 64, 512, 256, B.SIC_PATH_SOLVE_FIRST),
        (I.landau(n_sheets=2048, n_tracers=16384, n_cells=4096, n_steps=2), 256, 1024, 2048, B.SIC_PATH_FUSED),
    ]
    for p, tile, block, grid, path in cases:
        print(f"case shapes {p.n_sheets}x{int(p.n_tracers[0])} on {p.n_cells} cells", flush=True)
        with B.Simulation(p, precision=B.SIC_FP64, history_rows=8) as s:
            t = B.sic_get_tuning(s.h)
            assert (t["tile_chunks"], t["block_threads"], t["grid_blocks"]) == (tile, block, grid)
            s.step(2)
            assert B.sic_last_step_path(s.h) == path
