"""Split-precision forms (integer cell index + float32 offset within a
sub-cell of 2^-20 cell, or + uint32 fraction of a cell; int64 fixed-point
deposit; float64 solve) against the FP64 oracle, plus the properties the
fixed-point deposit guarantees: exact charge conservation, bitwise
reproducibility and exact translation invariance."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import envelope_rel, periodic_diff

pytestmark = pytest.mark.gpu
SPLITS = [B.SIC_SPLIT_F32, B.SIC_SPLIT_U32]
FIELD_ENERGY_TOL = 1e-6  # relative (envelope) field-energy error over the run


def _run(p, prec, steps):
    with B.Simulation(p, precision=prec) as s:
        s.step(steps)
        x, v, step = s.state()
        d = s.diagnostics()
    return x, v, d


@pytest.mark.parametrize("prec", SPLITS)
def test_cold_oscillation_split_field_energy(prec):
    p = I.cold_oscillation()
    ref = O.run_problem(p)
    x, v, d = _run(p, prec, p.n_steps)
    err = envelope_rel(d["history"]["W_E"], ref["hist"][:, 2], p.dt)
    print(f"prec={prec} cold oscillation W_E envelope-relative error {err:.3e}", flush=True)
    assert err < FIELD_ENERGY_TOL


@pytest.mark.parametrize("prec", SPLITS)
def test_landau_split_field_energy(prec):
    p = I.landau()
    ref = O.run_problem(p)
    x, v, d = _run(p, prec, p.n_steps)
    W = d["history"]["W_E"]
    Wr = ref["hist"][:, 2]
    err = envelope_rel(W, Wr, p.dt)
    glob = float(np.max(np.abs(W - Wr)) / np.max(Wr))
    print(f"prec={prec} landau W_E envelope-relative {err:.3e} global {glob:.3e}", flush=True)
    assert err < FIELD_ENERGY_TOL


@pytest.mark.parametrize("prec", SPLITS)
def test_split_charge_exactly_conserved_and_bitwise_reproducible(prec):
    p = I.two_stream(n_sheets=32, n_tracers=512, n_cells=256, n_steps=300, alpha=0.05)
    runs = [_run(p, prec, p.n_steps) for _ in range(2)]
    (x0, v0, d0), (x1, v1, d1) = runs
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    h0, h1 = d0["history"], d1["history"]
    assert np.array_equal(h0["W_E"], h1["W_E"])
    assert np.array_equal(d0["rho"], d1["rho"]) and np.array_equal(d0["E"], d1["E"])
    # the fixed-point total is the same integer at every step
    assert np.all(h0["total_charge"] == h0["total_charge"][0])
    assert abs(h0["total_charge"][0] - p.L) < 1e-12 * p.L


def test_split_u32_translation_by_one_cell_rolls_density_bitwise():
    nc = 64
    p = I.random_sheets(11, 6, [100, 64, 65, 300, 2, 128], nc, L=float(nc), jitter=0.6)
    shifted = I.random_sheets(11, 6, [100, 64, 65, 300, 2, 128], nc, L=float(nc), jitter=0.6)
    shifted.x_full = np.mod(p.x0 + 1.0, p.L)
    with B.Simulation(p, precision=B.SIC_SPLIT_U32) as a, B.Simulation(shifted, precision=B.SIC_SPLIT_U32) as b:
        ra = a.diagnostics()["rho"]
        rb = b.diagnostics()["rho"]
    assert np.array_equal(np.roll(ra, 1), rb)


@pytest.mark.parametrize("prec", SPLITS)
def test_split_single_step_resync(prec):
    """From an oracle state, one split step stays within the quantisation of
    positions (2^-44 or 2^-32 of a cell; the F32 bound also covers the
    oracle's own float64 rounding of a position, about 2^-44 of a cell here)
    of the oracle step, and its field energy within the split forms' 1e-6."""
    p = I.landau(n_sheets=32, n_tracers=256, n_cells=128, n_steps=60)
    ref60 = O.run_problem(p, 60)
    ref61 = O.run(p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, ref60["x"], ref60["v"], 1, step0=60,
                  init_kick=False)
    with B.Simulation(p, precision=prec) as s:
        s.set_state(60, ref60["x"], ref60["v"])
        s.step(1)
        x, v, step = s.state()
        d = s.diagnostics()
    dx = p.L / p.n_cells
    q = 2.0 ** -41 if prec == B.SIC_SPLIT_F32 else 2.0 ** -31
    assert step == 61
    err_x = np.max(periodic_diff(x, ref61["x"], p.L)) / dx
    Wr = ref61["hist"][-1, 2]
    err_w = abs(d["last"]["W_E"] - Wr) / Wr
    print(f"prec={prec} resync step: position error {err_x:.3e} cell, W_E {err_w:.3e}", flush=True)
    assert err_x < 4 * q
    assert err_w < FIELD_ENERGY_TOL
