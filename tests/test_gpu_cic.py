"""First-order (W_1) weighting of segments (deposit_order 2, paper section
2.4) on the GPU against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import envelope_rel, periodic_diff, rel_inf

pytestmark = pytest.mark.gpu
RAGGED = [2, 3, 4, 63, 64, 65, 127, 128, 129, 300]


@pytest.mark.parametrize("nc", [1, 3, 16, 100, 1024, 4096])
def test_cic_deposit_matches_oracle_ragged(nc):
    closed = [1, 1, 0, 1, 0, 1, 1, 0, 1, 1]
    p = I.random_sheets(70 + nc, len(RAGGED), RAGGED, nc, L=2.3, jitter=0.8, closed=closed)
    with B.Simulation(p, deposit_order=2) as s:
        d = s.diagnostics()
    Q, ms = O.deposit(p.L, nc, p.n_tracers, p.q, p.closed, p.x0, order=2)
    dx = p.L / nc
    rho_o = Q / dx - Q.sum() / p.L
    err_rho = np.max(np.abs(d["rho"] - rho_o))
    assert err_rho < 1e-10 * max(1.0, np.max(np.abs(Q / dx)))
    E_o, W_o, qt = O.solve(p.L, nc, Q)
    assert rel_inf(d["E"], E_o) < 1e-10
    assert abs(d["last"]["W_E"] - W_o) <= 1e-10 * W_o
    # the hats sum to one at every point: the total is the segments' charge,
    # held by both sides to rounding
    n_seg = np.where(np.asarray(p.closed) != 0, p.n_tracers, np.asarray(p.n_tracers) - 1)
    exact = float(np.sum(np.asarray(p.q) * n_seg))
    assert abs(qt - exact) < 1e-14 * abs(exact)
    assert abs(d["last"]["total_charge"] - qt) < 1e-12 * abs(qt)
    assert abs(d["last"]["max_segment"] - ms) < 1e-13 * p.L


def test_cic_landau_full_run_fp64():
    p = I.landau()
    ref = O.run_problem(p, order=2)
    with B.Simulation(p, deposit_order=2) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"cic landau fp64 envelope error {err:.3e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_SPLIT_F32])
def test_cic_cold_oscillation_split(prec):
    p = I.cold_oscillation()
    ref = O.run_problem(p, order=2)
    with B.Simulation(p, precision=prec, deposit_order=2) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"cic cold oscillation prec={prec} envelope error {err:.3e}", flush=True)
    assert err < 1e-6
    assert np.all(h["total_charge"] == h["total_charge"][0])


def test_cic_batch_matches_alone_bitwise():
    prec = B.SIC_SPLIT_U32
    probs = [I.landau(n_sheets=8, n_tracers=130, n_cells=64, n_steps=19, alpha=0.1),
             I.two_stream(n_sheets=4, n_tracers=300, n_cells=1024, n_steps=27, alpha=0.05),
             I.random_sheets(12, 3, [2, 65, 128], 50, L=3.0, dt=0.04, n_steps=11, jitter=0.4)]
    b = B.sic_batch_create(sum(p.total_tracers for p in probs), 4, 1024, precision=prec, deposit_order=2)
    try:
        slots = [B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, p.n_steps,
                                   precision=prec, deposit_order=2) for p in probs]
        B.sic_batch_step(b, 30)
        assert sorted(B.sic_batch_poll(b)) == sorted(slots)
        for p, sl in zip(probs, slots):
            with B.Simulation(p, precision=prec, deposit_order=2) as s:
                s.step(p.n_steps)
                x, v, _ = s.state()
                W = s.diagnostics()["history"]["W_E"]
            xb, vb, st = B.sic_batch_get_state(b, sl, p.total_tracers)
            assert st == p.n_steps
            assert np.array_equal(x, xb) and np.array_equal(v, vb)
            assert np.array_equal(W, B.sic_batch_result(b, sl)["history"]["W_E"])
    finally:
        B.sic_batch_destroy(b)
