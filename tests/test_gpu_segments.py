"""Per-segment charges, vertically connected sheets (paper section 3.3.2)
and refinement (section 2.6) on the GPU against the oracle."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import envelope_rel, periodic_diff, rel_inf

pytestmark = pytest.mark.gpu
RAGGED = [2, 3, 4, 63, 64, 65, 127, 128, 129, 300]
CLOSED = [1, 0, 0, 1, 0, 1, 0, 1, 1, 0]


def _random_charges(p, seed):
    """Charges that differ from segment to segment (0 for the last tracer of
    an open sheet)."""
    rng = np.random.default_rng(seed)
    c = p.seg_charges * rng.uniform(0.3, 3.0, p.total_tracers)
    ends = np.cumsum(p.n_tracers) - 1
    c[ends[p.closed == 0]] = 0.0
    return c


@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("nc", [1, 2, 16, 100, 1024, 4096])
def test_segment_charge_deposit_matches_oracle(order, nc):
    p = I.random_sheets(300 + nc, len(RAGGED), RAGGED, nc, L=1.9, jitter=0.5, closed=CLOSED)
    c = _random_charges(p, nc)
    print(f"case segment charges order={order} nc={nc}", flush=True)
    with B.Simulation(p, deposit_order=order, seg_charges=c) as s:
        d = s.diagnostics()
        back = s.charges()
    assert np.array_equal(back, c)
    Q, ms = O.deposit(p.L, nc, p.n_tracers, p.q, p.closed, p.x0, order=order, c=c)
    dx = p.L / nc
    rho_o = Q / dx - Q.sum() / p.L
    err_rho = np.max(np.abs(d["rho"] - rho_o))
    tol = 1e-10 * max(1.0, np.max(np.abs(Q / dx)))
    if order == 1:
        # piecewise-linear gradients divide by segment lengths: next to a
        # nearly degenerate segment two correct FP64 deposits differ by as
        # much as the oracle moves under one-ulp position changes
        rng = np.random.default_rng(0)
        for _ in range(4):
            x2 = np.mod(p.x0 + rng.choice([-1.0, 0.0, 1.0], len(p.x0)) * np.spacing(p.x0), p.L)
            Q2, _ = O.deposit(p.L, nc, p.n_tracers, p.q, p.closed, x2, order=1, c=c)
            tol = max(tol, 4.0 * float(np.max(np.abs(Q2 - Q))) / dx)
    print(f"  |drho| {err_rho:.3e} tolerance {tol:.3e}", flush=True)
    assert err_rho < tol
    E_g, _, _ = O.solve(p.L, nc, d["rho"] * dx)
    assert rel_inf(d["E"], E_g) < 1e-10 or np.max(np.abs(E_g)) < 1e-14
    total = math.fsum(c)
    assert abs(d["last"]["total_charge"] - total) < 1e-11 * total
    assert abs(d["last"]["max_segment"] - ms) < 1e-13 * p.L


@pytest.mark.parametrize("use_c", [False, True])
def test_open_sheet_masses_and_steps_match_oracle(use_c):
    """Kinetic energy and momentum use tracer masses of half of each
    bounding segment, so an open sheet's end tracers weigh half; the same
    holds with per-segment charges."""
    p = I.random_sheets(41, 6, [2, 70, 3, 130, 64, 65], 40, L=2.0, jitter=0.3, vscale=0.4, dt=0.05,
                        closed=[0, 0, 1, 0, 1, 0])
    c = _random_charges(p, 5) if use_c else p.seg_charges
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, c, p.x0, p.v0, 6)
    with B.Simulation(p, seg_charges=c if use_c else None) as s:
        s.step(6)
        x, v, _ = s.state()
        h = s.diagnostics()["history"]
    assert np.max(periodic_diff(x, ref["x"], p.L)) < 1e-12 * p.L
    for n in range(6):
        for col, k in (("W_E", 2), ("KE", 3), ("momentum", 4)):
            r = ref["hist"][n, k]
            assert abs(h[col][n] - r) <= 1e-10 * max(abs(r), 1e-12), (col, n, h[col][n], r)


@pytest.mark.parametrize("order", [0, 2])
def test_vertical_landau_fp64_matches_oracle(order):
    p = I.landau_vertical(n_streams=26, n_positions=160, n_cells=40, n_steps=200)
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, order=order)
    with B.Simulation(p, deposit_order=order) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
        x, _, _ = s.state()
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"vertical landau order={order} fp64 envelope error {err:.3e}", flush=True)
    assert err < 1e-10
    assert np.max(periodic_diff(x, ref["x"], p.L)) < 1e-10 * p.L


def test_vertical_landau_linear_segments_fp64():
    """Piecewise-linear segments on vertical sheets: the neighbours' charges
    differ from segment to segment, and the zero-length start drops every
    gradient until the sheets have stretched."""
    p = I.landau_vertical(n_streams=26, n_positions=160, n_cells=40, n_steps=120)
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, order=1)
    with B.Simulation(p, deposit_order=1) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"vertical landau linear fp64 envelope error {err:.3e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_SPLIT_F32])
def test_vertical_landau_split(prec):
    p = I.landau_vertical(n_streams=26, n_positions=160, n_cells=40, n_steps=200)
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps)
    with B.Simulation(p, precision=prec) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"vertical landau prec={prec} envelope error {err:.3e}", flush=True)
    assert err < 1e-6
    assert np.all(h["total_charge"] == h["total_charge"][0])


def test_refine_pass_matches_oracle_exactly():
    """One refinement pass on the GPU inserts the same tracers, at the same
    positions, with the same velocities and charges as the oracle's."""
    p = I.random_sheets(77, 5, [40, 3, 64, 129, 9], 50, L=2.5, jitter=1.5, closed=[1, 0, 1, 1, 0])
    dx = p.L / p.n_cells
    c = p.seg_charges
    with B.Simulation(p, l_max=0.0, seg_charges=c, max_tracers=4 * p.total_tracers) as s:
        x0, v0, _ = s.state()
        added = s.refine(0.8 * dx)
        nt, tot = s.layout()
        x, v, _ = s.state()
        cc = s.charges()
        d = s.diagnostics()
    nt_o, x_o, v_o, c_o, add_o = O.refine(p.L, 0.8 * dx, p.n_tracers, p.closed, x0, v0, c)
    assert added == add_o > 20
    assert np.array_equal(nt, nt_o) and tot == len(x_o)
    assert np.array_equal(x, x_o) and np.array_equal(v, v_o) and np.array_equal(cc, c_o)
    Q, ms = O.deposit(p.L, p.n_cells, nt_o, p.q, p.closed, x_o, c=c_o)
    rho_o = Q / dx - Q.sum() / p.L
    assert np.max(np.abs(d["rho"] - rho_o)) < 1e-10 * np.max(np.abs(Q / dx))
    assert abs(d["last"]["max_segment"] - ms) < 1e-13 * p.L


def test_refinement_run_matches_oracle():
    """The section 2.6 two-stream run with refinement at one cell, through
    the onset of refinement: the GPU inserts the same tracers at every step
    (same count history) and its field energy follows the oracle's."""
    p = I.refinement_two_stream(n_steps=340)
    dx = p.L / p.n_cells
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, l_max=dx,
                    capacity=200_000)
    counts = [p.total_tracers]
    print(f"case refinement run, oracle final count {ref['count'][-1]}", flush=True)
    with B.Simulation(p, l_max=dx, max_tracers=200_000) as s:
        for _ in range(p.n_steps):
            s.step(1)
            counts.append(s.n)
        h = s.diagnostics()["history"]
        nt, _ = s.layout()
    assert ref["count"][-1] > 1.05 * ref["count"][0]  # refinement has started
    assert np.array_equal(np.array(counts), ref["count"])
    assert np.array_equal(nt, ref["n_tracers"])
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"refinement run envelope error {err:.3e}", flush=True)
    assert err < 1e-10
    assert np.max(np.abs(h["total_charge"] - ref["hist"][:, 5])) < 1e-12 * ref["hist"][0, 5]


def test_refinement_run_in_one_call_matches_oracle():
    """The same run as one sic_step call: refinement runs on the device after
    every move, with no host round trip between steps, and ends with the
    oracle's sheets, field-energy history and total charge."""
    p = I.refinement_two_stream(n_steps=340)
    dx = p.L / p.n_cells
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, l_max=dx,
                    capacity=200_000)
    print(f"case refinement run in one call, oracle final count {ref['count'][-1]}", flush=True)
    with B.Simulation(p, l_max=dx, max_tracers=200_000) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
        nt, tot = s.layout()
        x, v, step = s.state()
        c = s.charges()
    assert step == p.n_steps and tot == ref["count"][-1]
    assert np.array_equal(nt, ref["n_tracers"])
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"refinement run in one call: envelope error {err:.3e}", flush=True)
    assert err < 1e-10
    assert np.max(np.abs(h["total_charge"] - ref["hist"][:, 5])) < 1e-12 * ref["hist"][0, 5]
    assert np.array_equal(c, ref["c"])  # halved charges, exact in float64
    assert np.max(periodic_diff(x, ref["x"], p.L)) < 1e-9 * p.L


@pytest.mark.parametrize("prec", [B.SIC_FP64, B.SIC_SPLIT_U32])
def test_refinement_in_one_call_equals_step_by_step(prec):
    """Stepping 300 steps in one call (device refinement) and one step per
    call give the same insertions and, in the split form, the same bits."""
    p = I.refinement_two_stream(n_steps=300)
    dx = p.L / p.n_cells
    outs = []
    for per_call in (p.n_steps, 1):
        with B.Simulation(p, precision=prec, l_max=dx, max_tracers=200_000) as s:
            for _ in range(p.n_steps // per_call):
                s.step(per_call)
            x, v, _ = s.state()
            outs.append((s.layout()[0], x, v, s.charges(), s.diagnostics()["history"]["W_E"]))
    (nt1, x1, v1, c1, W1), (nt2, x2, v2, c2, W2) = outs
    assert np.array_equal(nt1, nt2) and np.array_equal(c1, c2)
    if prec == B.SIC_FP64:
        assert np.max(periodic_diff(x1, x2, p.L)) < 1e-10 * p.L
        assert np.max(np.abs(W1 - W2) / np.max(W2)) < 1e-10
    else:
        assert np.array_equal(x1, x2) and np.array_equal(v1, v2) and np.array_equal(W1, W2)


def test_refinement_over_capacity_during_steps_stops_there():
    """A run whose refinement outgrows its capacity stops at the step whose
    pass would not fit: that pass inserts nothing, sic_step reports
    SIC_ENOMEM, and the simulation keeps the tracers of the last pass that
    fitted, as the oracle's count history gives them."""
    p = I.refinement_two_stream(n_steps=340)
    dx = p.L / p.n_cells
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, l_max=dx,
                    capacity=200_000)
    cap = int(ref["count"][0] + (ref["count"][-1] - ref["count"][0]) // 2)
    m = int(np.nonzero(ref["count"] > cap)[0][0])  # the first step whose pass does not fit
    with B.Simulation(p, l_max=dx, max_tracers=cap) as s:
        with pytest.raises(B.SicError) as e:
            s.step(p.n_steps)
        assert e.value.status == 2
        x, v, step = s.state()
        _, tot = s.layout()
        assert step == m and tot == ref["count"][m - 1]
        # the simulation is usable afterwards: a step without refinement room fails the same way
        with pytest.raises(B.SicError):
            s.step(1)


def _envelope_errors(W, Wr, dt):
    P = int(math.ceil(2 * math.pi / dt))
    env = np.array([np.max(Wr[max(0, i - P): i + P + 1]) for i in range(len(Wr))])
    return np.abs(W - Wr) / env


@pytest.mark.parametrize("order", [1, 2])
def test_refinement_run_other_deposit_orders_match_oracle(order):
    """Refinement with piecewise-linear segments (whose gradients read the
    neighbouring segments' charges, halved by splits) and with first-order
    weighting, through the onset of refinement.

    In the folded vortex the piecewise-linear gradients divide by small
    centroid separations, and the run is chaotic: the oracle itself departs
    from its own history once its initial positions move by one ulp.  The
    GPU's deposit differs from the oracle's by rounding in every step, so
    its error grows the same way: the field energy is held to 1e-10 up to
    the step where the oracle's own departure under perturbations of a few
    ulps first reaches 1e-11 (a decade of margin, measured here), and past
    it oracle-resynchronised single steps are held to 1e-10."""
    p = I.refinement_two_stream(n_steps=320)
    dx = p.L / p.n_cells
    kw = dict(l_max=dx, capacity=200_000, order=order)
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, **kw)
    # the predictability horizon: the earliest step at which one of three
    # oracle runs from initial positions moved by up to two ulps departs from
    # the reference by 1e-11
    horizon = p.n_steps + 1
    for seed in (1, 2, 3):
        rng = np.random.default_rng(seed)
        x_ulp = p.x0 + rng.choice([-2.0, -1.0, 0.0, 1.0, 2.0], len(p.x0)) * np.spacing(p.x0)
        own = _envelope_errors(O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, x_ulp,
                                         p.v0, p.n_steps, **kw)["hist"][:, 2], ref["hist"][:, 2], p.dt)
        if np.any(own > 1e-11):
            horizon = min(horizon, int(np.argmax(own > 1e-11)))
    with B.Simulation(p, l_max=dx, max_tracers=200_000, deposit_order=order) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
        nt, tot = s.layout()
        print(f"refinement order={order}: {tot} tracers (oracle {ref['count'][-1]})", flush=True)
        assert ref["count"][-1] > ref["count"][0]
        assert np.array_equal(nt, ref["n_tracers"])
        err = _envelope_errors(h["W_E"], ref["hist"][:, 2], p.dt)
        print(f"refinement order={order}: oracle's own 1-ulp horizon step {horizon}; GPU error up to it "
              f"{err[:horizon].max():.3e}, whole run {err.max():.3e}", flush=True)
        assert err[:horizon].max() < 1e-10
        for target in (290, 305, 320):
            if target < horizon:
                continue
            st = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, target, **kw)
            one = O.run_seg(p.L, p.n_cells, p.dt, st["n_tracers"], p.closed, st["c"], st["x"], st["v"], 1,
                            step0=target, init_kick=False, **kw)
            s.load_state(target, st["n_tracers"], st["x"], st["v"], st["c"])
            s.step(1)
            nt1, _ = s.layout()
            x1, _, _ = s.state()
            W1 = s.diagnostics(history=False)["last"]["W_E"]
            assert np.array_equal(nt1, one["n_tracers"]), target
            assert np.max(periodic_diff(x1, one["x"], p.L)) < 1e-12 * p.L
            assert abs(W1 - one["hist"][-1, 2]) <= 1e-10 * one["hist"][-1, 2], (target, W1, one["hist"][-1, 2])


def test_refinement_resynchronised_steps_deep_in_the_nonlinear_phase():
    """At steps 300, 400 and 500 of the refined two-stream run the GPU is
    loaded with the oracle's refined state (sic_load_state) and takes one
    step with refinement: same insertions, same positions, same field
    energy."""
    p = I.refinement_two_stream(n_steps=500)
    dx = p.L / p.n_cells
    cap = 2_000_000
    with B.Simulation(p, l_max=dx, max_tracers=cap) as s:
        for target in (300, 400, 500):
            st = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, target,
                           l_max=dx, capacity=cap)
            one = O.run_seg(p.L, p.n_cells, p.dt, st["n_tracers"], p.closed, st["c"], st["x"], st["v"], 1,
                            step0=target, init_kick=False, l_max=dx, capacity=cap)
            s.load_state(target, st["n_tracers"], st["x"], st["v"], st["c"])
            s.step(1)
            nt, tot = s.layout()
            x, v, step = s.state()
            W = s.diagnostics(history=False)["last"]["W_E"]
            assert step == target + 1
            assert np.array_equal(nt, one["n_tracers"]), target
            assert np.max(periodic_diff(x, one["x"], p.L)) < 1e-12 * p.L
            assert abs(W - one["hist"][-1, 2]) <= 1e-10 * one["hist"][-1, 2]
            print(f"resync at {target}: {tot} tracers", flush=True)


def test_refinement_split_conserves_charge_exactly():
    p = I.refinement_two_stream(n_steps=360)
    dx = p.L / p.n_cells
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, l_max=dx,
                    capacity=200_000)
    with B.Simulation(p, precision=B.SIC_SPLIT_U32, l_max=dx, max_tracers=200_000) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
        n = s.n
    assert np.all(h["total_charge"] == h["total_charge"][0])
    err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
    print(f"refinement split U32 envelope error {err:.3e}, count {n} vs oracle {ref['count'][-1]}", flush=True)
    assert err < 1e-6
    assert abs(n - ref["count"][-1]) <= 0.01 * ref["count"][-1]


def test_refinement_beyond_capacity_is_refused_and_state_kept():
    p = I.refinement_two_stream(n_steps=10)
    dx = p.L / p.n_cells
    with B.Simulation(p, l_max=0.0, seg_charges=p.seg_charges, max_tracers=p.total_tracers + 10) as s:
        x0, v0, _ = s.state()
        with pytest.raises(B.SicError) as e:
            s.refine(0.01 * dx)  # would split every segment
        assert e.value.status == 2
        x1, v1, _ = s.state()
        assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
        assert s.refine(10 * dx) == 0
        s.step(3)


def test_load_state_round_trip_and_uniform_simulation_rejects_charges():
    p = I.landau_vertical(n_streams=10, n_positions=64, n_cells=32, n_steps=5)
    with B.Simulation(p) as s:
        s.step(5)
        x, v, step = s.state()
        c = s.charges()
        nt, _ = s.layout()
        W = s.diagnostics(history=False)["last"]["W_E"]
        s.load_state(step, nt, x, v, c)
        x2, v2, step2 = s.state()
        assert step2 == step and np.array_equal(x2, x) and np.array_equal(v2, v)
        s.step(0)  # brings the stale field up to date
        assert abs(s.diagnostics(history=False)["last"]["W_E"] - W) <= 1e-13 * W
    u = I.landau(n_sheets=4, n_tracers=64, n_cells=32, n_steps=3)
    with B.Simulation(u) as s:
        x, v, step = s.state()
        with pytest.raises(B.SicError) as e:
            s.load_state(step, u.n_tracers, x, v, u.seg_charges)
        assert e.value.status == 6
        with pytest.raises(B.SicError) as e:
            s.refine(0.1)
        assert e.value.status == 6


def test_batch_with_segment_charges_matches_alone():
    prec = B.SIC_SPLIT_U32
    probs = [I.landau_vertical(n_streams=26, n_positions=160, n_cells=40, n_steps=17),
             I.landau_vertical(n_streams=12, n_positions=100, n_cells=64, n_steps=23, alpha=0.2),
             I.landau(n_sheets=8, n_tracers=130, n_cells=64, n_steps=19, alpha=0.1)]
    # short vertical sheets leave most of each 64-tracer chunk empty: budget
    # the padded slots
    slots_needed = sum(int(np.sum((p.n_tracers + 63) // 64)) * 64 for p in probs)
    b = B.sic_batch_create(slots_needed, 4, 64, precision=prec, flags=B.SIC_BATCH_SEGMENT_CHARGES)
    try:
        slots = [B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, p.n_steps,
                                   precision=prec, seg_charges=p.c_full) for p in probs]
        B.sic_batch_step(b, 30)
        assert sorted(B.sic_batch_poll(b)) == sorted(slots)
        for p, sl in zip(probs, slots):
            with B.Simulation(p, precision=prec, seg_charges=p.seg_charges) as s:
                s.step(p.n_steps)
                x, v, _ = s.state()
                W = s.diagnostics()["history"]["W_E"]
            xb, vb, st = B.sic_batch_get_state(b, sl, p.total_tracers)
            assert st == p.n_steps
            assert np.array_equal(x, xb) and np.array_equal(v, vb)
            assert np.array_equal(W, B.sic_batch_result(b, sl)["history"]["W_E"])
            cb = B.sic_batch_get_charges(b, sl, p.total_tracers)
            assert np.max(np.abs(cb - p.seg_charges)) <= 1e-15 * np.max(p.seg_charges)  # fixed-point rounding
    finally:
        B.sic_batch_destroy(b)
    plain = B.sic_batch_create(1000, 1, 64)
    try:
        p = probs[0]
        with pytest.raises(B.SicError) as e:
            B.sic_batch_admit(plain, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, 3,
                              seg_charges=p.c_full)
        assert e.value.status == 6
    finally:
        B.sic_batch_destroy(plain)


def test_batch_refinement_matches_alone_bitwise():
    """Refining simulations in a batch (each growing inside its own
    reservation) beside non-refining ones: every instance ends bitwise equal
    to the same simulation run alone (split U32 form)."""
    prec = B.SIC_SPLIT_U32
    ts = I.refinement_two_stream(n_steps=330)
    dx = ts.L / ts.n_cells
    specs = [(ts, dx, 60_000), (I.refinement_two_stream(n_steps=300, ppc=8), 0.5 * dx, 80_000),
             (I.landau(n_sheets=8, n_tracers=130, n_cells=64, n_steps=250, alpha=0.1), 0.0, 0),
             (I.landau_vertical(n_streams=20, n_positions=90, n_cells=40, n_steps=200), 0.0, 0)]
    budget = sum(max(mt, int(np.sum((p.n_tracers + 63) // 64)) * 64) + 64 * len(p.n_tracers) for p, _, mt in specs)
    b = B.sic_batch_create(budget, 8, 128, precision=prec, flags=B.SIC_BATCH_SEGMENT_CHARGES)
    try:
        slots = [B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, p.n_steps,
                                   precision=prec, seg_charges=p.c_full, l_max=lm, max_tracers=mt)
                 for p, lm, mt in specs]
        B.sic_batch_step(b, 340)
        assert sorted(B.sic_batch_poll(b)) == sorted(slots)
        for (p, lm, mt), sl in zip(specs, slots):
            nt_b, tot_b = B.sic_batch_get_layout(b, sl, len(p.n_tracers))
            # alone with per-segment charges too, so both hold the same
            # fixed-point charge words
            with B.Simulation(p, precision=prec, l_max=lm, max_tracers=mt, seg_charges=p.seg_charges) as s:
                s.step(p.n_steps)
                nt_a, tot_a = s.layout()
                x, v, _ = s.state()
                W = s.diagnostics()["history"]["W_E"]
                c = s.charges()
            print(f"slot {sl}: {tot_b} tracers in the batch, {tot_a} alone", flush=True)
            assert np.array_equal(nt_a, nt_b) and tot_a == tot_b
            if lm:
                assert tot_a > p.total_tracers  # it refined
            xb, vb, st = B.sic_batch_get_state(b, sl, tot_b)
            assert st == p.n_steps
            assert np.array_equal(x, xb) and np.array_equal(v, vb)
            assert np.array_equal(W, B.sic_batch_result(b, sl)["history"]["W_E"])
            assert np.array_equal(c, B.sic_batch_get_charges(b, sl, tot_b))
        used, _ = B.sic_batch_usage(b)
        assert used == sum(max(mt, p.total_tracers) for p, _, mt in specs)
        for sl in slots:
            B.sic_batch_release(b, sl)
        assert B.sic_batch_usage(b) == (0, 0)
    finally:
        B.sic_batch_destroy(b)


def test_batch_refinement_fp64_follows_oracle():
    p = I.refinement_two_stream(n_steps=330)
    dx = p.L / p.n_cells
    ref = O.run_seg(p.L, p.n_cells, p.dt, p.n_tracers, p.closed, p.seg_charges, p.x0, p.v0, p.n_steps, l_max=dx,
                    capacity=100_000)
    other = I.landau(n_sheets=16, n_tracers=256, n_cells=128, n_steps=400, alpha=0.05)
    b = B.sic_batch_create(200_000, 4, 128, flags=B.SIC_BATCH_SEGMENT_CHARGES)
    try:
        s1 = B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, p.n_steps,
                               l_max=dx, max_tracers=100_000)
        s2 = B.sic_batch_admit(b, other.L, other.n_cells, other.dt, other.n_tracers, other.q, other.closed,
                               other.x0, other.v0, other.n_steps)
        B.sic_batch_step(b, 100)
        B.sic_batch_step(b, 300)
        nt, tot = B.sic_batch_get_layout(b, s1, len(p.n_tracers))
        h = B.sic_batch_result(b, s1)["history"]
        assert tot == ref["count"][-1] > ref["count"][0]
        assert np.array_equal(nt, ref["n_tracers"])
        err = envelope_rel(h["W_E"], ref["hist"][:, 2], p.dt)
        print(f"batch refinement fp64: {tot} tracers, envelope error {err:.3e}", flush=True)
        assert err < 1e-10
        ro = O.run_problem(other)
        ho = B.sic_batch_result(b, s2)["history"]
        assert envelope_rel(ho["W_E"], ro["hist"][:, 2], other.dt) < 1e-10
    finally:
        B.sic_batch_destroy(b)


def test_batch_refinement_needs_segment_charges_and_budget():
    p = I.refinement_two_stream(n_steps=10)
    plain = B.sic_batch_create(100_000, 2, 128)
    try:
        with pytest.raises(B.SicError) as e:
            B.sic_batch_admit(plain, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, 10, l_max=0.1)
        assert e.value.status == 6
    finally:
        B.sic_batch_destroy(plain)
    b = B.sic_batch_create(50_000, 4, 128, flags=B.SIC_BATCH_SEGMENT_CHARGES)
    try:
        B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, 10, l_max=0.1,
                          max_tracers=40_000)
        assert B.sic_batch_usage(b) == (40_000, 1)
        # the reservation counts: a second one does not fit the budget
        assert B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, 10, l_max=0.1,
                                 max_tracers=40_000, raise_busy=False) is None
    finally:
        B.sic_batch_destroy(b)
