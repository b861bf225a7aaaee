"""Batched execution: many independent simulations resident on the GPU,
advanced in shared launches, admitted and released while others run.
Every instance must give the result it gives alone (FP64: to rounding of
the atomic deposit order; split forms: bitwise)."""
import numpy as np
import pytest

from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import envelope_rel, periodic_diff

pytestmark = pytest.mark.gpu


def _mix():
    return [
        I.landau(n_sheets=16, n_tracers=200, n_cells=64, n_steps=37, alpha=0.05),
        I.two_stream(n_sheets=8, n_tracers=1000, n_cells=256, n_steps=80, alpha=0.01),
        I.cold_oscillation(n_tracers=130, n_cells=32, n_steps=55),
        I.random_sheets(5, 5, [64, 65, 2, 127, 400], 100, L=3.0, dt=0.03, n_steps=23, jitter=0.3),
        I.landau(k=0.3, n_sheets=4, n_tracers=64, n_cells=1024, n_steps=61, alpha=0.2),
    ]


def _alone(p, prec):
    with B.Simulation(p, precision=prec) as s:
        s.step(p.n_steps)
        x, v, step = s.state()
        d = s.diagnostics()
    return x, v, d


def _admit(b, p, prec, raise_busy=True):
    return B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, p.v0, p.n_steps,
                             precision=prec, raise_busy=raise_busy)


@pytest.mark.parametrize("prec", [B.SIC_FP64, B.SIC_SPLIT_F32, B.SIC_SPLIT_U32])
def test_batch_matches_alone(prec):
    probs = _mix()
    total = sum(p.total_tracers for p in probs)
    b = B.sic_batch_create(total + 1000, 8, 1024, precision=prec)
    try:
        slots = [_admit(b, p, prec) for p in probs]
        done = []
        for _ in range(20):
            B.sic_batch_step(b, 7)
            done += B.sic_batch_poll(b)
            if len(done) == len(probs):
                break
        assert sorted(done) == sorted(slots)
        for p, s in zip(probs, slots):
            x, v, d = _alone(p, prec)
            xb, vb, step = B.sic_batch_get_state(b, s, p.total_tracers)
            db = B.sic_batch_result(b, s, p.n_cells)
            assert step == p.n_steps and len(db["history"]) == p.n_steps + 1
            if prec == B.SIC_FP64:
                assert np.max(periodic_diff(xb, x, p.L)) < 1e-11 * p.L
                assert envelope_rel(db["history"]["W_E"], d["history"]["W_E"], p.dt) < 1e-11
            else:
                assert np.array_equal(xb, x) and np.array_equal(vb, v)
                assert np.array_equal(db["history"]["W_E"], d["history"]["W_E"])
                assert np.array_equal(db["rho"], d["rho"]) and np.array_equal(db["E"], d["E"])
    finally:
        B.sic_batch_destroy(b)


def test_continuous_admission_and_release():
    prec = B.SIC_SPLIT_U32
    probs = _mix()
    budget = probs[1].total_tracers + probs[0].total_tracers + 500
    b = B.sic_batch_create(budget, 2, 1024, precision=prec)
    try:
        pending = list(range(len(probs)))
        slot_of = {}
        finished = {}
        guard = 0
        while pending or slot_of:
            guard += 1
            assert guard < 200
            while pending:
                s = _admit(b, probs[pending[0]], prec, raise_busy=False)
                if s is None:
                    break
                slot_of[s] = pending.pop(0)
            assert slot_of, "a request that fits alone must be admitted into an empty batch"
            B.sic_batch_step(b, 5)
            for s in B.sic_batch_poll(b):
                i = slot_of.pop(s)
                p = probs[i]
                finished[i] = (B.sic_batch_get_state(b, s, p.total_tracers), B.sic_batch_result(b, s, p.n_cells))
                B.sic_batch_release(b, s)
        assert B.sic_batch_usage(b) == (0, 0)
        for i, p in enumerate(probs):
            (xb, vb, step), db = finished[i]
            x, v, d = _alone(p, prec)
            assert step == p.n_steps
            assert np.array_equal(xb, x) and np.array_equal(vb, v)
            assert np.array_equal(db["history"]["W_E"], d["history"]["W_E"])
    finally:
        B.sic_batch_destroy(b)


def test_admission_refusals():
    p = I.landau(n_sheets=4, n_tracers=100, n_cells=32, n_steps=10)
    b = B.sic_batch_create(p.total_tracers * 2, 3, 64)
    try:
        s0 = _admit(b, p, B.SIC_FP64)
        s1 = _admit(b, p, B.SIC_FP64)
        assert _admit(b, p, B.SIC_FP64, raise_busy=False) is None  # over the tracer budget
        big = I.landau(n_sheets=4, n_tracers=100, n_cells=128, n_steps=10)
        with pytest.raises(B.SicError) as e:
            _admit(b, big, B.SIC_FP64)  # more cells than the batch holds
        assert e.value.status == 1
        with pytest.raises(B.SicError) as e:
            _admit(b, p, B.SIC_SPLIT_U32)  # precision differs from the batch
        assert e.value.status == 1
        B.sic_batch_release(b, s0)
        s2 = _admit(b, p, B.SIC_FP64)
        assert s2 == s0
        assert B.sic_batch_usage(b) == (2 * p.total_tracers, 2)
        with pytest.raises(B.SicError):
            B.sic_batch_release(b, 2)  # not live
    finally:
        B.sic_batch_destroy(b)


def test_sparse_live_slots_after_release():
    """The whole-batch solve launches one workgroup per slot index up to the
    highest live one: with slots 1..5 released, slots 0 and 6 (and a slot
    admitted afterwards into the freed range) must still get their solves,
    bitwise as alone (split form)."""
    prec = B.SIC_SPLIT_U32
    probs = [I.random_sheets(40 + i, 3, [70, 64, 130], 64, L=2.0, dt=0.05, n_steps=30, jitter=0.3)
             for i in range(7)]
    late = I.landau(n_sheets=8, n_tracers=128, n_cells=64, n_steps=30, alpha=0.05)
    total = sum(p.total_tracers for p in probs) + late.total_tracers
    b = B.sic_batch_create(total + 1000, 8, 64, precision=prec)
    try:
        slots = [_admit(b, p, prec) for p in probs]
        assert slots == list(range(7))
        B.sic_batch_step(b, 4)
        for s in slots[1:6]:
            B.sic_batch_release(b, s)
        s_late = _admit(b, late, prec)
        assert s_late == 1  # lowest free slot
        B.sic_batch_step(b, 40)
        done = B.sic_batch_poll(b)
        assert sorted(done) == [0, 1, 6]
        for p, s in ((probs[0], 0), (probs[6], 6), (late, s_late)):
            x, v, _ = _alone(p, prec)
            xb, vb, step = B.sic_batch_get_state(b, s, p.total_tracers)
            assert step == p.n_steps
            assert np.array_equal(xb, x) and np.array_equal(vb, v)
    finally:
        B.sic_batch_destroy(b)
