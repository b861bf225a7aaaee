"""The deposit-only kernel against the oracle's exact overlap deposit.

A deposit that does not move the tracers uses the face-crossing form of the
constant-segment deposit (section 2.3): per tracer only its cell and the
segment length are computed, and the segments whose two ends lie in
different cells are queued per wavefront and processed 64 at a time.  The
sheets here are built to stress that path: tracers exactly on cell faces
(the W_0 tie rule decides the cell) and one ulp either side of them,
repeated tracers (zero-length segments on faces), a dense sheet with thousands of
tracers per cell (few crossings, long stretches between queue drains), a
sparse sheet whose segments cross many faces in both directions and across
the periodic boundary (covered-cell runs, a full queue every chunk), and
random walks on one and two cells.  FP64 is held to 1e-10 of the density
scale; the split forms deposit int64 fixed point, so their mesh must not
depend on how the sheets are cut into work items and workgroups.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd.inputs import Problem
from tests.parity import rel_inf

pytestmark = pytest.mark.gpu
TOL = 1e-10
# (chunks per work item, threads per workgroup, workgroups)
SHAPES = [(4, 64, 7), (256, 1024, 3), (16, 256, 100), (64, 512, 1)]


def _problem(name, L, nc, sheets, closed, q, c=None):
    n = np.array([len(s) for s in sheets], dtype=np.int32)
    x = np.concatenate(sheets).astype(np.float64)
    return Problem(name=name, L=L, n_cells=nc, dt=0.1, n_steps=1, n_tracers=n, q=np.asarray(q, np.float64),
                   closed=np.asarray(closed, np.int32), x_full=x, v_full=np.zeros_like(x), c_full=c)


def _cases():
    rng = np.random.default_rng(5)
    L = 3.7
    out = []
    nc = 64
    dx = L / nc
    faces = np.arange(nc) * dx
    on = np.repeat(faces, 3)
    near = np.sort(np.concatenate([np.nextafter(faces[1:], 0.0), faces[1:], np.nextafter(faces[1:], L)]))
    out.append(_problem("faces", L, nc, [on, faces[::-1].copy()], [1, 0], [0.01, 0.03]))
    out.append(_problem("near", L, nc, [near, on], [1, 1], [-0.02, 0.01]))
    dense = np.sort(rng.uniform(0.0, L, 200_000))
    out.append(_problem("dense", L, 16, [dense], [1], [1e-5]))
    nc = 4096
    dx = L / nc
    steps = rng.uniform(3.0, 11.0, 500) * dx * rng.choice([-1.0, 1.0], 500)
    sp = np.mod(np.cumsum(steps), L)
    out.append(_problem("sparse", L, nc, [sp, sp[:130].copy(), np.array([0.1 * L, 0.9 * L])], [1, 0, 0],
                        [0.3, 0.2, 1.0]))
    for nc in (1, 2):
        size = np.exp(rng.uniform(-14.0, np.log(0.4 * L), 3000))
        w = np.mod(np.cumsum(rng.standard_normal(3000) * size), L)
        out.append(_problem(f"walk{nc}", L, nc, [w, w[:65].copy()], [1, 0], [0.5, -0.25]))
    return out


CASES = _cases()


def _oracle(p, c=None):
    Q, ms = O.deposit(p.L, p.n_cells, p.n_tracers, p.q, p.closed, p.x0, c=c)
    dx = p.L / p.n_cells
    return Q / dx - Q.sum() / p.L, Q, ms


def _rho_after(s, shape):
    B.sic_set_tuning(s.h, *shape)
    s.deposit()
    s.solve()
    return s.diagnostics(history=False)


EXACT = [p for p in CASES if p.name != "near"]


@pytest.mark.parametrize("p", EXACT, ids=[p.name for p in EXACT])
def test_fp64_deposit_matches_oracle_at_every_launch_shape(p):
    print(f"case {p.name} nc={p.n_cells} tracers={p.total_tracers}", flush=True)
    rho_o, Q, ms = _oracle(p)
    scale = max(1.0, np.max(np.abs(rho_o + Q.sum() / p.L)))
    n_seg = np.where(p.closed != 0, p.n_tracers, p.n_tracers - 1)
    exact = float(np.sum(p.q * n_seg))
    with B.Simulation(p) as s:
        for shape in [None] + SHAPES:
            d = s.diagnostics(history=False) if shape is None else _rho_after(s, shape)
            assert rel_inf(d["rho"], rho_o, scale=scale) < TOL, shape
            assert abs(d["last"]["total_charge"] - exact) <= 1e-12 * np.sum(np.abs(p.q * n_seg)), shape
            assert abs(d["last"]["max_segment"] - ms) <= 1e-13 * p.L, shape


def test_fp64_segments_shorter_than_rounding_at_a_face():
    """Tracers one ulp either side of a face: which cell receives the charge
    of a segment shorter than the rounding of its ends' mesh coordinates is
    decided by that rounding (here the oracle's faces at j * dx and the GPU's
    x * (nc / L) differ by an ulp), so the two may place such a segment's
    charge on opposite sides of the face.  Everything else must agree: the
    totals, and the cells up to the charge of those segments."""
    p = next(c for c in CASES if c.name == "near")
    rho_o, Q_o, ms = _oracle(p)
    dx = p.L / p.n_cells
    x = np.split(p.x0, np.cumsum(p.n_tracers)[:-1])
    short = 0.0
    for xs, q in zip(x, p.q):
        d = np.abs(np.roll(xs, -1) - xs)
        d = np.minimum(d, p.L - d)
        short += abs(q) * np.count_nonzero(d < 1e-9 * dx)
    with B.Simulation(p) as s:
        for shape in [None] + SHAPES:
            d = s.diagnostics(history=False) if shape is None else _rho_after(s, shape)
            total = d["last"]["total_charge"]
            Q = (d["rho"] + total / p.L) * dx
            assert abs(total - Q_o.sum()) <= 1e-12 * np.sum(np.abs(p.q) * p.n_tracers), shape
            assert np.sum(np.abs(Q - Q_o)) <= 2.0 * short + 1e-12, shape
            assert abs(d["last"]["max_segment"] - ms) <= 1e-13 * p.L, shape


@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_SPLIT_F32])
@pytest.mark.parametrize("p", CASES, ids=[p.name for p in CASES])
def test_split_deposit_independent_of_launch_shape(p, prec):
    print(f"case {p.name} prec={prec}", flush=True)
    with B.Simulation(p, precision=prec) as s:
        d0 = s.diagnostics(history=False)
        for shape in SHAPES:
            d = _rho_after(s, shape)
            assert np.array_equal(d["rho"], d0["rho"]), shape
            assert d["last"]["total_charge"] == d0["last"]["total_charge"], shape
        x_held, _, _ = s.state()
    if p.name not in ("faces", "near"):
        # the exact deposit of the positions the split form holds (on faces the
        # read-back position may round to the other side of the face)
        rho_h, _, _ = _oracle(dataclasses.replace(p, x_full=x_held))
        assert rel_inf(d0["rho"], rho_h, scale=max(1.0, np.max(np.abs(rho_h)))) < 1e-8


@pytest.mark.parametrize("prec", [B.SIC_FP64, B.SIC_SPLIT_U32])
def test_per_segment_charges_through_the_queue(prec):
    p0 = next(c for c in CASES if c.name == "sparse")  # many crossings per chunk
    rng = np.random.default_rng(11)
    c = rng.uniform(0.05, 1.0, p0.total_tracers)
    ends = np.cumsum(p0.n_tracers.astype(np.int64)) - 1
    c[ends[p0.closed == 0]] = 0.0
    p = _problem("sparse_c", p0.L, p0.n_cells, np.split(p0.x0, np.cumsum(p0.n_tracers)[:-1]), p0.closed, p0.q, c=c)
    rho_o, _, ms = _oracle(p, c=c)
    tol = TOL if prec == B.SIC_FP64 else 1e-6
    with B.Simulation(p, precision=prec) as s:
        d0 = s.diagnostics(history=False)
        assert rel_inf(d0["rho"], rho_o, scale=max(1.0, np.max(np.abs(rho_o)))) < tol
        assert abs(d0["last"]["max_segment"] - ms) <= (1e-13 if prec == B.SIC_FP64 else 1e-8) * p.L
        for shape in SHAPES:
            d = _rho_after(s, shape)
            if prec == B.SIC_FP64:
                assert rel_inf(d["rho"], rho_o, scale=max(1.0, np.max(np.abs(rho_o)))) < tol, shape
            else:
                assert np.array_equal(d["rho"], d0["rho"]), shape
