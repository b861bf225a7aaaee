"""Diagnostics flags on the GPU against the oracle's flags column.

The library's flags are sticky (a bit once set stays set for the rest of the
simulation), the oracle's are per row, so the GPU history is compared with
the running OR of the oracle's rows.  LONG_SEGMENT warns that a segment has
stretched beyond 0.45 L, close to the half box where the shorter way round
changes side (the periodic closure of section 2.3, sheets stretching to box
size in sections 2.6 and 3.2); NONFINITE reports a non-finite field,
segment length or move."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I

pytestmark = pytest.mark.gpu
PRECS = [B.SIC_FP64, B.SIC_SPLIT_U32, B.SIC_SPLIT_F32]


def _sticky(col):
    return np.bitwise_or.accumulate(np.asarray(col).astype(np.int64))


def _stretching(n_background_sheets):
    """A uniform cold background plus one open two-tracer sheet whose ends
    move apart at 0.52 each: its segment (0.3 L at first, L = 1) passes
    0.45 L between steps 14 and 15 (dt 0.01), far from a step boundary."""
    nb, ntb = n_background_sheets, 64
    L, nc = 1.0, 32
    xb = np.tile(np.arange(ntb) * (L / ntb) + 0.25 / ntb, nb)
    x = np.concatenate([xb, [0.35, 0.65]])
    v = np.concatenate([np.zeros(nb * ntb), [-0.52, 0.52]])
    nt = np.array([ntb] * nb + [2], np.int32)
    q = np.array([L / (ntb * nb)] * nb + [1e-4])
    closed = np.array([1] * nb + [0], np.int32)
    return I.Problem(name="stretching", L=L, n_cells=nc, dt=0.01, n_steps=40, n_tracers=nt, q=q, closed=closed,
                     x_full=x, v_full=v)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_bg", [2, 40], ids=["resident", "graphs"])
def test_long_segment_flag_matches_oracle(prec, n_bg):
    p = _stretching(n_bg)
    print(f"case long segment prec={prec} background sheets={n_bg}", flush=True)
    ref = O.run_problem(p)
    with B.Simulation(p, precision=prec) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
    fo = _sticky(ref["hist"][:, 7])
    assert fo[0] == 0 and fo[-1] == 2 and np.argmax(fo == 2) == 15
    assert np.array_equal(h["flags"].astype(np.int64), fo)
    tol = 1e-12 if prec == B.SIC_FP64 else 1e-9
    assert np.max(np.abs(h["max_segment"] - ref["hist"][:, 6])) < tol * p.L


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(4, 32), (40, 64)], ids=["resident", "graphs"])
def test_nonfinite_velocity_flag_matches_oracle(prec, shape):
    """One tracer's velocity is NaN (passed in device memory, which the
    library does not scan).  From the first move on, every row has the
    NONFINITE bit on both sides.  In float64 the tracer's position becomes
    NaN and its two segments deposit nothing, on both sides, so the field
    energy still matches; a split position has no NaN and keeps its place."""
    import torch

    m, nt = shape
    p = I.landau(n_sheets=m, n_tracers=nt, n_cells=16, n_steps=5)
    v0 = np.array(p.v0)
    v0[5] = np.nan
    print(f"case nonfinite velocity prec={prec} sheets={m} tracers={nt}", flush=True)
    ref = O.run(p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, p.x0, v0, p.n_steps)
    x0_d = torch.from_numpy(np.array(p.x0)).cuda()
    v0_d = torch.from_numpy(v0).cuda()
    with B.Simulation(p, precision=prec, x0=x0_d, v0=v0_d) as s:
        s.step(p.n_steps)
        h = s.diagnostics()["history"]
        x, v, _ = s.state()
    fo = _sticky(ref["hist"][:, 7])
    assert fo[0] == 0 and np.all(fo[1:] == 1)
    assert np.array_equal(h["flags"].astype(np.int64), fo)
    assert np.isnan(v[5]) and np.sum(np.isnan(v)) == 1
    if prec == B.SIC_FP64:
        assert np.isnan(x[5]) and np.sum(np.isnan(x)) == 1
        Wr = ref["hist"][:, 2]
        assert np.max(np.abs(h["W_E"] - Wr) / np.max(Wr)) < 1e-10
        assert np.allclose(h["total_charge"], ref["hist"][:, 5], rtol=1e-12, atol=0)
    else:
        assert np.all(np.isfinite(x))
        assert abs(x[5] - O.wrap(p.x0[5], p.L)) < 2.0 ** -30 * p.L / p.n_cells
