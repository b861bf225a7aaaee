"""The no-allocation variant of sic_set_state against sic_set_state itself,
through the C ABI: two calls in a row (a larger simulation, then a smaller
one), host and device inputs, and the size limit."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I

pytestmark = pytest.mark.gpu


def _state_after(p, prec, step, x, v, noalloc, device=False):
    import torch

    with B.Simulation(p, precision=prec) as s:
        if device:
            x, v = torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda()
        (B.sic_set_state_noalloc if noalloc else B.sic_set_state)(s.h, step, x, v)
        xs, vs, st = s.state()
        s.step(5)
        x5, v5, st5 = s.state()
        d = s.diagnostics()
    return xs, vs, st, x5, v5, st5, d


@pytest.mark.parametrize("prec", [B.SIC_SPLIT_U32, B.SIC_FP64])
def test_set_state_noalloc_matches_set_state(prec):
    # two calls in a row: 256 x 1024 tracers, then 8 x 200
    for p in (I.landau(n_sheets=256, n_tracers=1024, n_cells=256, n_steps=30),
              I.landau(n_sheets=8, n_tracers=200, n_cells=64, n_steps=30, alpha=0.05)):
        ref = O.run_problem(p, 30)
        x, v = ref["x"], ref["v"]
        print(f"case noalloc set_state prec={prec} tracers={p.total_tracers}", flush=True)
        a = _state_after(p, prec, 30, x, v, noalloc=True)
        b = _state_after(p, prec, 30, x, v, noalloc=False)
        assert a[2] == b[2] == 30 and a[5] == b[5] == 35
        # the history starts at the step the state was set at
        for r in (a, b):
            assert list(r[6]["history"]["step"]) == list(range(30, 36))
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        if prec == B.SIC_FP64:
            # float64 atomics may add in another order over the five steps
            assert np.max(np.abs(a[3] - b[3])) < 1e-12 * p.L
            assert np.allclose(a[6]["history"]["W_E"], b[6]["history"]["W_E"], rtol=1e-12, atol=0)
        else:
            assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])
            assert np.array_equal(a[6]["history"]["W_E"], b[6]["history"]["W_E"])
        # device inputs bypass the staging array
        c = _state_after(p, prec, 30, x, v, noalloc=True, device=True)
        assert np.array_equal(c[0], b[0]) and np.array_equal(c[1], b[1])


def test_set_state_noalloc_rejects_oversize_host_inputs():
    n = B.SIC_NOALLOC_MAX_TRACERS + 64
    p = I.landau(n_sheets=n // 64, n_tracers=64, n_cells=64, n_steps=1)
    with B.Simulation(p) as s:
        x0, v0, _ = s.state()
        with pytest.raises(B.SicError):
            B.sic_set_state_noalloc(s.h, 3, x0, v0)
        # nothing changed
        x1, v1, st = s.state()
        assert st == 0 and np.array_equal(x0, x1) and np.array_equal(v0, v1)
