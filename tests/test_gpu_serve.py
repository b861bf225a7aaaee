"""Serving on the GPU: requests admitted while others run, each result equal
to the same simulation run alone and to the oracle's run of it."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from paper_1506_07207_amd import serve as S
from tests.parity import envelope_rel

pytestmark = pytest.mark.gpu


def _small_stream(n, rate, seed):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        spec = I.BatchSpec("landau" if i % 2 else "two_stream", float(rng.uniform(0.2, 0.6)),
                           float(np.exp(rng.uniform(np.log(1e-3), np.log(0.5)))), 2 * int(rng.integers(4, 17)),
                           int(rng.integers(64, 400)), int(2 ** rng.integers(6, 11)), float(rng.uniform(0.05, 0.1)),
                           int(rng.integers(20, 120)))
        out.append(I.Request(i, t, spec, False))
    return out


@pytest.mark.parametrize("prec", [B.SIC_FP64, B.SIC_SPLIT_U32])
def test_served_results_equal_alone(prec):
    reqs = _small_stream(40, rate=400.0, seed=prec + 1)
    classes = (S.SizeClass(256, 60_000, 12), S.SizeClass(1024, 200_000, 8))
    ex = S.GpuExecutor(classes=classes, precision=prec, history_rows=256, keep_history=True)
    try:
        rep = S.Server(ex, chunk_steps=16).run(reqs, prepare=S.serve_prepare(ex))
    finally:
        ex.close()
    assert len(rep.completed()) == len(reqs)
    overlapped = sum(1 for a in rep.records for b in rep.records
                     if a.rid < b.rid and b.admitted < a.completed)
    assert overlapped > 0, "no request was admitted while another was running"
    tol = 1e-10 if prec == B.SIC_FP64 else 1e-6
    for r, req in zip(rep.records, reqs):
        p = req.spec.build()
        with B.Simulation(p, precision=prec) as s:
            s.step(p.n_steps)
            W = s.diagnostics(history=False)["last"]["W_E"]
        if prec == B.SIC_FP64:
            assert abs(r.final_W_E - W) <= 1e-10 * W
        else:
            assert r.final_W_E == W
        # the served history against the oracle
        ref = O.run_problem(p)["hist"][:, 2]
        assert r.W_E_history is not None and len(r.W_E_history) == p.n_steps + 1
        err = envelope_rel(r.W_E_history, ref, p.dt)
        assert err < tol, (r.rid, err)
    q = rep.latency_quantiles()
    assert 0 < q[0.5] <= q[0.99]
