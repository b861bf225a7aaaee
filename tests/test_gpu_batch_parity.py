"""The 4096-instance mixed batch the benchmark times, against the oracle
instance by instance: every instance for its first 10 steps, and a sample
stratified by problem type, mesh size, amplitude and tracer count for 200
steps (past saturation for the large-amplitude two-stream instances), in
the benchmark's default launch shape."""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.parity import envelope, field_scale, rel_inf

pytestmark = pytest.mark.gpu
FIRST = 10
LONG = 200
SPECS = I.batch_mix(4096)


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


def _oracle(i, steps):
    """W_E history and final field of instance i (the oracle releases the
    interpreter lock, so threads run in parallel)."""
    p = SPECS[i].build()
    r = O.run_problem(p, steps)
    return r["hist"][:, 2].copy(), r["E"].copy()


def _stratified(limit=64):
    """Up to two instances per (type, mesh size, amplitude, size) bin, plus
    the largest instance."""
    bins = {}
    for i, s in enumerate(SPECS):
        key = (s.kind, 0 if s.n_cells <= 128 else (1 if s.n_cells <= 512 else 2),
               0 if s.alpha < 0.02 else (1 if s.alpha < 0.1 else 2), 0 if s.tracers < 200_000 else 1)
        bins.setdefault(key, []).append(i)
    pick = [i for key in sorted(bins) for i in bins[key][:2]]
    big = int(np.argmax([s.tracers for s in SPECS]))
    if big not in pick:
        pick.append(big)
    return pick[:limit]


@pytest.fixture(scope="module")
def oracle_first():
    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        return list(ex.map(lambda i: _oracle(i, FIRST), range(len(SPECS))))


@pytest.fixture(scope="module")
def oracle_long():
    idx = _stratified()
    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        return idx, list(ex.map(lambda i: _oracle(i, LONG), idx))


@pytest.mark.parametrize("prec,tol", [(B.SIC_FP64, 1e-10), (B.SIC_SPLIT_U32, 1e-6), (B.SIC_SPLIT_F32, 1e-6)])
def test_mixed_batch_every_instance_and_stratified_long(prec, tol, oracle_first, oracle_long):
    import torch

    total = sum(s.tracers for s in SPECS)
    print(f"case mixed batch, every instance, prec={prec}", flush=True)
    b = B.sic_batch_create(total, len(SPECS), 1024, precision=prec, history_rows=256)
    try:
        for s in SPECS:
            p = s.build()
            x0 = torch.from_numpy(p.line).cuda().repeat(p.n_sheets)
            v0 = torch.from_numpy(p.sheet_v).cuda().repeat_interleave(int(p.n_tracers[0]))
            B.sic_batch_admit(b, p.L, p.n_cells, p.dt, p.n_tracers, p.q, p.closed, x0, v0, p.n_steps, precision=prec)
        B.sic_batch_step(b, FIRST)
        worst_w = worst_e = 0.0
        for i, (W_o, E_o) in enumerate(oracle_first):
            r = B.sic_batch_result(b, i, SPECS[i].n_cells)
            h = r["history"]
            assert h["step"][-1] == FIRST, i
            ew = float(np.max(np.abs(h["W_E"] - W_o)) / np.max(W_o))
            ee = rel_inf(r["E"], E_o)
            worst_w, worst_e = max(worst_w, ew), max(worst_e, ee)
            assert ew < tol and ee < tol, (i, SPECS[i], ew, ee)
        print(f"  all {len(SPECS)} instances, {FIRST} steps: worst W_E {worst_w:.2e}, worst E {worst_e:.2e}",
              flush=True)
        B.sic_batch_step(b, LONG - FIRST)
        idx, refs = oracle_long
        for i, (W_o, E_o) in zip(idx, refs):
            s = SPECS[i]
            r = B.sic_batch_result(b, i, s.n_cells)
            h = r["history"]
            assert h["step"][-1] == LONG, i
            err = float(np.max(np.abs(h["W_E"] - W_o) / envelope(W_o, s.dt)))
            ee = rel_inf(r["E"], E_o, scale=field_scale(E_o, W_o, s.dt, s.build().L))
            print(f"  instance {i} {s.kind} k={s.k:.3f} alpha={s.alpha:.2e} {s.n_sheets}x{s.n_tracers} "
                  f"on {s.n_cells}: W_E {err:.2e}, E {ee:.2e}", flush=True)
            assert err < tol and ee < tol, (i, s, err, ee)
    finally:
        B.sic_batch_destroy(b)
