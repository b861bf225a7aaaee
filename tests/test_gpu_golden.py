"""The HIP path against the values the paper prints (the fixtures under
``tests/golden/``), measured on its own runs: the two-stream growth rate of
section 3.2 on the section 2.6 set-up, and the section 3.3 convergence slopes
of the potential-energy error for constant and linear segments."""

import numpy as np
import pytest

from paper_1506_07207_amd import binding as B
from paper_1506_07207_amd import inputs as I
from tests.test_oracle_golden import CV, TS, WB, growth_fit

pytestmark = pytest.mark.gpu


def _hist(p, order=0, steps=None):
    steps = p.n_steps if steps is None else steps
    with B.Simulation(p, deposit_order=order) as s:
        s.step(steps)
        h = s.diagnostics()["history"]
    assert h["step"][-1] == steps
    return np.stack([h["step"].astype(np.float64), h["t"], h["W_E"]], axis=1)


def test_section_2_6_set_up_grows_at_half_the_beam_frequency():
    p = I.refinement_two_stream(n_steps=250)
    print("case two-stream section 2.6 set-up, 250 steps", flush=True)
    h = _hist(p)
    assert h[h[:, 1] <= 19.0, 2].max() < 0.05 * h[:, 2].max()
    gamma = growth_fit(h, 12.0, 19.0)
    assert abs(gamma / (TS["max_growth_over_wb"] * WB) - 1.0) < 0.03, gamma


def test_potential_energy_error_falls_at_twice_the_order():
    Ns = np.array([16, 32, 64])
    for order, key, tol in ((0, "epot_slope_constant", 0.15), (1, "epot_slope_linear", 0.25)):
        print(f"case convergence slopes order={order}", flush=True)
        gold = _hist(I.convergence_landau(4096, 128), order)[:, 2]
        errs = [np.mean(np.abs(_hist(I.convergence_landau(int(N), 128), order)[:, 2] - gold)) for N in Ns]
        slopes = np.diff(np.log(errs)) / np.diff(np.log(Ns))
        print(f"  slopes {slopes}", flush=True)
        assert np.all(np.abs(slopes - CV[key]) < tol), (order, slopes)
