"""Seeded synthetic initial conditions for 1D1V simplex-in-cell runs.

This module builds inputs only: tracer positions and velocities, per-sheet
segment charges, mesh and time-step parameters.  It holds none of the step's
arithmetic (no deposit, field solve, gather or push), so both the FP64 CPU
oracle and the GPU library consume exactly the same arrays.

Units: plasma frequency 1, mean electron density 1, so a sheet set whose
weights sum to one carries total charge L on a box of length L.

Sheet model (paper section 3, cold-sheet start): a warm plasma is a set of
"horizontal" cold sheets, evenly spaced in velocity, each with a charge weight
proportional to the Maxwellian at its velocity (section 3.3).  Within a sheet
the tracers are evenly spaced in a Lagrangian coordinate q_t = t L / N_t and
mapped to positions so that the tracer density follows 1 + alpha cos(k x)
(the exact inverse of the cumulative density, solved by Newton iteration to
round-off).  All sheets of one instance share the same positions, as in the
paper's phase-space setup figure (section 3.3.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional

import numpy as np

__all__ = [
    "Problem",
    "lagrangian_grid",
    "density_positions",
    "maxwellian_sheets",
    "cold_oscillation",
    "landau",
    "two_stream",
    "cold_two_stream",
    "landau_vertical",
    "refinement_two_stream",
    "uniform_sheet",
    "random_sheets",
    "batch_mix",
    "BatchSpec",
    "request_stream",
]


@dataclasses.dataclass
class Problem:
    """One independent 1D1V instance.

    ``line`` holds the N_t tracer positions shared by every sheet and
    ``sheet_v`` the per-sheet velocity, so large instances stay compact until
    ``x0``/``v0`` are requested.  Non-uniform instances set ``x_full``/``v_full``.
    """

    name: str
    L: float
    n_cells: int
    dt: float
    n_steps: int
    n_tracers: np.ndarray  # int32 [M]
    q: np.ndarray  # float64 [M], charge carried by every segment of the sheet
    closed: np.ndarray  # int32 [M]
    line: Optional[np.ndarray] = None  # float64 [N_t] shared positions
    sheet_v: Optional[np.ndarray] = None  # float64 [M]
    x_full: Optional[np.ndarray] = None
    v_full: Optional[np.ndarray] = None
    c_full: Optional[np.ndarray] = None  # float64 [T] per-segment charges (replace q)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_sheets(self) -> int:
        return int(len(self.n_tracers))

    @property
    def total_tracers(self) -> int:
        return int(np.sum(self.n_tracers, dtype=np.int64))

    @property
    def x0(self) -> np.ndarray:
        if self.x_full is not None:
            return self.x_full
        return np.tile(self.line, self.n_sheets)

    @property
    def v0(self) -> np.ndarray:
        if self.v_full is not None:
            return self.v_full
        return np.repeat(self.sheet_v, self.n_tracers)

    @property
    def uniform(self) -> bool:
        return self.x_full is None

    @property
    def seg_charges(self) -> np.ndarray:
        """Charge of every segment, indexed by the tracer it starts at (the
        last tracer of an open sheet starts none: 0)."""
        if self.c_full is not None:
            return self.c_full
        c = np.repeat(self.q, self.n_tracers)
        ends = np.cumsum(self.n_tracers.astype(np.int64)) - 1
        c[ends[self.closed == 0]] = 0.0
        return c


def lagrangian_grid(n: int, L: float) -> np.ndarray:
    """Evenly spaced Lagrangian coordinates q_t = t L / n, t = 0..n-1."""
    return np.arange(n, dtype=np.float64) * (L / n)


def density_positions(n: int, L: float, k: float, alpha: float) -> np.ndarray:
    """Positions whose tracer density is proportional to 1 + alpha cos(k x).

    Solves x + (alpha/k) sin(k x) = q_t for every Lagrangian coordinate by
    Newton iteration (the cumulative density is monotone for alpha < 1).
    """
    if not (0.0 <= alpha < 1.0):
        raise ValueError("alpha must lie in [0, 1)")
    q = lagrangian_grid(n, L)
    if alpha == 0.0:
        return q
    x = q.copy()
    for _ in range(60):
        f = x + (alpha / k) * np.sin(k * x) - q
        fp = 1.0 + alpha * np.cos(k * x)
        step = f / fp
        x_new = x - step
        if np.all(np.abs(x_new - x) <= 2.0 * np.spacing(np.maximum(np.abs(x), L))):
            x = x_new
            break
        x = x_new
    # positions stay in [0, L): F(0) = 0 and F(L) = L
    x = np.where(x < 0.0, 0.0, x)
    return x


def maxwellian_sheets(m: int, vth: float = 1.0, vmax_units: float = 6.0, drift: float = 0.0,
                      weight: float = 1.0):
    """M sheet velocities at the midpoints of [-vmax, vmax] (in units of vth)
    around ``drift``, with weights proportional to the Maxwellian, normalised
    to sum to ``weight``."""
    u = -vmax_units + (np.arange(m, dtype=np.float64) + 0.5) * (2.0 * vmax_units / m)
    w = np.exp(-0.5 * u * u)
    w = weight * w / np.sum(w)
    return drift + vth * u, w


def _uniform_problem(name, L, n_cells, dt, n_steps, line, sheet_v, sheet_w, meta):
    m = len(sheet_v)
    nt = len(line)
    return Problem(
        name=name,
        L=float(L),
        n_cells=int(n_cells),
        dt=float(dt),
        n_steps=int(n_steps),
        n_tracers=np.full(m, nt, dtype=np.int32),
        q=np.asarray(sheet_w, dtype=np.float64) * (L / nt),
        closed=np.ones(m, dtype=np.int32),
        line=np.ascontiguousarray(line, dtype=np.float64),
        sheet_v=np.ascontiguousarray(sheet_v, dtype=np.float64),
        meta=dict(meta),
    )


def cold_oscillation(n_tracers: int = 1024, n_cells: int = 128, k: float = 0.5, alpha: float = 0.01,
                     dt: float = 0.1, n_steps: int = 200) -> Problem:
    """Cold plasma oscillation of a single sheet (paper section 3.1).

    The sheet is displaced in position, x = q + (alpha/k) sin(k q), and starts
    at rest; the box holds one wavelength, L = 2 pi / k.
    """
    L = 2.0 * math.pi / k
    q = lagrangian_grid(n_tracers, L)
    line = q + (alpha / k) * np.sin(k * q)
    return _uniform_problem("cold_oscillation", L, n_cells, dt, n_steps, line,
                            np.zeros(1), np.ones(1), dict(k=k, alpha=alpha))


def landau(k: float = 0.5, alpha: float = 0.01, n_sheets: int = 256, n_tracers: int = 512,
           n_cells: int = 256, dt: float = 0.1, n_steps: int = 1000, vth: float = 1.0,
           vmax_units: float = 6.0) -> Problem:
    """Warm Maxwellian plasma (v_th = 1) with a density perturbation
    1 + alpha cos(k x): linear Landau damping (paper section 3.3)."""
    L = 2.0 * math.pi / k
    line = density_positions(n_tracers, L, k, alpha)
    v, w = maxwellian_sheets(n_sheets, vth, vmax_units)
    return _uniform_problem("landau", L, n_cells, dt, n_steps, line, v, w,
                            dict(k=k, alpha=alpha, vth=vth))


def two_stream(k: float = 0.2, alpha: float = 0.001, n_sheets: int = 512, n_tracers: int = 4096,
               n_cells: int = 1024, dt: float = 0.05, n_steps: int = 2000, vb: float = 2.4,
               vth: float = 0.5, vmax_units: float = 6.0) -> Problem:
    """Two Maxwellian beams at +-vb (paper section 3.2), each with half of the
    charge, perturbed in density by 1 + alpha cos(k x)."""
    if n_sheets % 2:
        raise ValueError("two_stream needs an even sheet count")
    L = 2.0 * math.pi / k
    line = density_positions(n_tracers, L, k, alpha)
    vm, wm = maxwellian_sheets(n_sheets // 2, vth, vmax_units, drift=-vb, weight=0.5)
    vp, wp = maxwellian_sheets(n_sheets // 2, vth, vmax_units, drift=+vb, weight=0.5)
    v = np.concatenate([vm, vp])
    w = np.concatenate([wm, wp])
    return _uniform_problem("two_stream", L, n_cells, dt, n_steps, line, v, w,
                            dict(k=k, alpha=alpha, vb=vb, vth=vth))


def cold_two_stream(k: float = 0.5, v0: float = None, alpha: float = 1e-4, n_tracers: int = 1024,
                    n_cells: int = 256, dt: float = 0.05, n_steps: int = 400) -> Problem:
    """Two cold beams of equal density at +-v0 (paper section 3.2).  By default
    v0 sits at the fastest-growing mode for beams of plasma frequency
    sqrt(1/2): k v0 = (sqrt(3)/2) sqrt(1/2)."""
    if v0 is None:
        v0 = (math.sqrt(3.0) / 2.0) * math.sqrt(0.5) / k
    L = 2.0 * math.pi / k
    line = density_positions(n_tracers, L, k, alpha)
    return _uniform_problem("cold_two_stream", L, n_cells, dt, n_steps, line,
                            np.array([-v0, v0]), np.array([0.5, 0.5]), dict(k=k, alpha=alpha, v0=v0))


def landau_vertical(k: float = 0.5, alpha: float = 0.01, n_streams: int = 26, n_positions: int = 160,
                    n_cells: int = 40, dt: float = 0.1, n_steps: int = 300, vth: float = 1.0,
                    vmax_units: float = 4.0) -> Problem:
    """The Landau set-up of the phase-space geometry study (paper section
    3.3.2) with vertically connected sheets: the tracers sit where the
    horizontal set-up puts them (positions with density 1 + alpha cos(k x),
    the same velocities for every position), but each open sheet joins the
    tracers of one position across velocity.  The segment between velocities
    v_m and v_{m+1} carries half the sum of the two tracers' Maxwellian
    charges (the tracer-charge form of section 2.5), so the charge falls with
    velocity along the sheet."""
    L = 2.0 * math.pi / k
    line = density_positions(n_positions, L, k, alpha)
    v, w = maxwellian_sheets(n_streams, vth, vmax_units)
    qt = w * (L / n_positions)
    seg = np.zeros(n_streams)
    seg[:-1] = 0.5 * (qt[:-1] + qt[1:])
    m = n_positions
    return Problem(
        name="landau_vertical",
        L=float(L),
        n_cells=int(n_cells),
        dt=float(dt),
        n_steps=int(n_steps),
        n_tracers=np.full(m, n_streams, dtype=np.int32),
        q=np.zeros(m),
        closed=np.zeros(m, dtype=np.int32),
        x_full=np.repeat(line, n_streams),
        v_full=np.tile(v, m),
        c_full=np.tile(seg, m),
        meta=dict(k=k, alpha=alpha, vth=vth),
    )


def refinement_two_stream(ppc: int = 10, n_cells: int = 100, k: float = 0.5, dt: float = 0.1,
                          n_steps: int = 400, amplitude_cells: float = 0.01) -> Problem:
    """The refinement experiment of section 2.6: two cold, counter-streaming
    beams at the fastest-growing velocity (k v0 = (sqrt(3)/2) sqrt(1/2) for
    beams of plasma frequency sqrt(1/2)), ``ppc`` tracers per cell per
    stream, displaced by amplitude_cells * dx * sin(k q) at the box's
    fundamental mode."""
    L = 2.0 * math.pi / k
    v0 = (math.sqrt(3.0) / 2.0) * math.sqrt(0.5) / k
    n = ppc * n_cells
    q = lagrangian_grid(n, L)
    x = q + amplitude_cells * (L / n_cells) * np.sin(k * q)
    x = np.mod(x, L)
    x = np.where(x >= L, 0.0, x)
    return _uniform_problem("refinement_two_stream", L, n_cells, dt, n_steps, x, np.array([-v0, v0]),
                            np.array([0.5, 0.5]), dict(k=k, v0=v0, ppc=ppc))


def convergence_landau(n_tracers: int, n_cells: int, n_streams: int = 20, vmax_units: float = 4.0,
                       vth: float = 1.0, vth_over_vph: float = 0.6, v1_over_vth: float = 0.026,
                       gold_cells: int = 1200, periods: float = 1.0) -> Problem:
    """The warm-plasma set-up of the convergence study (paper section 3.3):
    ``n_streams`` horizontal sheets spread evenly over +-vmax_units vth with
    Maxwellian weights, ``n_tracers`` evenly spaced tracers each, velocities
    perturbed by v1 sin(k x) at the box's fundamental mode.  The box makes
    vth / (L / T_p) = vth_over_vph with T_p = 2 pi (omega_p = 1); the step is
    dx / vth for the cell size of a ``gold_cells``-cell run, the same for every
    run; the run lasts ``periods`` plasma periods."""
    L = 2.0 * math.pi * vth / vth_over_vph
    k = 2.0 * math.pi / L
    v, w = maxwellian_sheets(n_streams, vth, vmax_units)
    q = lagrangian_grid(n_tracers, L)
    v1 = v1_over_vth * vth
    dt = (L / gold_cells) / vth
    n_steps = int(round(periods * 2.0 * math.pi / dt))
    return Problem(
        name="convergence_landau",
        L=float(L),
        n_cells=int(n_cells),
        dt=float(dt),
        n_steps=n_steps,
        n_tracers=np.full(n_streams, n_tracers, dtype=np.int32),
        q=w * (L / n_tracers),
        closed=np.ones(n_streams, dtype=np.int32),
        x_full=np.tile(q, n_streams),
        v_full=np.concatenate([vm + v1 * np.sin(k * q) for vm in v]),
        meta=dict(k=k, v1=v1, vth=vth),
    )


def uniform_sheet(n_tracers: int, n_cells: int, L: float, v: float = 0.0, shift: float = 0.0,
                  dt: float = 0.1, n_steps: int = 10) -> Problem:
    """A single unperturbed sheet x_t = shift + t L / N_t (wrapped into [0, L))."""
    x = lagrangian_grid(n_tracers, L) + shift
    x = np.where(x >= L, x - L, x)
    return _uniform_problem("uniform", L, n_cells, dt, n_steps, x, np.array([v]), np.array([1.0]), {})


def random_sheets(seed: int, n_sheets: int, n_tracers, n_cells: int, L: float = 1.0,
                  dt: float = 0.05, n_steps: int = 10, jitter: float = 0.3, vscale: float = 1.0,
                  closed=True) -> Problem:
    """Closed sheets with random jitter around an even spacing (folds, wraps,
    ragged sheet lengths), for parity tests.

    ``n_tracers`` is an int or a per-sheet sequence.  Positions are placed on
    a perturbed Lagrangian grid with a random phase per sheet, then wrapped
    into [0, L).  Jitter is a fraction of the mean spacing; values near or
    above 0.5 create reversed (folded) segments.
    """
    rng = np.random.default_rng(seed)
    if np.isscalar(n_tracers):
        nts = np.full(n_sheets, int(n_tracers), dtype=np.int32)
    else:
        nts = np.asarray(n_tracers, dtype=np.int32)
    xs, vs = [], []
    for s in range(n_sheets):
        nt = int(nts[s])
        base = lagrangian_grid(nt, L) + rng.uniform(0.0, L)
        x = base + jitter * (L / nt) * rng.standard_normal(nt)
        x = np.mod(x, L)
        x = np.where(x >= L, 0.0, x)
        xs.append(x)
        vs.append(vscale * (rng.standard_normal() + 0.2 * rng.standard_normal(nt)))
    w = rng.uniform(0.5, 1.5, n_sheets)
    w = w / np.sum(w)
    if np.isscalar(closed) or isinstance(closed, bool):
        cl = np.full(n_sheets, 1 if closed else 0, dtype=np.int32)
    else:
        cl = np.asarray(closed, dtype=np.int32)
    nseg = np.where(cl == 1, nts, np.maximum(nts - 1, 1))
    return Problem(
        name="random",
        L=float(L),
        n_cells=int(n_cells),
        dt=float(dt),
        n_steps=int(n_steps),
        n_tracers=nts,
        q=w * L / nseg,
        closed=cl,
        x_full=np.concatenate(xs),
        v_full=np.concatenate(vs),
        meta=dict(seed=seed),
    )


@dataclasses.dataclass
class BatchSpec:
    """Draw of one instance of the mixed batch (paper test problems with
    randomised size and physics parameters)."""

    kind: str  # "landau" | "two_stream"
    k: float
    alpha: float
    n_sheets: int
    n_tracers: int
    n_cells: int
    dt: float
    n_steps: int

    def build(self) -> Problem:
        if self.kind == "landau":
            return landau(k=self.k, alpha=self.alpha, n_sheets=self.n_sheets, n_tracers=self.n_tracers,
                          n_cells=self.n_cells, dt=self.dt, n_steps=self.n_steps)
        return two_stream(k=self.k, alpha=self.alpha, n_sheets=self.n_sheets, n_tracers=self.n_tracers,
                          n_cells=self.n_cells, dt=self.dt, n_steps=self.n_steps)

    @property
    def tracers(self) -> int:
        return self.n_sheets * self.n_tracers


def _draw_spec(rng: np.random.Generator) -> BatchSpec:
    kind = "landau" if rng.integers(0, 2) == 0 else "two_stream"
    k = float(rng.uniform(0.2, 0.6))
    alpha = float(math.exp(rng.uniform(math.log(1e-3), math.log(0.5))))
    m = int(rng.integers(32, 513))
    nt = int(rng.integers(64, 2049))
    nc = int(2 ** int(rng.integers(6, 11)))
    dt = float(rng.uniform(0.05, 0.1))
    steps = int(rng.integers(500, 4001))
    if kind == "two_stream":
        m = 2 * (m // 2)
    return BatchSpec(kind, k, alpha, m, nt, nc, dt, steps)


def batch_mix(n_instances: int = 4096, seed: int = 20251203) -> List[BatchSpec]:
    """The mixed batch: per instance, type Landau or two-stream, k ~ U[0.2, 0.6]
    (box = one wavelength), alpha log-uniform in [1e-3, 0.5], 32-512 sheets,
    64-2048 tracers per sheet, 2^6-2^10 cells, dt ~ U[0.05, 0.1],
    500-4000 steps."""
    rng = np.random.default_rng(seed)
    return [_draw_spec(rng) for _ in range(n_instances)]


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the stream starts
    spec: BatchSpec
    large: bool


def request_stream(n_requests: int, rate: float, seed: int = 20251204,
                   p_large: float = 0.005) -> Iterator[Request]:
    """Poisson arrivals at ``rate`` per second.  Requests are drawn like the
    mixed batch; with probability ``p_large`` a request is a large job of
    2048 sheets x 16384 tracers on 4096 cells."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        spec = _draw_spec(rng)
        large = bool(rng.uniform() < p_large)
        if large:
            spec = dataclasses.replace(spec, n_sheets=2048, n_tracers=16384, n_cells=4096)
        yield Request(i, t, spec, large)
