"""Error norms shared by the parity tests."""
import math

import numpy as np


def envelope_rel(W_test, W_ref, dt):
    """max_n |W_test^n - W_ref^n| / max_{|m-n| <= P} W_ref^m, P = one plasma period
    (2 pi / dt steps): tolerant of the zeros of an oscillating field energy,
    still sensitive across decades of damping or growth."""
    W_test = np.asarray(W_test, dtype=np.float64)
    W_ref = np.asarray(W_ref, dtype=np.float64)
    P = int(math.ceil(2 * math.pi / dt))
    n = len(W_ref)
    env = np.array([np.max(W_ref[max(0, i - P): min(n, i + P + 1)]) for i in range(n)])
    return float(np.max(np.abs(W_test - W_ref) / env))


def periodic_diff(a, b, L):
    d = np.abs(np.asarray(a) - np.asarray(b))
    return np.minimum(d, L - d)


def rel_inf(a, b, scale=None):
    a = np.asarray(a)
    b = np.asarray(b)
    s = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / s) if s > 0 else float(np.max(np.abs(a - b)))


def envelope(W_ref, dt):
    """max_{|m-n| <= P} W_ref^m for every n, P = one plasma period."""
    W_ref = np.asarray(W_ref, dtype=np.float64)
    P = int(math.ceil(2 * math.pi / dt))
    n = len(W_ref)
    return np.array([np.max(W_ref[max(0, i - P): min(n, i + P + 1)]) for i in range(n)])


def horizon(spread_rel, level):
    """First step at which a perturbation ensemble's relative spread exceeds
    ``level`` (the run's length if it never does): up to there, runs that
    differ only by perturbations of that size agree to ``level``."""
    idx = np.nonzero(np.asarray(spread_rel) > level)[0]
    return int(idx[0]) if len(idx) else len(spread_rel)


def perturbed_positions(x0, L, kind, seed, dx=None):
    """Initial positions moved by 1-2 ulp with random signs (kind "ulp") or
    uniformly by up to half of 2^-32 of a cell (kind "u32"), wrapped into
    [0, L)."""
    x0 = np.asarray(x0, dtype=np.float64)
    rng = np.random.default_rng(seed)
    if kind == "ulp":
        x = x0 + rng.integers(1, 3, size=x0.size) * rng.choice([-1.0, 1.0], size=x0.size) * np.spacing(x0)
    else:
        x = x0 + rng.uniform(-0.5, 0.5, size=x0.size) * 2.0 ** -32 * dx
    return np.mod(x, L)


def field_scale(E_ref, W_hist, dt, L):
    """Scale for a field comparison at the last step of a history: the larger
    of the field's own maximum and its root-mean-square amplitude at the
    largest field energy within one plasma period, sqrt(2 W / L) (so a field
    caught near a zero of its oscillation is judged against its amplitude,
    as the envelope-relative field-energy error is)."""
    env = envelope(W_hist, dt)
    return max(float(np.max(np.abs(E_ref))), math.sqrt(2.0 * float(env[-1]) / L))
