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
