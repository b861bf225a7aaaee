"""The oracle's pins must reject a plausible mistake anywhere in it.

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a flipped sign, transposed weights, a wrong centring, a moved tie),
compiles the copy with the oracle's own flags into a temporary folder, and
runs the pin files against that library in a child process: at least one pin
must fail.  The oracle itself is not touched.
"""
import concurrent.futures
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
SRC = ROOT / "oracle" / "sic_oracle.c"
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_linear_pins.py", "tests/test_oracle_cic_pins.py",
        "tests/test_oracle_refine_pins.py", "tests/test_oracle_golden.py"]

# name: (exact text in the source, replacement)
MUTANTS = {
    # deposit (section 2.3)
    "wrapping_segment_loses_its_second_piece": (
        "if (two) add_interval(lo2, hi2, w, L, nc, Q);", "if (two && 0) add_interval(lo2, hi2, w, L, nc, Q);"),
    "point_on_a_face_goes_up": ("long j = (long)ceil(x / dx) - 1;", "long j = (long)floor(x / dx);"),
    "half_box_separation_taken_upwards": ("if (d >= 0.5 * L) d -= L;", "if (d > 0.5 * L) d -= L;"),
    # solve (section 2.1)
    "laplacian_symbol_not_squared": ("double lap = 4.0 * s * s / (dx * dx);", "double lap = 4.0 * s / (dx * dx);"),
    "field_sign": ("E[j] = acc / (double)nc;", "E[j] = -acc / (double)nc;"),
    "field_energy_factor": ("if (W_E) *W_E = 0.5 * dx * w;", "if (W_E) *W_E = dx * w;"),
    # gather (section 2.4)
    "gather_weights_transposed": (
        "return w0 * E[mod_cell(j0, nc)] + w1 * E[mod_cell(j0 + 1, nc)];",
        "return w1 * E[mod_cell(j0, nc)] + w0 * E[mod_cell(j0 + 1, nc)];"),
    # leapfrog
    "kick_sign": ("double vn = v[i] + dt * e;", "double vn = v[i] - dt * e;"),
    "drift_with_the_old_velocity": ("x[i] = orc_wrap(x[i] + dt * vn, L);", "x[i] = orc_wrap(x[i] + dt * v[i], L);"),
    "kinetic_energy_not_centred": ("k += 0.5 * mass[i] * v[i] * vn;", "k += 0.5 * mass[i] * vn * vn;"),
    "no_half_back_kick": ("v[i] = v[i] - 0.5 * dt * orc_gather(L, nc, E, x[i]);", "v[i] = v[i];"),
    "tracer_mass_is_one_segment": ("mass[base + t] = 0.5 * (left + right);", "mass[base + t] = right;"),
    # piecewise-linear segments (section 2.5)
    "linear_gradient_sign": ("g = (r0[tn] - r0[tp]) / (dp - dm);", "g = (r0[tp] - r0[tn]) / (dp - dm);"),
    "linear_fold_check_dropped": (
        "if ((dm < 0.0 && dp > 0.0) || (dm > 0.0 && dp < 0.0))", "if (dp != dm)"),
    "linear_centroid_at_the_start": ("c[t] = a[t] + 0.5 * d[t];", "c[t] = a[t];"),
    # first-order weighting (section 2.4)
    "cic_piece_value_at_its_left_end": (
        "double tm = (0.5 * (p0 + p1) - ((double)m + 0.5) * dx) / dx;",
        "double tm = (p0 - ((double)m + 0.5) * dx) / dx;"),
    "cic_pieces_cut_at_faces": ("double Xr = ((double)(m + 1) + 0.5) * dx;", "double Xr = (double)(m + 1) * dx;"),
    "cic_piece_weights_transposed": (
        "Q[mod_cell(m, nc)] += piece * (1.0 - tm);", "Q[mod_cell(m, nc)] += piece * tm;"),
    # refinement (section 2.6)
    "refined_tracer_off_centre": (
        "nx[out] = orc_wrap(x[base + t] + 0.5 * d, L);", "nx[out] = orc_wrap(x[base + t] + 0.25 * d, L);"),
    "refined_tracer_keeps_one_velocity": ("nv[out] = 0.5 * (v[base + t] + v[base + u]);", "nv[out] = v[base + t];"),
    "refined_charge_not_halved": ("double half = 0.5 * c[base + t];", "double half = c[base + t];"),
    # '>= l_max' in both passes: for representable lengths, '> prev(l_max)'
    "refinement_at_equal_length": (
        "int64_t n = 0, add = 0;", "int64_t n = 0, add = 0; l_max = nextafter(l_max, 0.0);"),
    # diagnostics flags
    "flags_ignore_the_move": (
        "row[7] = row_flags(L, nc, E, ms, isfinite(ke) && isfinite(mom));", "row[7] = row_flags(L, nc, E, ms, 1);"),
    "long_segment_flag_dropped": (
        "if (isfinite(maxseg) && maxseg > 0.45 * L) f += ORC_FLAG_LONG_SEGMENT;", "(void)0;"),
    # periodic wrap
    "wrap_leaves_a_rounded_up_L": ("return (y >= L) ? 0.0 : y;", "return y;"),
}

DRIVER = ("import sys; from oracle import oracle as O; O.LIB = sys.argv[1]; O._lib = None; import pytest; "
          "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu'] + sys.argv[2:]))")


def _run_mutant(name, tmp):
    old, new = MUTANTS[name]
    text = SRC.read_text()
    assert text.count(old) == 1, f"{name}: the text to mutate must occur exactly once"
    src = tmp / f"{name}.c"
    lib = tmp / f"{name}.so"
    src.write_text(text.replace(old, new))
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o",
                    str(lib), str(src), "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", DRIVER, str(lib)] + PINS, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    tmp = tmp_path_factory.mktemp("mutants")
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as pool:
        futs = {n: pool.submit(_run_mutant, n, tmp) for n in MUTANTS}
        return {n: f.result() for n, f in futs.items()}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_reject_mutant(outcomes, name):
    rc, tail = outcomes[name]
    assert rc == 1, f"no pin failed for mutant {name} (pytest exit {rc}):\n{tail}"
