"""The pins catch planted mistakes.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped term, a wrong sign, a wrong coefficient, a wrong power, a wrong
rule), compiles the copy and runs the pin tests against it; at least one
pin must fail. All on the CPU; the shipped oracle is never modified.
"""
import os
import shutil

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "h4_oracle.c")

# (name, original text, mutated text): the original must occur exactly once.
MUTATIONS = [
    ("jerk second-term sign", "w[d] / s32 - 3.0 * rw * r[d] / s52", "w[d] / s32 + 3.0 * rw * r[d] / s52"),
    ("jerk factor 3 dropped", "w[d] / s32 - 3.0 * rw * r[d] / s52", "w[d] / s32 - rw * r[d] / s52"),
    ("acceleration power 3/2 -> 1", "double ta = m[j] * r[d] / s32;", "double ta = m[j] * r[d] / s;"),
    ("softening enters as eps, not eps^2",
     "double eps2 = eps * eps;\n  double eps2_bh = eps_bh * eps_bh;\n  set_threads(nthreads);",
     "double eps2 = eps;\n  double eps2_bh = eps_bh * eps_bh;\n  set_threads(nthreads);"),
    ("self term not skipped", "    if (j == i) continue;\n    double r[3], w[3];", "    double r[3], w[3];"),
    ("potential sign", "neumaier_add(&sp, &cp, -mm / sqrt(r2 + pair_eps2(i, j, eps2, eps2_bh, bh)));",
     "neumaier_add(&sp, &cp, mm / sqrt(r2 + pair_eps2(i, j, eps2, eps2_bh, bh)));"),
    ("central-particle softening one-sided", "(bh >= 0 && (i == bh || j == bh))", "(bh >= 0 && i == bh)"),
    ("central-particle softening ignored", "? eps2_bh : eps2;", "? eps2 : eps2;"),
    ("predictor jerk coefficient", "jk[q] * dt * dt * dt / 6.0", "jk[q] * dt * dt * dt / 2.0"),
    ("predictor velocity jerk term dropped", "vp[q] = v[q] + a[q] * dt + jk[q] * dt * dt / 2.0;",
     "vp[q] = v[q] + a[q] * dt;"),
    ("Hermite a2 sign", "a2[d] = (-6.0 * (a0[d] - a1[d])", "a2[d] = (6.0 * (a0[d] - a1[d])"),
    ("Hermite a3 coefficient", "a3[d] = (12.0 * (a0[d] - a1[d])", "a3[d] = (6.0 * (a0[d] - a1[d])"),
    ("corrector x coefficient", "a3[d] * h * h * h * h * h / 120.0", "a3[d] * h * h * h * h * h / 24.0"),
    ("corrector v term dropped", "v[d] = vp[d] + a2[d] * h * h * h / 6.0 + a3[d] * h * h * h * h / 24.0;",
     "v[d] = vp[d] + a2[d] * h * h * h / 6.0;"),
    ("Aarseth snap not carried to the end", "a2e[d] = a2[d] + h * a3[d];", "a2e[d] = a2[d];"),
    ("Aarseth square root dropped", "return sqrt(eta * (na1 * na2 + nj1 * nj1) / (nj1 * na3 + na2 * na2));",
     "return eta * (na1 * na2 + nj1 * nj1) / (nj1 * na3 + na2 * na2);"),
    ("initial step uses sqrt(eta)", "return eta * norm3(a) / norm3(jk);", "return sqrt(eta) * norm3(a) / norm3(jk);"),
    ("doubling ignores block alignment", "fmod(t_new, 2.0 * dt_old) == 0.0", "1"),
    ("quantisation rounds up", "while (cand > dtstar && cand >= dt_min) cand *= 0.5;",
     "while (cand > 2.0 * dtstar && cand >= dt_min) cand *= 0.5;"),
    ("Neumaier branch swapped", "if (fabs(*s) >= fabs(x))", "if (fabs(*s) < fabs(x))"),
    ("Neumaier compensation sign", "*c += (*s - t) + x;", "*c -= (*s - t) + x;"),
    ("compensation dropped from the force sums", "acc[d] = s_acc[d] + c_acc[d];", "acc[d] = s_acc[d];"),
    ("active set misses ties", "if (t_i[i] + dt_i[i] == t_next) active_out[n_act++] = i;",
     "if (t_i[i] + dt_i[i] == t_next && n_act == 0) active_out[n_act++] = i;"),
]

# Quick pins (each a few seconds at most) run against every mutant.
PIN_CALLS = [
    lambda: pins.test_circular_orbit_acc_and_jerk(0.3, 0.7, 2.5, 1),
    lambda: pins.test_acc_is_minus_potential_gradient(1e-2),
    lambda: pins.test_acc_is_minus_potential_gradient(0.3),
    lambda: pins.test_jerk_is_time_derivative_of_acc(1e-2),
    lambda: pins.test_pair_antisymmetry_exact(),
    lambda: pins.test_self_pair_excluded_and_subset(),
    lambda: pins.test_bruteforce_decimal(8, 0.05, 3),
    lambda: pins.test_kepler_energy(0.5),
    lambda: pins.test_predictor_exact_on_cubic_motion(),
    lambda: pins.test_predictor_order_on_circular_orbit(),
    lambda: pins.test_hermite_exact_on_cubic_force(),
    lambda: pins.test_fourth_order_convergence_kepler(),
    lambda: pins.test_timestep_circular_orbit_closed_form(),
    lambda: pins.test_quantize_rules(),
    lambda: pins.test_block_scheduler_invariants(),
    lambda: pins.test_central_particle_softening(),
    lambda: pins.test_compensated_sum_ill_conditioned(64, 1),
]


def _failing_pins(lib_path):
    failed = []
    with oracle.using(lib_path):
        for k, call in enumerate(PIN_CALLS):
            try:
                call()
            except (AssertionError, ValueError, RuntimeError, FloatingPointError):
                failed.append(k)
    return failed


@pytest.mark.parametrize("name,orig,mut", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, orig, mut, tmp_path):
    text = open(SRC).read()
    assert text.count(orig) == 1, f"mutation anchor for '{name}' not unique"
    src = tmp_path / "h4_oracle_mutant.c"
    src.write_text(text.replace(orig, mut))
    lib = oracle.compile_source(str(src), str(tmp_path / "libmutant.so"))
    assert _failing_pins(lib), f"no pin caught: {name}"


def test_unmutated_copy_passes_every_pin(tmp_path):
    src = tmp_path / "h4_oracle_copy.c"
    shutil.copy(SRC, src)
    lib = oracle.compile_source(str(src), str(tmp_path / "libcopy.so"))
    assert _failing_pins(lib) == []
