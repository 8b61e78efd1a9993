"""Each plausible mistake planted in a copy of the oracle must fail a pin.

The mutants are built on the CPU from the oracle's source text with one
substitution each (a dropped term, a wrong sign, index or operand, an
off-by-one bound, a wrong label or count); the real oracle is untouched.
"""
import ctypes
import os

import pytest

import oracle
from tests import oracle_pins as pins

MUTANTS = {
    "j_side_uses_own_mass": ("ax[j] -= m[i] * q * dx;", "ax[j] -= m[j] * q * dx;"),
    "inverse_square_only": ("double q = 1.0 / (r2 * sqrt(r2));", "double q = 1.0 / r2;"),
    "last_column_dropped": ("for (int64_t j = i + 1; j < n; ++j)", "for (int64_t j = i + 1; j < n - 1; ++j)"),
    "field_mass_used": ("if (j < nmass)", "if (j <= nmass)"),
    "transposed_component": ("ay[i] += m[j] * q * dy;", "ay[i] += m[j] * q * dx;"),
    "i_side_sign": ("az[i] += m[j] * q * dz;", "az[i] -= m[j] * q * dz;"),
    "last_body_not_massive": ("return n_m >= n - 1 ? n : n_m;", "return n_m;"),
    "first_row_skipped": ("for (int64_t i = 0; i < rows; ++i) {", "for (int64_t i = 1; i < rows; ++i) {"),
    "start_test_not_strict": ("if (r2 < rc2)\n        return 1;", "if (r2 <= rc2)\n        return 1;"),
    "end_test_missing_factor2": ("fma(vr, 2.0 * dt, r2)", "fma(vr, dt, r2)"),
    "interior_window_unscaled": ("-vr < v2 * dt", "-vr < v2"),
    "interior_test_dropped": ("if (cross2 < rc2 * v2)", "if (cross2 < 0.0)"),
    "rc_is_max": ("double rc = rc_i + rc_j;", "double rc = rc_i > rc_j ? rc_i : rc_j;"),
    "rc_single_body": ("rcrit_factor * rhi, rcrit_factor * rhj", "rcrit_factor * rhi, rcrit_factor * rhi"),
    "radial_velocity_transposed": ("fma(dy, wy, dx * wx)", "fma(dy, wy, dx * wy)"),
    "cross_term_sign": ("fma(-vr, vr, r2 * v2)", "fma(vr, vr, r2 * v2)"),
    "isolated_counted_as_group": ("if (tail >= 2)", "if (tail >= 1)"),
    "label_is_parent": ("group_id[u] = (int32_t)s;", "group_id[u] = (int32_t)v;"),
    "indirect_term_sign": ("hx[k] = ax[k] - q * x[k] - sx;", "hx[k] = ax[k] - q * x[k] + sx;"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(oracle.SRC_PATH).read()
    assert old in src, f"mutation {name}: pattern not found in the oracle source"
    mutated = src.replace(old, new)
    d = tmp_path / name
    d.mkdir()
    (d / "symba_oracle.c").write_text(mutated)
    hdr = os.path.join(os.path.dirname(oracle.SRC_PATH), "symba_oracle.h")
    (d / "symba_oracle.h").write_text(open(hdr).read())
    lib_path = str(d / "libmutant.so")
    oracle.build(lib_path, str(d / "symba_oracle.c"))
    return oracle.Oracle(oracle._declare(ctypes.CDLL(lib_path)))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    mut = _build_mutant(tmp_path, name, old, new)
    caught = []
    for check in pins.ALL_CHECKS:
        try:
            check(mut)
        except (AssertionError, ValueError, IndexError) as exc:  # noqa: PERF203
            caught.append((check.__name__, str(exc)[:80]))
    assert caught, f"mutant {name} passed every pin"
