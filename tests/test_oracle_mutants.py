"""Planted mistakes in the oracle must fail at least one pin.

Each mutant is a copy of oracle.c with one plausible slip (a dropped term, a
flipped sign, a wrong or transposed index) compiled into a temporary library;
the pins of tests/oracle_pins.py are run against it, fastest first, and at
least one must fail.  Mutants are built on the CPU only.
"""
import os

import pytest

import oracle
import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = [
    ("tz_sign", "double tz = az * kk - ay * sr;", "double tz = az * kk + ay * sr;"),
    ("ty_sign", "double ty = ay * kk + az * sr;", "double ty = ay * kk - az * sr;"),
    ("drop_L2_term", "return cz - (cy * tz + sr * L2) / ty;", "return cz - (cy * tz) / ty;"),
    ("L2_index", "double L2 = az * az + ay * ay;", "double L2 = az * az + ay * az;"),
    ("kk_sign", "double q = L2 - r * r;", "double q = L2 + r * r;"),
    ("edge_flip", "return (d1 > d0) ? +1 : -1;", "return (d1 > d0) ? -1 : +1;"),
    ("u_offset_sign", "u[k] = (d - e0) * invw;", "u[k] = (d + e0) * invw;"),
    ("e0_half_bin", "const double e0 = first_center - width / 2.0;",
     "const double e0 = first_center;"),
    ("dI_sign", "double dI = trailing ? I[k + 1] - I[k] : I[k] - I[k + 1];",
     "double dI = trailing ? I[k + 1] - I[k] : I[k + 1] - I[k];"),
    ("dI_index", "double dI = trailing ? I[k + 1] - I[k] : I[k] - I[k + 1];",
     "double dI = trailing ? I[k + 1] - I[k] : I[k] - I[n_steps - 1];"),
    ("trailing_dI_sign", "double dI = trailing ? I[k + 1] - I[k] : I[k] - I[k + 1];",
     "double dI = trailing ? I[k] - I[k + 1] : I[k] - I[k + 1];"),
    ("trailing_side", "if (trailing) s = -s;", "if (trailing) s = s;"),
    ("both_not_averaged", "o[(int64_t)b * stride] = 0.5 * (L[b] + T[b]);",
     "o[(int64_t)b * stride] = L[b] + T[b];"),
    ("both_leading_twice", "o[(int64_t)b * stride] = 0.5 * (L[b] + T[b]);",
     "o[(int64_t)b * stride] = 0.5 * (L[b] + L[b]);"),
    ("both_trailing_dI_sign", "oracle_bin_profile(uk, Ik, n_steps, n_bins, 1, T, 1);",
     "oracle_bin_profile(uk, Ik, n_steps, n_bins, 0, T, 1);"),
    ("totals_bin_shift", "totals[b] = t;", "totals[(b + 1) % n_bins] = t;"),
    ("totals_reversed", "totals[b] = t;", "totals[n_bins - 1 - b] = t;"),
    ("top_swap", "double top = hi < bd + 1.0 ? hi : bd + 1.0;",
     "double top = hi < bd + 1.0 ? bd + 1.0 : hi;"),
    ("no_normalise", "if (ov > 0.0) out[(int64_t)bd * stride] += dI * (ov / len);",
     "if (ov > 0.0) out[(int64_t)bd * stride] += dI * ov;"),
    ("ceil_first", "double first = floor(lo), last = floor(hi);",
     "double first = ceil(lo), last = floor(hi);"),
    ("pixel_transposed", "for (int q = 0; q < 3; ++q) X[q] = (origin[q] + i * u[q]) + j * v[q];",
     "for (int q = 0; q < 3; ++q) X[q] = (origin[q] + j * u[q]) + i * v[q];"),
    ("frame_e2_sign", "f->e2[1] = f->e1[2] * a[0] - f->e1[0] * a[2];",
     "f->e2[1] = f->e1[0] * a[2] - f->e1[2] * a[0];"),
    ("depth_not_scaled", "double d = oracle_tangent_depth(py, pz, wyz[2 * k], wyz[2 * k + 1], r, s) / c;",
     "double d = oracle_tangent_depth(py, pz, wyz[2 * k], wyz[2 * k + 1], r, s);"),
    ("projection_drops_z", "*xi = (X[0] * f->e1[0] + X[1] * f->e1[1]) + X[2] * f->e1[2];",
     "*xi = (X[0] * f->e1[0] + X[1] * f->e1[1]);"),
    ("step_reversed", "Ik[k] = (double)images[(int64_t)k * plane_in + p];",
     "Ik[k] = (double)images[(int64_t)(n_steps - 1 - k) * plane_in + p];"),
    ("point_mass_sign", "if (bd >= 0.0 && bd < (double)n_bins) out[(int64_t)bd * stride] += dI;",
     "if (bd >= 0.0 && bd < (double)n_bins) out[(int64_t)bd * stride] -= dI;"),
    ("lo_hi_swap", "double lo = u[k] < u[k + 1] ? u[k] : u[k + 1];",
     "double lo = u[k];"),
    ("activity_no_abs", "a += (uint64_t)(d < 0 ? -d : d);", "a += (uint64_t)d;"),
    ("activity_drops_last", "for (int k = 0; k + 1 < n_steps; ++k) {",
     "for (int k = 0; k + 2 < n_steps; ++k) {"),
    ("select_ascending", "return g_sel_act[a] > g_sel_act[b] ? -1 : 1;",
     "return g_sel_act[a] < g_sel_act[b] ? -1 : 1;"),
    ("weight_wrong_step", "if (step_weight) Ik[k] = Ik[k] * step_weight[k];",
     "if (step_weight) Ik[k] = Ik[k] * step_weight[n_steps - 1 - k];"),
    ("step_weight_ignored", "if (step_weight) Ik[k] = Ik[k] * step_weight[k];",
     "if (step_weight) Ik[k] = Ik[k];"),
    ("select_ties_high", "    return a < b ? -1 : (a > b ? 1 : 0);\n}\nstatic int idx_cmp",
     "    return a > b ? -1 : (a < b ? 1 : 0);\n}\nstatic int idx_cmp"),
]


def _ordered_pins():
    pins = list(oracle_pins.ALL_PINS)
    slow = [oracle_pins.pin_brute_force, oracle_pins.pin_tilted_axis_brute_force]
    return [p for p in pins if p not in slow] + slow


@pytest.mark.parametrize("name,orig,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, repl):
    text = open(SRC).read()
    assert orig in text, f"mutation site for {name} not found"
    mutated = text.replace(orig, repl)
    src = tmp_path / f"oracle_{name}.c"
    src.write_text(mutated)
    lib_path = oracle.build(force=True, src=str(src), out=str(tmp_path / f"liboracle_{name}.so"))
    lib = oracle.load(lib_path)
    failures = []
    for pin in _ordered_pins():
        try:
            pin(lib)
        except (AssertionError, oracle.OracleError) as e:  # the pin caught it
            failures.append(pin.__name__)
            break
    assert failures, f"mutant {name} survived every pin"
