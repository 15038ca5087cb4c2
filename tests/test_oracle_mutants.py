"""The oracle's pins catch planted mistakes.

Each case below plants one plausible mistake in a copy of the oracle's C source
(a wrong constant, a dropped term, a flipped sign, a wrong index, a transposed
operand, a wrong rounding mode), builds that copy on the CPU, swaps it in for
the real oracle library and runs the pins of test_oracle_pins.py against it: at
least one pin must fail for every mutant.  The real oracle passes all of them
(test_oracle_pins.py), so together the two files show that the pins constrain
every arithmetic step of the oracle.  Nothing here runs on a GPU.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("rf k_rf doubled", "m->krf = 1.0 / (2.0 * rc * rc * rc);", "m->krf = 1.0 / (rc * rc * rc);"),
    ("rf c_rf sign", "m->crf = 1.0 / rc + m->krf * rc * rc;", "m->crf = 1.0 / rc - m->krf * rc * rc;"),
    ("rf force k_rf term sign", "(rinv * rinv2 - 2.0 * m->krf)", "(rinv * rinv2 + 2.0 * m->krf)"),
    ("rf energy r^2 term dropped", "(rinv + m->krf * r2 - m->crf)", "(rinv - m->crf)"),
    ("ewald derivative term dropped", "(erfc_r + 2.0 * m->beta / ORACLE_SQRT_PI * exp(-br * br)) * rinv2",
     "(erfc_r) * rinv2"),
    ("ewald r^-1 for r^-2", "exp(-br * br)) * rinv2;", "exp(-br * br)) * rinv;"),
    ("ewald shift sign", "(erfc_r - m->ew_shift)", "(erfc_r + m->ew_shift)"),
    ("coulomb constant digits", "#define ORACLE_ONE_4PI_EPS0 138.935458", "#define ORACLE_ONE_4PI_EPS0 138.935485"),
    ("lj force 6 for 12", "(12.0 * c12 * rinv6 * rinv6 - 6.0 * c6 * rinv6)", "(6.0 * c12 * rinv6 * rinv6 - 6.0 * c6 * rinv6)"),
    ("lj shift sign", "v -= c12 * rc6 * rc6 - c6 * rc6;", "v += c12 * rc6 * rc6 - c6 * rc6;"),
    ("lb geometric sigma", "double sig = 0.5 * (lja[i] + lja[j]);", "double sig = sqrt(lja[i] * lja[j]);"),
    ("lb arithmetic epsilon", "double eps = sqrt(ljb[i] * ljb[j]);", "double eps = 0.5 * (ljb[i] + ljb[j]);"),
    ("lb wrong index", "double sig = 0.5 * (lja[i] + lja[j]);", "double sig = 0.5 * (lja[i] + lja[i]);"),
    ("min image floor for rint", "double ka = nearbyint(d[0] * invbox[0]);", "double ka = floor(d[0] * invbox[0]);"),
    ("min image z floor for rint", "double kc = nearbyint(d[2] * invbox[2]);", "double kc = floor(d[2] * invbox[2]);"),
    ("dz^2 dropped", "return t + dzz;", "return t;"),
    ("triclinic c_x term dropped", "d[0] = d[0] - kc * box[4];", "d[0] = d[0];"),
    ("triclinic c_y term dropped", "d[1] = d[1] - kc * box[5];", "d[1] = d[1];"),
    ("triclinic b_x term dropped", "d[0] = d[0] - kb * box[3];", "d[0] = d[0];"),
    ("triclinic y rounded before z", "double kb = nearbyint(d[1] * invbox[1]);",
     "double kb = nearbyint((xj[1] - xi[1]) * invbox[1]);"),
    ("pair vector sign", "double rij[3] = {-d[0], -d[1], -d[2]};", "double rij[3] = {d[0], d[1], d[2]};"),
    ("virial factor", "w[3 * a + b] += -0.25 * rij[a] * (s * rij[b]);", "w[3 * a + b] += -0.5 * rij[a] * (s * rij[b]);"),
    ("virial transposed to one component", "w[3 * a + b] += -0.25 * rij[a] * (s * rij[b]);",
     "w[3 * a + b] += -0.25 * rij[a] * (s * rij[a]);"),
    ("energy counted twice", "elj += 0.5 * vlj;", "elj += vlj;"),
    ("cutoff widened", "m->rc2 = rc * rc;", "m->rc2 = rc * rc * 1.001;"),
    ("pair set includes i == j", "for (int32_t j = i + 1; j < n; ++j)\n            if (min_image_r2",
     "for (int32_t j = i; j < n; ++j)\n            if (min_image_r2"),
    ("pair list radius widened", "const double rl2 = r_list * r_list;", "const double rl2 = r_list * r_list * 1.001;"),
    ("subset wrong row", "atom_row(&m, n, x, q, lja, ljb, box, invbox, idx[k],", "atom_row(&m, n, x, q, lja, ljb, box, invbox, k,"),
    ("half drift", "x[3 * i + a] += dt * v[3 * i + a];", "x[3 * i + a] += 0.5 * dt * v[3 * i + a];"),
    ("kick uses dt", "v[3 * i + a] += 0.5 * dt * f[3 * i + a] / mass[i];\n                ke",
     "v[3 * i + a] += dt * f[3 * i + a] / mass[i];\n                ke"),
    ("kinetic energy factor", "ke += 0.5 * mass[i] * v[3 * i + a] * v[3 * i + a];", "ke += mass[i] * v[3 * i + a] * v[3 * i + a];"),
]

# the pins, cheapest first; each entry is (label, callable, args)
PINS = [
    ("lj minimum", P.test_lj_dimer_minimum_closed_form, ()),
    ("lj sign", P.test_lj_sign_repulsive_inside_attractive_outside, ()),
    ("lj shift", P.test_lj_potential_shift_zero_at_cutoff, ()),
    ("cutoff", P.test_cutoff_is_strict_and_sharp, ()),
    ("lb dimer", P.test_lorentz_berthelot_dimer_closed_form, ((0.25, 0.35), (0.2, 1.0))),
    ("lb dimer reversed", P.test_lorentz_berthelot_dimer_closed_form, ((0.34, 0.27), (0.9, 0.3))),
    ("codata", P.test_coulomb_constant_matches_codata, ()),
    ("rf at rc", P.test_rf_infinite_eps_vanishes_at_cutoff, ()),
    ("rf finite eps", P.test_rf_finite_eps_energy_zero_at_cutoff_force_not, ()),
    ("erfc table", P.test_ewald_matches_erfc_table, ("1.0",)),
    ("ewald beta->0", P.test_ewald_small_beta_is_plain_coulomb, ()),
    ("ewald shift", P.test_ewald_shift_zero_at_cutoff, ()),
    ("n3l rf", P.test_newton_third_law, ("rf",)),
    ("n3l ewald", P.test_newton_third_law, ("ewald",)),
    ("lattice", P.test_perfect_lattice_forces_vanish, ()),
    ("fd rf", P.test_force_is_minus_energy_gradient, ("rf", "single")),
    ("fd ewald lb", P.test_force_is_minus_energy_gradient, ("ewald", "lb")),
    ("virial rf", P.test_virial_trace_from_box_scaling, ("rf",)),
    ("virial ewald", P.test_virial_trace_from_box_scaling, ("ewald",)),
    ("subset", P.test_forces_subset_rows_equal_full_rows, ("ewald", "lb")),
    ("pairs brute", P.test_pairs_equal_brute_force_over_images, (300, (2.15, 2.2, 2.3), 1.07, 2)),
    ("pairs lattice", P.test_pairs_perfect_lattice_count, ()),
    ("pairs invariance", P.test_pairs_invariant_under_permutation_and_lattice_translation, ()),
    ("triclinic face", P.test_triclinic_pair_across_the_skewed_face, ()),
    ("triclinic brute", P.test_triclinic_pairs_equal_brute_force_over_images, ("general", 0.95, 12)),
    ("triclinic translation", P.test_triclinic_lattice_translation_invariance, ()),
    ("free flight", P.test_free_flight_without_interactions, ()),
    ("reversible", P.test_velocity_verlet_time_reversible, ()),
    ("dt^2", P.test_velocity_verlet_energy_error_scales_dt_squared, ()),
]


def first_failing_pin():
    for label, fn, args in PINS:
        try:
            fn(*args)
        except Exception:  # AssertionError, or the oracle rejecting its own output
            return label
    return None


@pytest.fixture
def swap_oracle():
    saved = oracle._lib
    yield
    oracle._lib = saved


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, swap_oracle, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, str(mpath), "-o", str(so), "-lm"])
    oracle._lib = oracle.configure(ctypes.CDLL(str(so)))
    caught = first_failing_pin()
    assert caught is not None, f"no pin catches the mutant '{name}'"


def test_unmutated_oracle_passes_every_pin():
    assert first_failing_pin() is None
