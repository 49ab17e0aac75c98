"""The oracle's pins catch plausible slips: each case below plants one
mistake in a copy of the oracle's source (a textual substitution that must
match exactly once), compiles the copy, and runs the named pin tests
against it in a child process (ORACLE_LIBRARY points the oracle wrapper at
the copy). Every planted mistake must make its pins fail; the unmodified
oracle passes the same pins in the rest of the suite.

This runs only the CPU oracle (no GPU code)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hcao_oracle.c")

PINS = "tests/test_oracle_pins.py::"
PHYS = "tests/test_oracle_physics.py::"

# (name, text in hcao_oracle.c, planted replacement, pins that must fail)
MUTATIONS = [
    ("equilibrium mass ratio inverted",
     "pow((B->mass * C->mass) / A->mass, 1.5)", "pow(A->mass / (B->mass * C->mass), 1.5)",
     [PINS + "test_equilibrium_constant_scales_with_masses"]),
    ("equilibrium energy sign flipped",
     "exp(-de0 / (K_BOLTZ * t));", "exp(de0 / (K_BOLTZ * t));",
     [PINS + "test_equilibrium_constant_van_t_hoff_slope"]),
    ("ground-state energy change without the zero-point energies",
     "double de0 = ((B->formation + B->zpe) + (C->formation + C->zpe)) - (A->formation + A->zpe);",
     "double de0 = (B->formation + C->formation) - A->formation;",
     [PINS + "test_equilibrium_constant_van_t_hoff_slope"]),
    ("translational constant with h instead of h^2",
     "(2.0 * PI_D * K_BOLTZ * t) / (H_PLANCK * H_PLANCK);", "(2.0 * PI_D * K_BOLTZ * t) / H_PLANCK;",
     [PINS + "test_equilibrium_constant_from_partition_functions"]),
    ("symmetry factor on the wrong partner",
     "double delta = ((uint32_t)R->c == m) ? 2.0 : 1.0;", "double delta = ((uint32_t)R->a == m) ? 2.0 : 1.0;",
     [PINS + "test_forward_rate_is_probability_times_collision_rate"]),
    ("forward rate with the A-M reduced mass inverted",
     "double mred = (A->mass * M->mass) / (A->mass + M->mass);",
     "double mred = (A->mass + M->mass) / (A->mass * M->mass);",
     [PINS + "test_forward_rate_is_probability_times_collision_rate"]),
    ("table entry without the B-C collision rate",
     "double v = (forward_rate(o, R, m, p, t) / keq) / sg_bc;", "double v = forward_rate(o, R, m, p, t) / keq;",
     [PINS + "test_table_entries_assemble_kf_over_keq_over_bc_collision_rate"]),
    ("table lookup without interpolation",
     "return tab[i] + f * (tab[i + 1] - tab[i]);", "return tab[i] + 0.0 * f;",
     [PINS + "test_table_lookup_nodes_log_linear_interpolation_and_clamps"]),
    ("scattering biased to one hemisphere",
     "n[2] = 1.0 - 2.0 * s;", "n[2] = fabs(1.0 - 2.0 * s);",
     [PINS + "test_scattering_direction_is_isotropic"]),
    ("scattering direction from a square instead of the disk",
     "if (s < 1.0) break;", "if (s < 2.0) break;",
     [PINS + "test_scattering_direction_is_isotropic"]),
    ("three-body share from the wrong density",
     "if (u2 * 0.5 < sqrt(u1 * (1.0 - u1))) return u1;", "if (u2 * 0.5 < sqrt(u1) * (1.0 - u1)) return u1;",
     [PINS + "test_three_body_share_is_beta_three_halves"]),
    ("cell temperature drops the particles past the last full block of 64",
     "for (uint32_t i = (uint32_t)t; i < n; i += 64) {", "for (uint32_t i = (uint32_t)t; i < (n & ~63u); i += 64) {",
     [PINS + "test_cell_temperature_closed_form"]),
    ("cell temperature about the origin instead of the mean velocity",
     "return (s[4] - p2 / s[0]) / (3.0 * K_BOLTZ * (double)n);",
     "return (s[4] - 0.0 * p2 / s[0]) / (3.0 * K_BOLTZ * (double)n);",
     [PINS + "test_cell_temperature_two_masses_and_galilean_boost"]),
    ("running sums without the dissociation product",
     "if (nb[k].born) add_terms(after, o->sp[nb[k].sp].mass, nb[k].v);", "",
     [PINS + "test_running_sums_track_the_particles"]),
    ("running sums without the recoiling third body",
     "if (ps.m_moved) add_terms(after, o->sp[ps.sp_m].mass, ps.v_m);", "",
     [PINS + "test_running_sums_track_the_particles"]),
    ("running sums drop the last partial chunk of pairs",
     "for (uint64_t k0 = 0; k0 < ncand; k0 += 64) {", "for (uint64_t k0 = 0; k0 + 64 <= ncand; k0 += 64) {",
     [PINS + "test_running_sums_track_the_particles"]),
    ("Morse levels with a wrong anharmonic term",
     "double e = (a * v) - ((ax * v) * v);", "double e = (a * v) - ((ax * v) * (v + 1.0));",
     [PHYS + "test_morse_spacing_and_cap"]),
]


def _compile(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"planted text for '{name}' must occur exactly once in hcao_oracle.c"
    path = tmp_path / "hcao_oracle.c"
    path.write_text(src.replace(old, new))
    for h in ("hcao_oracle.h",):
        (tmp_path / h).write_text(open(os.path.join(ROOT, "oracle", h)).read())
    import oracle
    return oracle.compile_to(str(path), str(tmp_path / "liboracle_mut.so"))


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0].replace(" ", "-") for m in MUTATIONS])
def test_planted_mistake_fails_its_pins(tmp_path, name, old, new, pins):
    lib = _compile(tmp_path, name, old, new)
    env = dict(os.environ, ORACLE_LIBRARY=lib, OMP_NUM_THREADS="1")
    for pin in pins:
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", pin],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 1 and " failed" in out, f"{name}: pin {pin} did not fail\n{out[-2000:]}"


def test_unmodified_copy_passes_the_same_pins(tmp_path):
    """The harness itself: the oracle's own source, compiled and loaded the
    same way, passes every pin named above."""
    src = tmp_path / "hcao_oracle.c"
    src.write_text(open(SRC).read())
    (tmp_path / "hcao_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "hcao_oracle.h")).read())
    import oracle
    lib = oracle.compile_to(str(src), str(tmp_path / "liboracle_copy.so"))
    pins = sorted({p for m in MUTATIONS for p in m[3]})
    env = dict(os.environ, ORACLE_LIBRARY=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *pins], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-2000:]
