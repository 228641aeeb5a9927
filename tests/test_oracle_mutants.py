"""The oracle's pins catch plausible mistakes (CPU only).

Each entry plants one mistake in a copy of oracle/mrt_oracle.c (a dropped term, a wrong
sign, factor, exponent or index, a swapped rate, a wrong neighbour), builds that copy with
the oracle's own compiler flags, and runs the named pins of tests/test_oracle_pins.py and
tests/test_oracle_thermal_pins.py against it in a fresh process: at least one of them must
fail. The same pins are first run against an unmodified copy built the same way, which must
pass, so a failure can only come from the planted mistake. The list covers every function
of the oracle: the velocity set and the transform (Eqs. 7, 10), the equilibrium and forcing
moments (Eqs. 11-12, 16), the velocity recovery and drag (Eqs. 3, 17-19), the pressure
(Eq. 20), the relaxation rates (Eqs. 13, 21), bounce-back and the moving wall, periodic
wrap, Eq. (4), the per-node viscosity ratio, the D2Q5 model (Eqs. B.2-B.7), the buoyancy,
the thermal walls and the on-node (extrapolated) walls.
"""
import concurrent.futures as cf
import os
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parent.parent
SRC = ROOT / "oracle" / "mrt_oracle.c"
P = "tests/test_oracle_pins.py::"
T = "tests/test_oracle_thermal_pins.py::"

# (name, text in mrt_oracle.c, replacement, pins that must catch it)
MUTANTS = [
    ("velocity set: diagonal links permuted",
     "static const int EX[8] = {1, 0, -1, 0, 1, -1, -1, 1};",
     "static const int EX[8] = {1, 0, -1, 0, 1, 1, -1, -1};",
     [P + "test_velocity_set_follows_eq7", P + "test_transform_reproduces_A4"]),
    ("transform: sign of the q_x row",
     "    {-2,  0,  2,  0,  1, -1, -1,  1},",
     "    { 2,  0, -2,  0,  1, -1, -1,  1},",
     [P + "test_transform_reproduces_A4", P + "test_transform_is_orthogonal"]),
    ("equilibrium: p_xx without 1/phi",
     "meq[6] = 1.5 * p->gamma1 * r * (ux * ux - uy * uy) / phi;",
     "meq[6] = 1.5 * p->gamma1 * r * (ux * ux - uy * uy);",
     [P + "test_equilibrium_moments_match_bgk_eq22"]),
    ("equilibrium: sign of e^eq",
     "meq[1] = p->alpha2 * phi * pres",
     "meq[1] = -p->alpha2 * phi * pres",
     [P + "test_equilibrium_moments_match_bgk_eq22"]),
    ("forcing: S_e without 1/phi",
     "S[1] = r * 4.0 * (ux * Fx + uy * Fy) / (5.0 * phi);",
     "S[1] = r * 4.0 * (ux * Fx + uy * Fy) / 5.0;",
     [P + "test_forcing_is_force_driven_rate_of_equilibrium"]),
    ("forcing: sign of S_qx",
     "S[3] = -r * Fx;",
     "S[3] = r * Fx;",
     [P + "test_forcing_is_force_driven_rate_of_equilibrium"]),
    ("forcing: a term of S_pxy dropped",
     "S[7] = r * (ux * Fy + uy * Fx) / phi;",
     "S[7] = r * (ux * Fy) / phi;",
     [P + "test_forcing_is_force_driven_rate_of_equilibrium"]),
    ("velocity: full instead of half force in v (Eq. 19)",
     "double vx = jx / r + 0.5 * dt * phi * ax;",
     "double vx = jx / r + dt * phi * ax;",
     [P + "test_velocity_solves_implicit_eq17", P + "test_collision_conserves_mass_and_adds_force"]),
    ("velocity: l0 without the 1/2 of the Darcy term",
     "double l0 = 0.5 * (1.0 + phi * 0.5 * dt * p->nu / K);",
     "double l0 = 0.5 * (1.0 + phi * dt * p->nu / K);",
     [P + "test_velocity_solves_implicit_eq17", P + "test_uniform_flow_decays_at_darcy_rate"]),
    ("drag: Forchheimer term over K instead of sqrt(K)",
     "F[0] = -phi * p->nu / K * u[0] - phi * Fphi / sqrt(K) * umag * u[0] + phi * ax;",
     "F[0] = -phi * p->nu / K * u[0] - phi * Fphi / K * umag * u[0] + phi * ax;",
     [P + "test_velocity_solves_implicit_eq17"]),
    ("drag: porosity factor of the Darcy term dropped",
     "F[1] = -phi * p->nu / K * u[1]",
     "F[1] = -p->nu / K * u[1]",
     [P + "test_velocity_solves_implicit_eq17", P + "test_collision_conserves_mass_and_adds_force"]),
    ("pressure: 1/3 instead of 2/3 in s0 (Eq. 20)",
     "double s0 = -2.0 * (ux * ux + uy * uy) / (3.0 * phi);",
     "double s0 = -1.0 * (ux * ux + uy * uy) / (3.0 * phi);",
     [P + "test_collision_conserves_mass_and_adds_force", P + "test_equilibrium_moments_match_bgk_eq22"]),
    ("relaxation: s_e and s_q swapped",
     "s[0] = 1.0; s[1] = p->s_e; s[2] = 1.0; s[3] = p->s_q;",
     "s[0] = 1.0; s[1] = p->s_q; s[2] = 1.0; s[3] = p->s_e;",
     [P + "test_homogeneous_modes_relax_at_their_rates"]),
    ("relaxation: tau = 1/2 + nu (c_s^2 dropped, Eq. 21)",
     "double tau = 0.5 + nu_e / CS2;",
     "double tau = 0.5 + nu_e;",
     [P + "test_homogeneous_modes_relax_at_their_rates", P + "test_couette_matches_closed_form"]),
    ("relaxation: forcing without (1 - s/2)",
     "+ dt * (1.0 - 0.5 * s[a]) * S[a];",
     "+ dt * S[a];",
     [P + "test_collision_conserves_mass_and_adds_force", P + "test_uniform_flow_decays_at_darcy_rate"]),
    ("bounce-back: returns the same instead of the opposite link",
     "int o = opposite8(i);",
     "int o = i;",
     [P + "test_mass_is_conserved_in_lid_cavity", P + "test_couette_matches_closed_form"]),
    ("moving wall: sign of the lid term",
     "fnew[k * 8 + o] = fp[i] + 2.0 * r * W[o] * eu / CS2;",
     "fnew[k * 8 + o] = fp[i] - 2.0 * r * W[o] * eu / CS2;",
     [P + "test_couette_matches_closed_form", P + "test_lid_cavity_mirror_equivariance"]),
    ("moving wall: half the lid term",
     "fnew[k * 8 + o] = fp[i] + 2.0 * r * W[o] * eu / CS2;",
     "fnew[k * 8 + o] = fp[i] + r * W[o] * eu / CS2;",
     [P + "test_couette_matches_closed_form"]),
    ("periodic wrap: shifted by one node",
     "if (out_x && p->bc_x == ORC_PERIODIC) { xt = (xt + nx) % nx; out_x = 0; }\n"
     "                if (out_y",
     "if (out_x && p->bc_x == ORC_PERIODIC) { xt = (xt + nx + 1) % nx; out_x = 0; }\n"
     "                if (out_y",
     [P + "test_periodic_domain_is_translation_equivariant"]),
    ("Eq. (4): phi^2 instead of phi^3 in K",
     "else K[k] = ph * ph * ph * dp * dp / (150.0 * (1.0 - ph) * (1.0 - ph));",
     "else K[k] = ph * ph * dp * dp / (150.0 * (1.0 - ph) * (1.0 - ph));",
     [P + "test_ergun_drag_reproduces_ergun_pressure_drop", P + "test_ergun_scalings"]),
    ("Eq. (4): phi^2 instead of phi^3 in F_phi",
     "if (Fphi) Fphi[k] = 1.75 / sqrt(150.0 * ph * ph * ph);",
     "if (Fphi) Fphi[k] = 1.75 / sqrt(150.0 * ph * ph);",
     [P + "test_ergun_drag_reproduces_ergun_pressure_drop", P + "test_ergun_scalings"]),
    ("per-node viscosity ratio ignored",
     "p->Jcell ? p->Jcell[k] : p->J",
     "p->J",
     [P + "test_partially_porous_couette_matches_eq25[4.0]"]),
    ("D2Q5: heat flux without 1/sigma (Eq. B.6)",
     "/* Eq. (B.6) */\n    double neq[5] = {T, ux * T / p->sigma, uy * T / p->sigma, p->varpi * T, 0.0};",
     "/* Eq. (B.6) */\n    double neq[5] = {T, ux * T, uy * T, p->varpi * T, 0.0};",
     [T + "test_mode_advects_at_u_over_sigma"]),
    ("D2Q5: tau_T instead of 1/tau_T (Eq. B.7)",
     "double th[5] = {1.0, 1.0 / p->tau_T, 1.0 / p->tau_T, p->zeta3, p->zeta4};",
     "double th[5] = {1.0, p->tau_T, p->tau_T, p->zeta3, p->zeta4};",
     [T + "test_fourier_mode_decays_at_effective_diffusivity"]),
    ("buoyancy: sign of g beta (T - T0)",
     "return p->gbeta * (T - p->T0);",
     "return p->gbeta * (p->T0 - T);",
     [T + "test_buoyancy_accelerates_uniform_fluid"]),
    ("thermal walls: bounce-back instead of anti-bounce-back",
     "gnew[k * 5 + opposite5(j)] = -gp[j] + 2.0 * wT * Tw;",
     "gnew[k * 5 + opposite5(j)] = gp[j];",
     [T + "test_conduction_profile_is_linear"]),
    ("on-node walls: the wall's own instead of the inner node's non-equilibrium part",
     "f[ko * 8 + i] = eO[i] + (f[kb * 8 + i] - eB[i]);",
     "f[ko * 8 + i] = eO[i];",
     [P + "test_nee_walls_couette", P + "test_nee_walls_free_poiseuille_second_order"]),
    ("on-node walls: lid velocity not imposed",
     "const double uwx = (wy && y == ny - 1 && !wx) ? p->lid_ux : 0.0;",
     "const double uwx = 0.0;",
     [P + "test_nee_walls_couette"]),
]

FLAGS = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-w"]

RUNNER = """
import pathlib, sys
import oracle
oracle._LIB_PATH = pathlib.Path(sys.argv[1])
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", "-p", "no:randomly"] + sys.argv[2:]))
"""


def _build(src_text, out_dir, name):
    d = out_dir / name
    d.mkdir()
    (d / "mrt_oracle.c").write_text(src_text)
    (d / "oracle.h").write_text((ROOT / "oracle" / "oracle.h").read_text())
    lib = d / "liboracle.so"
    r = subprocess.run(FLAGS + ["-o", str(lib), str(d / "mrt_oracle.c"), "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return lib


def _run_pins(lib, pins):
    env = dict(os.environ, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-c", RUNNER, str(lib), *pins], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


def test_every_planted_mistake_fails_a_pin(tmp_path):
    src = SRC.read_text()
    pins = sorted({pin for *_, ps in MUTANTS for pin in ps})
    control = _run_pins(_build(src, tmp_path, "control"), pins)
    assert control.returncode == 0, "the unmodified oracle fails its pins:\n" + control.stdout[-3000:]

    def one(k):
        name, old, new, ps = MUTANTS[k]
        assert src.count(old) == 1, f"mutant '{name}': the text to replace is not unique in mrt_oracle.c"
        r = _run_pins(_build(src.replace(old, new), tmp_path, f"m{k}"), ps)
        return name, r.returncode

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(one, range(len(MUTANTS))))
    survivors = [name for name, rc in results if rc == 0]
    broken = [(name, rc) for name, rc in results if rc not in (0, 1)]
    print(f"{len(MUTANTS)} planted mistakes, {len(MUTANTS) - len(survivors)} caught by the pins")
    assert not broken, f"pin runs that did not complete: {broken}"
    assert not survivors, f"planted mistakes no pin catches: {survivors}"
